// Judge of a predicted field against a reference field: interface position
// and L2 error, per grid of a batch.
//
// Interface: the zero level set, sampled as the points where phi changes sign
// along an edge between two adjacent cell centres, located by linear
// interpolation.  The interface error is the Hausdorff distance between the
// two point sets (physical units, cell size h).  Each crossing searches the
// other field's crossings on the edges of the cells within `window` cells of
// its own; with no partner there the distance is reported as +inf.  Any
// partner outside the window is at least (window - 1) h away, so the value is
// exact whenever it is <= (window - 1) h -- enough for a decision at h.
// If neither field has a crossing the distance is 0; if only one has, inf.
//
// L2: root mean square of (a - b) over the grid.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "ac_internal.h"

// Scratch of the allocation-free judge (ac_judge_2d_noalloc): the same three
// words per grid as the caller's workspace of ac_judge_2d (distance bits,
// squared-error sum, crossing flags), for at most kJudgeNoallocMaxBatch grids:
// 192 KiB held on every device the library runs on until the process ends.
// Host code never passes `scratch` itself to a kernel (on the host it is only
// a stand-in for the symbol); it takes the device address that
// hipGetSymbolAddress reports for the current device.
constexpr int kJudgeNoallocMaxBatch = 16384;
static __device__ __align__(256) unsigned scratch[3 * kJudgeNoallocMaxBatch];

namespace ac {

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
ac_status scratch_ptr(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(AC_ERR_UNSUPPORTED, "device %d beyond the %d devices the static scratch serves", dev,
                    kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(AC_ERR_HIP, "hipGetSymbolAddress(scratch) returned null");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return AC_OK;
}

// A workgroup judges a kJTX x kJTY tile of one grid.  Both fields are staged
// in LDS over the tile and the cells within the search window around it, the
// tile's crossings are collected into a list, and the list is then shared
// out over all lanes: the nearest-partner searches (the bulk of the work)
// read LDS, and no lane idles for want of a crossing of its own.
constexpr int kJTX = 64, kJTY = 16, kJThreads = 256;
constexpr int kJMaxList = 4 * kJTX * kJTY;   // two edges per cell in each field

// The staged region of a tile at (x0, y0) for window w: columns x0-w ..
// x0+kJTX+w and rows y0-w .. y0+kJTY+w (a cell's crossing edges reach one
// cell further than the window).
__host__ __device__ constexpr int judge_region_x(int w) { return kJTX + 2 * w + 1; }
__host__ __device__ constexpr int judge_region_y(int w) { return kJTY + 2 * w + 1; }

size_t judge_lds_bytes(int w) {
    return (2 * (size_t)judge_region_x(w) * judge_region_y(w) + kJMaxList + 1) * 4;
}

// A staged field: values of the region whose first cell is (rx0, ry0), row pitch RX.
struct Staged {
    const float *v;
    int RX, rx0, ry0;
    __device__ float at(int i, int j) const { return v[(j - ry0) * RX + (i - rx0)]; }
};

// Crossing on the edge from cell (i, j) to (i + di, j + dj); returns false if
// the sign does not change.  Coordinates in cell units (cell (i, j) centre at
// (i, j)).
__device__ inline bool crossing(const Staged &f, int nx, int ny, int i, int j, int di, int dj,
                                float *px, float *py) {
    const int i2 = i + di, j2 = j + dj;
    if (i2 >= nx || j2 >= ny) return false;
    const float a = f.at(i, j), b = f.at(i2, j2);
    if ((a > 0.f) == (b > 0.f)) return false;
    const float t = a / (a - b);
    *px = i + di * t;
    *py = j + dj * t;
    return true;
}

// min distance from (px, py) to the crossings of g in the window around cell (i, j)
__device__ inline float nearest(const Staged &g, int nx, int ny, int i, int j, int w, float px,
                                float py) {
    float best = INFINITY;
    for (int jj = max(j - w, 0); jj <= min(j + w, ny - 1); ++jj)
        for (int ii = max(i - w, 0); ii <= min(i + w, nx - 1); ++ii)
            for (int e = 0; e < 2; ++e) {
                float qx, qy;
                if (crossing(g, nx, ny, ii, jj, e == 0, e == 1, &qx, &qy)) {
                    const float d = sqrtf((qx - px) * (qx - px) + (qy - py) * (qy - py));
                    best = fminf(best, d);
                }
            }
    return best;
}

// grid (tiles_x * tiles_y, batch), kJThreads threads, judge_lds_bytes(w) of LDS
__global__ void __launch_bounds__(kJThreads)
judge_kernel(const float *__restrict__ a, const float *__restrict__ b, int nx, int ny, int w,
             int tiles_x, unsigned *dist_bits, float *sq, int *count)
{
    extern __shared__ float jlds[];
    const int n = blockIdx.y;
    const size_t cells = (size_t)nx * ny;
    const float *fa = a + n * cells, *fb = b + n * cells;
    const int x0 = (int)(blockIdx.x % tiles_x) * kJTX, y0 = (int)(blockIdx.x / tiles_x) * kJTY;
    const int RX = judge_region_x(w), RY = judge_region_y(w), rx0 = x0 - w, ry0 = y0 - w;
    float *la = jlds, *lb = jlds + RX * RY;
    int *list = reinterpret_cast<int *>(lb + RX * RY);
    int *nlist = list + kJMaxList;
    const int t = threadIdx.x;
    if (t == 0) *nlist = 0;
    // cells outside the grid are staged as 0 and never read: every search
    // and edge is clamped to the grid first
    for (int k = t; k < RX * RY; k += kJThreads) {
        const int gx = rx0 + k % RX, gy = ry0 + k / RX;
        const bool in = gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        const size_t o = in ? (size_t)gy * nx + gx : 0;
        la[k] = in ? fa[o] : 0.f;
        lb[k] = in ? fb[o] : 0.f;
    }
    __syncthreads();
    const Staged sa{la, RX, rx0, ry0}, sb{lb, RX, rx0, ry0};
    float local = 0.f, ssq = 0.f;
    int cnt = 0;
    // the tile's own cells: squared differences and the list of crossings
    // (cell, edge, field)
    for (int c = t; c < kJTX * kJTY; c += kJThreads) {
        const int i = x0 + c % kJTX, j = y0 + c / kJTX;
        if (i >= nx || j >= ny) continue;
        const float d = sa.at(i, j) - sb.at(i, j);
        ssq += d * d;
        for (int e = 0; e < 2; ++e) {
            float px, py;
            if (crossing(sa, nx, ny, i, j, e == 0, e == 1, &px, &py)) {
                list[atomicAdd(nlist, 1)] = c | e << 16;
                cnt |= 1;
            }
            if (crossing(sb, nx, ny, i, j, e == 0, e == 1, &px, &py)) {
                list[atomicAdd(nlist, 1)] = c | e << 16 | 1 << 17;
                cnt |= 2;
            }
        }
    }
    __syncthreads();
    const int nl = *nlist;
    for (int k = t; k < nl; k += kJThreads) {
        // a crossing of one field searches the other field's crossings
        const int v = list[k], c = v & 0xffff, e = (v >> 16) & 1, in_b = v >> 17;
        const int i = x0 + c % kJTX, j = y0 + c / kJTX;
        float px = 0.f, py = 0.f;
        crossing(in_b ? sb : sa, nx, ny, i, j, e == 0, e == 1, &px, &py);
        local = fmaxf(local, nearest(in_b ? sa : sb, nx, ny, i, j, w, px, py));
    }
    for (int o = 32; o > 0; o >>= 1) {
        ssq += __shfl_xor(ssq, o);
        local = fmaxf(local, __shfl_xor(local, o));
        cnt |= __shfl_xor(cnt, o);
    }
    if ((t & 63) == 0) {
        // non-negative floats order like their bit patterns (+inf is the largest)
        if (local > 0.f) atomicMax(dist_bits + n, __float_as_uint(local));
        if (cnt) atomicOr(count + n, cnt);
        atomicAdd(sq + n, ssq);
    }
}

__global__ void judge_finish_kernel(const unsigned *dist_bits, const float *sq, const int *count,
                                    int batch, size_t cells, float h, float *iface, float *l2)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= batch) return;
    float d = __uint_as_float(dist_bits[n]);
    if (count[n] == 0) d = 0.f;                                    // no interface in either
    else if (count[n] != 3) d = INFINITY;                          // an interface in one only
    iface[n] = d * h;
    l2[n] = sqrtf(sq[n] / (float)cells);
}

__global__ void judge_zero_kernel(unsigned *dist_bits, float *sq, int *count, int batch)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n < batch) { dist_bits[n] = 0u; sq[n] = 0.f; count[n] = 0; }
}

}  // namespace

}  // namespace ac

using namespace ac;

namespace {

ac_status judge_args(const float *a, const float *b, int32_t batch, int32_t nx, int32_t ny, double h,
                     int32_t window, const float *iface_err, const float *l2_err) {
    if (!a || !b || !iface_err || !l2_err) return fail(AC_ERR_INVALID_ARG, "null pointer argument");
    if (batch < 1 || nx < 1 || ny < 1 || window < 1 || window > 16 || !(h > 0) || !std::isfinite(h))
        return fail(AC_ERR_INVALID_ARG, "bad judge sizes (batch %d, %d x %d, window %d)", batch, nx, ny, window);
    if (batch > 65535) return fail(AC_ERR_UNSUPPORTED, "batch above 65535");
    return AC_OK;
}

// The three launches of a judgement; workspace holds 3 * batch words.
ac_status judge_launch(const float *a, const float *b, int32_t batch, int32_t nx, int32_t ny, double h,
                       int32_t window, float *iface_err, float *l2_err, void *workspace,
                       hipStream_t st) {
    unsigned *dist = static_cast<unsigned *>(workspace);
    float *sq = reinterpret_cast<float *>(dist + batch);
    int *cnt = reinterpret_cast<int *>(sq + batch);
    hipLaunchKernelGGL(judge_zero_kernel, dim3((batch + 255) / 256), dim3(256), 0, st, dist, sq, cnt, batch);
    const long long cells = (long long)nx * ny;
    const int tiles_x = (nx + kJTX - 1) / kJTX;
    const long long tiles = (long long)tiles_x * ((ny + kJTY - 1) / kJTY);
    if (tiles > INT_MAX) return fail(AC_ERR_UNSUPPORTED, "grid %d x %d has too many judge tiles", nx, ny);
    hipLaunchKernelGGL(judge_kernel, dim3((unsigned)tiles, batch), dim3(kJThreads), judge_lds_bytes(window),
                       st, a, b, nx, ny, (int)window, tiles_x, dist, sq, cnt);
    hipLaunchKernelGGL(judge_finish_kernel, dim3((batch + 255) / 256), dim3(256), 0, st, dist, sq, cnt,
                       batch, (size_t)cells, (float)h, iface_err, l2_err);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? AC_OK : hip_fail(e, "judge launch");
}

}  // namespace

extern "C" {

ac_status ac_judge_2d(const float *a, const float *b, int32_t batch, int32_t nx, int32_t ny,
                      double h, int32_t window, float *iface_err, float *l2_err, void *workspace,
                      void *stream)
{
    g_err.clear();
    ac_status s = judge_args(a, b, batch, nx, ny, h, window, iface_err, l2_err);
    if (s != AC_OK) return s;
    if (!workspace) return fail(AC_ERR_INVALID_ARG, "null workspace");
    return judge_launch(a, b, batch, nx, ny, h, window, iface_err, l2_err, workspace,
                        reinterpret_cast<hipStream_t>(stream));
}

ac_status ac_judge_2d_noalloc(const float *a, const float *b, int32_t batch, int32_t nx, int32_t ny,
                              double h, int32_t window, float *iface_err, float *l2_err, void *stream)
{
    g_err.clear();
    ac_status s = judge_args(a, b, batch, nx, ny, h, window, iface_err, l2_err);
    if (s != AC_OK) return s;
    if (batch > kJudgeNoallocMaxBatch)
        return fail(AC_ERR_INVALID_ARG, "batch %d exceeds the %d grids of the static judge scratch",
                    batch, kJudgeNoallocMaxBatch);
    void *ws = nullptr;
    s = scratch_ptr(&ws);
    if (s != AC_OK) return s;
    return judge_launch(a, b, batch, nx, ny, h, window, iface_err, l2_err, ws,
                        reinterpret_cast<hipStream_t>(stream));
}

int64_t ac_judge_workspace_bytes(int32_t batch) { return (int64_t)batch * 12; }

}  // extern "C"
