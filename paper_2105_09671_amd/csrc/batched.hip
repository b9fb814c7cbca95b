// Batched stepping: many independent 2D grids (own size, h, dt, eps) advanced
// by one persistent kernel, captured once in a hipGraph and replayed.
//
// Work decomposition.  Every instance is cut into the same tiles as the
// single-grid tiled kernels, with the tile body its plan chooses (reg2d.h for
// register tiles, tile2d.h for LDS tiles).  One "item" is one tile of one instance;
// the item list is the same for every temporal block ("phase") of tb_depth
// steps.  A grid of workgroups, sized to what the device holds at once, takes
// the items of phase b from ticket counters, meets at a phase barrier, and
// moves on to phase b+1 (instances ping-pong between phi and work, so the
// barrier is what makes the halo of phase b+1 see the finished phase b).
//
// XCD-aware schedule: the dispatcher places workgroup g on XCD g mod 8, and
// each XCD has its own L2.  The item list is split into 8 contiguous ranges,
// each with its own ticket counter, and XCD x's workgroups take tickets of
// range x only, so the tiles of one instance -- which re-read each other's
// halos -- share one L2.
//
// No workgroup waits for another one to start: tickets are monotonic across
// phases (ticket t of range x is item t mod n_x of phase t / n_x), a
// workgroup holding a ticket of a later phase keeps it until it gets there,
// and the barrier counts finished items, not arrived workgroups.  So the
// kernel completes whether or not every workgroup of the grid is resident at
// once.  Waits are bounded (poll count and wall clock): a workgroup that
// gives up raises the error flag and every workgroup leaves at its next
// barrier, so the kernel always drains; the host reports the flag through
// ac_check().  The counters are zeroed by a small kernel captured in front of
// the persistent kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <list>
#include <mutex>
#include <vector>

#include "reg2d.h"
#include "reg2w.h"
#include "reg3d.h"
#include "stream3d.h"
#include "tile2d.h"

namespace ac {

struct BatchInst {
    void *phi, *work;
    int nx, ny;
    double alpha, r;
    int nz, tiles_x;   // 3D batches: depth and xy tiles along x (LDS tiles)
    int rtiles_x;      // 3D batches: xy tiles along x of the register tiles
    int lx, ly;        // 3D batches: this instance's LDS tile
    int lz;            // 3D batches: this instance's z segment (LDS tiles)
};

// sync[0]: items finished (over all phases); sync[1 + x]: tickets taken from
// XCD x's item range.
constexpr int SYNC_WORDS = 9;

__global__ void batch_reset_kernel(unsigned *sync) {
    if (threadIdx.x < SYNC_WORDS) sync[threadIdx.x] = 0u;
}

// Masked batches: copy the items of active instances, in order, to `out` and
// their number to *count.  One workgroup of 1024 threads scans the list in
// chunks with an LDS prefix sum, so the order (and hence the XCD grouping of
// neighbouring tiles) is kept.
__global__ void __launch_bounds__(1024)
batch_compact_kernel(const int4 *__restrict__ items, int n_items, const int *__restrict__ active,
                     int4 *__restrict__ out, int *count)
{
    __shared__ int scan[1024];
    int base = 0;
    for (int c0 = 0; c0 < n_items; c0 += 1024) {
        const int i = c0 + threadIdx.x;
        int4 it{0, 0, 0, 0};
        int f = 0;
        if (i < n_items) {
            it = items[i];
            f = active[it.x] != 0;
        }
        scan[threadIdx.x] = f;
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {       // inclusive Hillis-Steele scan
            const int v = threadIdx.x >= (unsigned)d ? scan[threadIdx.x - d] : 0;
            __syncthreads();
            scan[threadIdx.x] += v;
            __syncthreads();
        }
        if (f) out[base + scan[threadIdx.x] - 1] = it;
        const int total = scan[1023];
        __syncthreads();
        base += total;
    }
    if (threadIdx.x == 0) *count = base;
}

// End of a phase for this workgroup: publish its `mine` finished items and wait
// until `target` items are finished in total.  Returns false once any
// workgroup has given up waiting (after spin_limit polls or wall_limit ticks
// of the constant-rate clock).  Release fence, relaxed add, relaxed polls,
// then one acquire fence: the counter's adds form one release sequence, so
// the fences order every workgroup's stores before every other's loads.  An
// acquire on each poll would invalidate the XCD's L2 at every poll, under the
// workgroups still computing there.
__device__ __forceinline__ bool phase_sync(unsigned *done, unsigned mine, unsigned target, int *err,
                                           long long spin_limit, long long wall_limit) {
    __shared__ int s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // publish this workgroup's stores
        if (mine) __hip_atomic_fetch_add(done, mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int ok = 1;
        long long spins = 0;
        const long long t0 = wall_clock64();
        while (__hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { ok = 0; break; }
            if (++spins > spin_limit || wall_clock64() - t0 > wall_limit) {
                atomicExch(err, 1);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(4);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // see every other workgroup's stores
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// Copy the output region of one tile from src to dst (final odd-count fix-up):
// the region of the register tiling (reg2d.h) when REG, else the uniform
// tiling of the LDS bodies.
template <typename T, bool REG>
__device__ void copy_tile(const T *src, T *dst, int nx, int ny, int LX, int LY, int K, int tx,
                          int ty) {
    int x0, x1, y0, y1;
    if constexpr (REG) {
        int ld;
        reg2d_tile_span(tx, reg2d_tiles_1d(nx, LX, K), nx, LX, K, &ld, &x0, &x1);
        reg2d_tile_span(ty, reg2d_tiles_1d(ny, LY, K), ny, LY, K, &ld, &y0, &y1);
    } else {
        x0 = tx * (LX - 2 * K);
        y0 = ty * (LY - 2 * K);
        x1 = min(x0 + LX - 2 * K, nx);
        y1 = min(y0 + LY - 2 * K, ny);
    }
    const int w = x1 - x0;
    for (int i = threadIdx.x; i < w * (y1 - y0); i += blockDim.x) {
        const int y = y0 + i / w, x = x0 + i % w;
        dst[(size_t)y * nx + x] = src[(size_t)y * nx + x];
    }
}

// One tile of one instance with the single-grid plan's tile body: BODY_REG
// (registers, 64-wide), BODY_INPLACE (one LDS buffer, 64-wide), BODY_LDS2
// (two LDS buffers, width LXC, or LX at run time when LXC = 0) or BODY_REGW
// (per item: wide = 1, the 128-wide register tile of reg2w.h, LY / 2 rows, for
// instances at least 128 wide; wide = 0, the 64-wide one).
enum { BODY_LDS2 = 0, BODY_INPLACE = 1, BODY_REG = 2, BODY_REGW = 3 };

template <typename T, int LXC, int BODY>
__device__ __forceinline__ void tile_item(const T *src, T *dst, const BatchInst &I, int LX, int LY,
                                          int K, int k, int tx, int ty, int wide, unsigned char *smem)
{
    if constexpr (BODY == BODY_REGW) {
        if (wide)
            reg2w_body<T, kRegWRows>(src, dst, I.nx, I.ny, (T)I.alpha, (T)I.r, K, k, tx, ty,
                                     reinterpret_cast<T *>(smem));
        else
            reg2d_body<T, kRegRows>(src, dst, I.nx, I.ny, (T)I.alpha, (T)I.r, K, k, tx, ty,
                                    reinterpret_cast<T *>(smem));
    } else if constexpr (BODY == BODY_REG)
        reg2d_body<T, kRegRows>(src, dst, I.nx, I.ny, (T)I.alpha, (T)I.r, K, k, tx, ty,
                                reinterpret_cast<T *>(smem));
    else if constexpr (BODY == BODY_INPLACE)
        tile2d_body<T, 64, Rows<T>::value, true, INPLACE_LB, INPLACE_D>(
            src, dst, I.nx, I.ny, (T)I.alpha, (T)I.r, 64, LY, K, k, tx, ty, smem);
    else
        tile2d_body<T, LXC>(src, dst, I.nx, I.ny, (T)I.alpha, (T)I.r, LX, LY, K, k, tx, ty, smem);
}

template <typename T, int LXC, int BODY>
__global__ void __launch_bounds__(1024)
batched_kernel(const BatchInst *__restrict__ inst, const int4 *__restrict__ items, int n_items,
               int LX, int LY, int K, int nblocks, int base, int rem, int copy_back,
               const int *__restrict__ n_active, unsigned *sync, int *err, long long spin_limit,
               long long wall_limit)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ unsigned s_ticket;
    if (n_active) n_items = *n_active;            // masked: `items` is the compacted list
    const int xcd = blockIdx.x & 7;
    const int lo = (int)((long long)n_items * xcd / 8);
    const unsigned cnt = (unsigned)((long long)n_items * (xcd + 1) / 8 - lo);
    unsigned *tickets = sync + 1 + xcd;
    const int phases = nblocks + (copy_back ? 1 : 0);   // copy_back: a last copy phase
    if (threadIdx.x == 0) s_ticket = atomicAdd(tickets, 1u);
    __syncthreads();
    unsigned t = s_ticket;
    for (int b = 0; b < phases; ++b) {
        const unsigned end = (unsigned)(b + 1) * cnt;
        const int k = base + (b < rem ? 1 : 0);
        unsigned mine = 0;
        while (t < end) {
            const int4 it = items[lo + (int)(t - (unsigned)b * cnt)];
            __syncthreads();                      // every lane has read s_ticket
            unsigned next = 0;
            if (threadIdx.x == 0) next = atomicAdd(tickets, 1u);   // in flight during the item
            const BatchInst I = inst[it.x];
            if (b < nblocks) {
                const T *src = static_cast<const T *>((b & 1) ? I.work : I.phi);
                T *dst = static_cast<T *>((b & 1) ? I.phi : I.work);
                tile_item<T, LXC, BODY>(src, dst, I, LX, LY, K, k, it.y, it.z, it.w, smem_raw);
            } else {   // odd number of single-step phases: the result sits in work
                const bool wide = BODY == BODY_REGW && it.w;
                copy_tile<T, BODY == BODY_REG || BODY == BODY_REGW>(
                    static_cast<const T *>(I.work), static_cast<T *>(I.phi), I.nx, I.ny,
                    wide ? 128 : LX, wide ? LY / 2 : LY, K, it.y, it.z);
            }
            if (threadIdx.x == 0) s_ticket = next;
            __syncthreads();                      // LDS is reused by the next item
            t = s_ticket;
            ++mine;
        }
        if (b + 1 < phases &&
            !phase_sync(sync, mine, (unsigned)(b + 1) * (unsigned)n_items, err, spin_limit, wall_limit))
            return;
    }
}

// Phase-graph mode: one launch per phase (captured as consecutive graph nodes),
// one workgroup per item, no waiting inside the kernel.  Workgroup g runs on
// XCD g mod 8 and takes item (g mod 8) * per + g / 8, so each XCD's workgroups
// cover one contiguous slice of the list (neighbouring tiles share an L2).
// The ordering between phases is the kernel boundary, whose cache release and
// acquire the command processor performs once per launch, where the
// persistent kernel's barrier has every workgroup do its own.
template <typename T, int LXC, int BODY>
__global__ void __launch_bounds__(1024)
batched_phase_kernel(const BatchInst *__restrict__ inst, const int4 *__restrict__ items,
                     int n_items, int LX, int LY, int K, int k, int phase, int copy,
                     const int *__restrict__ n_active)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    if (n_active) n_items = *n_active;
    const int per = (n_items + 7) / 8;
    const int i = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    if ((int)(blockIdx.x >> 3) >= per || i >= n_items) return;     // whole workgroup
    const int4 it = items[i];
    const BatchInst I = inst[it.x];
    if (!copy) {
        const T *src = static_cast<const T *>((phase & 1) ? I.work : I.phi);
        T *dst = static_cast<T *>((phase & 1) ? I.phi : I.work);
        tile_item<T, LXC, BODY>(src, dst, I, LX, LY, K, k, it.y, it.z, it.w, smem_raw);
    } else {
        const bool wide = BODY == BODY_REGW && it.w;
        copy_tile<T, BODY == BODY_REG || BODY == BODY_REGW>(
            static_cast<const T *>(I.work), static_cast<T *>(I.phi), I.nx, I.ny, wide ? 128 : LX,
            wide ? LY / 2 : LY, K, it.y, it.z);
    }
}

// Copy the output region of one 3D item (xy tile, z segment) from src to dst.
template <typename T>
__device__ void copy_tile3d(const T *src, T *dst, int nx, int ny, int nz, int OX, int OY, int LZ,
                            int tiles_x, int tile, int zseg) {
    const int x0 = (tile % tiles_x) * OX, y0 = (tile / tiles_x) * OY, z0 = zseg * LZ;
    const int w = min(x0 + OX, nx) - x0, hh = min(y0 + OY, ny) - y0, d = min(z0 + LZ, nz) - z0;
    const long long n = (long long)w * hh * d;
    for (long long i = threadIdx.x; i < n; i += blockDim.x) {
        const int x = x0 + (int)(i % w), y = y0 + (int)((i / w) % hh), z = z0 + (int)(i / ((long long)w * hh));
        const size_t c = ((size_t)z * ny + y) * nx + x;
        dst[c] = src[c];
    }
}

// Copy the output region of one register-tile 3D item (flush xy tiles of 64 x
// 32 cells, z segment of LZ planes) from src to dst.
template <typename T>
__device__ void copy_tile3d_reg(const T *src, T *dst, int nx, int ny, int nz, int K, int LZ,
                                int tiles_x, int tile, int zseg) {
    int lx0, ox0, ox1, ly0, oy0, oy1;
    reg2d_tile_span(tile % tiles_x, tiles_x, nx, 64, K, &lx0, &ox0, &ox1);
    reg2d_tile_span(tile / tiles_x, reg2d_tiles_1d(ny, 32, K), ny, 32, K, &ly0, &oy0, &oy1);
    const int z0 = zseg * LZ, w = ox1 - ox0, hh = oy1 - oy0, d = min(z0 + LZ, nz) - z0;
    const long long n = (long long)w * hh * d;
    for (long long i = threadIdx.x; i < n; i += blockDim.x) {
        const int x = ox0 + (int)(i % w), y = oy0 + (int)((i / w) % hh), z = z0 + (int)(i / ((long long)w * hh));
        const size_t c = ((size_t)z * ny + y) * nx + x;
        dst[c] = src[c];
    }
}

// One 3D item for one phase: it.w = 0 runs the LDS z-streaming body on an LX x
// LY tile and LZ-plane segment, it.w = 1 (FP32, 512 threads) the register
// body on a flush 64 x 32 tile and LZR-plane segment.  Both give the bits of
// ac_step_3d.  copy: the final copy phase of the item's output region.
template <typename T, int K, int CPT, bool REG>
__device__ __forceinline__ void batch3d_item(const BatchInst &I, int4 it, int phase, bool copy, int LX,
                                             int LY, int LZ, int LZR, unsigned char *smem_raw)
{
    if (!copy) {
        const T *src = static_cast<const T *>((phase & 1) ? I.work : I.phi);
        T *dst = static_cast<T *>((phase & 1) ? I.phi : I.work);
        if constexpr (REG && sizeof(T) == 4) {
            if (it.w) {
                reg3d_body<T, K, kReg3dRows, true>(src, dst, I.nx, I.ny, I.nz, (T)I.alpha, (T)I.r, LZR,
                                                   I.rtiles_x, it.y, it.z,
                                                   reinterpret_cast<T *>(smem_raw));
                return;
            }
        }
        stream3d_body<T, K, CPT>(src, dst, I.nx, I.ny, I.nz, (T)I.alpha, (T)I.r, I.lx, I.ly, I.lz,
                                 I.tiles_x, it.y, it.z, smem_raw);
    } else if (REG && it.w) {
        copy_tile3d_reg<T>(static_cast<const T *>(I.work), static_cast<T *>(I.phi), I.nx, I.ny, I.nz, K,
                           LZR, I.rtiles_x, it.y, it.z);
    } else {
        copy_tile3d<T>(static_cast<const T *>(I.work), static_cast<T *>(I.phi), I.nx, I.ny, I.nz,
                       I.lx - 2 * K, I.ly - 2 * K, I.lz, I.tiles_x, it.y, it.z);
    }
}

// 3D batch: items (instance, xy tile, z segment, body); every phase advances each
// item by K steps with a z-streaming body of ac_step_3d (batch3d_item).  Phases are
// numbered from phase0 for the phi/work ping-pong, so a second launch can run
// a shorter remainder phase.  Scheduling as in batched_kernel.
template <typename T, int K, int CPT, bool REG>
__global__ void __launch_bounds__(512)
batched3d_kernel(const BatchInst *__restrict__ inst, const int4 *__restrict__ items, int n_items,
                 int LX, int LY, int LZ, int LZR, int nphase, int phase0, int copy_back,
                 unsigned *sync, int *err, long long spin_limit, long long wall_limit)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ unsigned s_ticket;
    const int xcd = blockIdx.x & 7;
    const int lo = (int)((long long)n_items * xcd / 8);
    const unsigned cnt = (unsigned)((long long)n_items * (xcd + 1) / 8 - lo);
    unsigned *tickets = sync + 1 + xcd;
    const int phases = nphase + (copy_back ? 1 : 0);
    if (threadIdx.x == 0) s_ticket = atomicAdd(tickets, 1u);
    __syncthreads();
    unsigned t = s_ticket;
    for (int b = 0; b < phases; ++b) {
        const unsigned end = (unsigned)(b + 1) * cnt;
        unsigned mine = 0;
        while (t < end) {
            const int4 it = items[lo + (int)(t - (unsigned)b * cnt)];
            __syncthreads();                      // every lane has read s_ticket
            unsigned next = 0;
            if (threadIdx.x == 0) next = atomicAdd(tickets, 1u);
            const BatchInst I = inst[it.x];
            batch3d_item<T, K, CPT, REG>(I, it, phase0 + b, b >= nphase, LX, LY, LZ, LZR, smem_raw);
            if (threadIdx.x == 0) s_ticket = next;
            __syncthreads();
            t = s_ticket;
            ++mine;
        }
        if (b + 1 < phases &&
            !phase_sync(sync, mine, (unsigned)(b + 1) * (unsigned)n_items, err, spin_limit, wall_limit))
            return;
    }
}

// Phase-graph mode for 3D batches: one launch per phase, one workgroup per item
// (XCD-aware slices as in batched_phase_kernel).  copy: the final copy phase.
template <typename T, int K, int CPT, bool REG>
__global__ void __launch_bounds__(512)
batched3d_phase_kernel(const BatchInst *__restrict__ inst, const int4 *__restrict__ items,
                       int n_items, int LX, int LY, int LZ, int LZR, int phase, int copy)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int per = (n_items + 7) / 8;
    const int i = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    if ((int)(blockIdx.x >> 3) >= per || i >= n_items) return;     // whole workgroup
    const int4 it = items[i];
    const BatchInst I = inst[it.x];
    batch3d_item<T, K, CPT, REG>(I, it, phase, copy != 0, LX, LY, LZ, LZR, smem_raw);
}

// ---------------------------------------------------------------- host ----

namespace {

long long g_spin_limit = 20000000;   // ~2 s of polling per barrier
bool g_persistent = false;           // false: a graph of one launch per phase
constexpr int64_t kMaxGraphBlocks = 2048;   // temporal blocks per captured graph
constexpr int kRegBatchLZ = 32;             // z segment of a register-tile 3D batch item
constexpr int kBatch3dCellsPerThread = 2;   // largest per-instance LDS tile: this many cells per thread

struct Plan {
    // key
    int dim = 2;
    std::vector<ac_instance2d> inst;
    std::vector<ac_instance3d> inst3;
    int64_t nsteps;
    int32_t dtype;
    ac_tune tune;
    const int *active;
    int device;
    // device state
    BatchInst *d_inst = nullptr;
    int4 *d_items = nullptr;
    int4 *d_compact = nullptr;      // masked plans: active items of the current call
    int *d_count = nullptr;
    unsigned *d_bar = nullptr;
    int *d_err = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    int grid = 0, n_items = 0;
    ac_batch_info info{};
};

std::mutex g_mu;
std::list<Plan> g_plans;          // most recently used first
constexpr size_t kMaxPlans = 64;
hipStream_t g_capture_stream[64];

bool same_inst(const ac_instance2d &a, const ac_instance2d &b) {
    return a.phi == b.phi && a.work == b.work && a.nx == b.nx && a.ny == b.ny && a.h == b.h &&
           a.dt == b.dt && a.eps == b.eps;
}

bool key_equal(const Plan &p, const ac_instance2d *inst, int32_t n, int64_t nsteps,
               int32_t dtype, const ac_tune &t, const int *active, int dev) {
    if (p.dim != 2 || p.device != dev || p.nsteps != nsteps || p.dtype != dtype || (int32_t)p.inst.size() != n ||
        p.active != active)
        return false;
    if (std::memcmp(&p.tune, &t, sizeof t) != 0) return false;
    for (int32_t i = 0; i < n; ++i)
        if (!same_inst(p.inst[i], inst[i])) return false;
    return true;
}

void release(Plan &p) {
    if (p.exec) (void)hipGraphExecDestroy(p.exec);
    if (p.graph) (void)hipGraphDestroy(p.graph);
    if (p.d_inst) (void)hipFree(p.d_inst);
    if (p.d_items) (void)hipFree(p.d_items);
    if (p.d_compact) (void)hipFree(p.d_compact);
    if (p.d_count) (void)hipFree(p.d_count);
    if (p.d_bar) (void)hipFree(p.d_bar);
    if (p.d_err) (void)hipFree(p.d_err);
    p.exec = nullptr; p.graph = nullptr; p.d_inst = nullptr; p.d_items = nullptr;
    p.d_compact = nullptr; p.d_count = nullptr;
    p.d_bar = nullptr; p.d_err = nullptr;
}

template <typename T, int LXC, int BODY = BODY_LDS2>
const void *kernel_ptr() { return (const void *)batched_kernel<T, LXC, BODY>; }

template <typename T, int LXC, int BODY = BODY_LDS2>
const void *phase_kernel_ptr() { return (const void *)batched_phase_kernel<T, LXC, BODY>; }

// the tile body the single-grid plan chose (AC_KERNEL_2D_*)
int body_of(int plan_kernel) {
    return plan_kernel == AC_KERNEL_2D_REG       ? BODY_REG
           : plan_kernel == AC_KERNEL_2D_REGW    ? BODY_REGW
           : plan_kernel == AC_KERNEL_2D_INPLACE ? BODY_INPLACE
                                                 : BODY_LDS2;
}

template <typename T>
const void *phase_kernel_of(int LX, int body) {
    if (body == BODY_REG) return phase_kernel_ptr<T, 64, BODY_REG>();
    if (body == BODY_REGW) return phase_kernel_ptr<T, 64, BODY_REGW>();
    if (body == BODY_INPLACE) return phase_kernel_ptr<T, 64, BODY_INPLACE>();
    if (LX == 64) return phase_kernel_ptr<T, 64>();
    if (LX == 128) return phase_kernel_ptr<T, 128>();
    return phase_kernel_ptr<T, 0>();
}

template <typename T>
const void *kernel_of(int LX, int body) {
    if (body == BODY_REG) return kernel_ptr<T, 64, BODY_REG>();
    if (body == BODY_REGW) return kernel_ptr<T, 64, BODY_REGW>();
    if (body == BODY_INPLACE) return kernel_ptr<T, 64, BODY_INPLACE>();
    if (LX == 64) return kernel_ptr<T, 64>();
    if (LX == 128) return kernel_ptr<T, 128>();
    return kernel_ptr<T, 0>();
}

const void *select_phase_kernel(int32_t dtype, int LX, int plan_kernel) {
    return dtype == AC_F64 ? phase_kernel_of<double>(LX, body_of(plan_kernel))
                           : phase_kernel_of<float>(LX, body_of(plan_kernel));
}

const void *select_kernel(int32_t dtype, int LX, int plan_kernel) {
    return dtype == AC_F64 ? kernel_of<double>(LX, body_of(plan_kernel))
                           : kernel_of<float>(LX, body_of(plan_kernel));
}

// Validate every instance (no HIP call) and check no two buffers overlap.
ac_status validate_batch(const ac_instance2d *inst, int32_t n, int64_t nsteps, int32_t dtype,
                         std::vector<double> *alpha, std::vector<double> *r) {
    if (n < 0 || (n > 0 && !inst)) return fail(AC_ERR_INVALID_ARG, "bad instance array");
    alpha->resize(n);
    r->resize(n);
    std::vector<std::pair<uintptr_t, uintptr_t>> ranges;
    ranges.reserve(2 * (size_t)n);
    for (int32_t i = 0; i < n; ++i) {
        const ac_instance2d &I = inst[i];
        if (I.nx < 1 || I.ny < 1)
            return fail(AC_ERR_INVALID_ARG, "instance %d: nx, ny must be >= 1", i);
        ac_status s = validate(I.phi, I.work, (int64_t)I.nx * I.ny, 2, I.h, I.dt, I.eps, nsteps,
                               dtype, &(*alpha)[i], &(*r)[i]);
        if (s != AC_OK) {
            std::string m = g_err;
            return fail(s, "instance %d: %s", i, m.c_str());
        }
        const size_t bytes = (size_t)I.nx * I.ny * elem_size(dtype);
        ranges.push_back({(uintptr_t)I.phi, (uintptr_t)I.phi + bytes});
        ranges.push_back({(uintptr_t)I.work, (uintptr_t)I.work + bytes});
    }
    std::sort(ranges.begin(), ranges.end());
    for (size_t i = 1; i < ranges.size(); ++i)
        if (ranges[i].first < ranges[i - 1].second)
            return fail(AC_ERR_INVALID_ARG, "instance buffers overlap");
    return AC_OK;
}

ac_status build_plan(Plan &p, const ac_instance2d *inst, int32_t n, int64_t nsteps, int32_t dtype,
                     const ac_tune &tune, const std::vector<double> &alpha,
                     const std::vector<double> &r, const DevInfo &dev) {
    const size_t elem = elem_size(dtype);
    // launch shape: the single-grid tiled plan for the same tune (forced tiled).
    // kernel AC_KERNEL_2D_REGW: register tiles 128 wide (and half as tall, the
    // same waves) for instances at least 128 wide, 64 wide for the others; the
    // plan is made for the 64-wide tile
    ac_tune t = tune;
    if (!t.tb_depth && !t.tile_x && !t.tile_y && !t.kernel) {
        // default: depth 8, 128-wide register tiles for the instances at least
        // 128 wide, 64-wide ones of twice the height for the others; FP32 128
        // x 96 (12 waves), FP64 128 x 64 (8 waves).  Measured on the 512-grid
        // batch: FP32 2797-2813 GLUPS against 2686-2700 with 64 x 128 tiles
        // for every instance (128 x 64: 2673-2684, 128 x 128: 2013); FP64 1682
        // against 1571-1575 (128 x 96: 1216)
        t.kernel = AC_KERNEL_2D_REGW;
        t.tb_depth = 8;
        t.tile_y = dtype == AC_F32 ? 96 : 64;
    }
    const bool wide = t.kernel == AC_KERNEL_2D_REGW;
    if (wide) {
        t.kernel = AC_KERNEL_2D_REG;
        if (t.tile_x == 128) t.tile_x = 64;
        if (t.tile_y > 0) t.tile_y *= 2;                 // given as the wide tile's height
    }
    if (t.tile_x == 0) t.tile_x = 64;
    // other shapes fill in from depth 8 on 64 x 128 register tiles (8 waves),
    // the fastest 64-wide tile on the 512-grid batch in both precisions (FP32
    // 2692 GLUPS, FP64 1539; depth 7 on 64 x 128: 2602 / 1489; depth 8 on
    // 64 x 192: 2625 / 1482)
    if (t.tile_y == 0) t.tile_y = 128;
    if (t.tb_depth == 0) t.tb_depth = 8;
    ac_plan tp;
    ac_status s = make_plan2d(4096, 4096, nsteps, elem, &t, dev, &tp);
    if (s != AC_OK) return s;
    if (tp.kernel == AC_KERNEL_2D_REGW)
        return fail(AC_ERR_UNSUPPORTED, "batches run 64-wide tiles (kernel %d is 128 wide)", tp.kernel);
    if (wide && tp.kernel != AC_KERNEL_2D_REG)
        return fail(AC_ERR_UNSUPPORTED, "128-wide batch tiles need the register tile body");
    const int LX = tp.tile_x, LY = tp.tile_y, K = tp.tb_depth;
    const int OX = LX - 2 * K, OY = LY - 2 * K;
    std::vector<BatchInst> hi(n);
    std::vector<int4> items;
    for (int32_t i = 0; i < n; ++i) {
        hi[i] = BatchInst{inst[i].phi, inst[i].work, inst[i].nx, inst[i].ny, alpha[i], r[i]};
        // register tiles sit flush against the domain edges (reg2d.h)
        const bool reg = tp.kernel == AC_KERNEL_2D_REG;
        const int w = wide && inst[i].nx >= 128 ? 1 : 0;
        const int tx = w ? reg2d_tiles_1d(inst[i].nx, 128, K)
                       : reg ? reg2d_tiles_1d(inst[i].nx, LX, K) : (inst[i].nx + OX - 1) / OX;
        const int ty = w ? reg2d_tiles_1d(inst[i].ny, LY / 2, K)
                       : reg ? reg2d_tiles_1d(inst[i].ny, LY, K) : (inst[i].ny + OY - 1) / OY;
        for (int y = 0; y < ty; ++y)
            for (int x = 0; x < tx; ++x) items.push_back(int4{i, x, y, w});
    }
    const Chunks c = plan_chunks(nsteps, K);
    // tickets and finished-item counts are 32-bit and monotonic over the call
    if (((double)c.n + 2.0) * (double)items.size() + 1e6 > (double)INT_MAX)
        return fail(AC_ERR_UNSUPPORTED, "%zu tiles x %lld phases exceed the 32-bit work counters",
                    items.size(), (long long)c.n);
    // workgroup size and LDS follow the tile body the plan chose
    const int body_kernel = wide ? AC_KERNEL_2D_REGW : tp.kernel;
    const void *kern = select_kernel(dtype, LX, body_kernel);
    const size_t lds = wide ? std::max((size_t)tp.lds_bytes, tile2d_regw_lds_bytes(LY / 2, elem))
                            : (size_t)tp.lds_bytes;
    const int threads = tp.threads;
    set_lds_limit(kern, lds);
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, lds);
    if (e != hipSuccess) return hip_fail(e, "occupancy query");
    if (per_cu < 1) return fail(AC_ERR_UNSUPPORTED, "batched kernel does not fit on a CU");
    // every workgroup must be resident at once (grid barrier); 8 | grid
    int grid = per_cu * dev.cus;
    const int want = (int)std::min<size_t>((size_t)grid, (items.size() + 7) / 8 * 8);
    grid = std::max(8, want / 8 * 8);
    p.n_items = (int)items.size();
    p.grid = grid;
    if ((e = hipMalloc(&p.d_inst, sizeof(BatchInst) * std::max<int32_t>(n, 1))) != hipSuccess ||
        (e = hipMalloc(&p.d_items, sizeof(int4) * std::max<size_t>(items.size(), 1))) != hipSuccess ||
        (p.active && (e = hipMalloc(&p.d_compact, sizeof(int4) * std::max<size_t>(items.size(), 1))) != hipSuccess) ||
        (p.active && (e = hipMalloc(&p.d_count, sizeof(int))) != hipSuccess) ||
        (e = hipMalloc(&p.d_bar, sizeof(unsigned) * SYNC_WORDS)) != hipSuccess ||
        (e = hipMalloc(&p.d_err, sizeof(int))) != hipSuccess) {
        release(p);
        return fail(AC_ERR_NOMEM, "batched plan allocation: %s", hipGetErrorString(e));
    }
    if (n > 0) e = hipMemcpy(p.d_inst, hi.data(), sizeof(BatchInst) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess && !items.empty())
        e = hipMemcpy(p.d_items, items.data(), sizeof(int4) * items.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(p.d_err, 0, sizeof(int));
    if (e != hipSuccess) { release(p); return hip_fail(e, "batched plan upload"); }

    // capture [reset barrier, persistent kernel] on a library-owned stream
    hipStream_t &cs = g_capture_stream[p.device];
    if (!cs && (e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess) {
        release(p);
        return hip_fail(e, "capture stream");
    }
    if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
        release(p);
        return hip_fail(e, "begin capture");
    }
    if (g_persistent) hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, cs, p.d_bar);
    if (p.active)
        hipLaunchKernelGGL(batch_compact_kernel, dim3(1), dim3(1024), 0, cs, p.d_items, p.n_items,
                           p.active, p.d_compact, p.d_count);
    const int nblocks = (int)c.n;
    const long long spin = g_spin_limit;
    // wall-clock bound of one wait: about 2 s of the constant-rate clock
    int clock_khz = 0;
    if (hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, p.device) != hipSuccess ||
        clock_khz <= 0)
        clock_khz = 100000;
    const long long wall = g_spin_limit == 0 ? 0 : 2000LL * clock_khz;
    const int cb = c.copy_back ? 1 : 0;
    const int base = (int)c.base, rem = (int)c.rem, ni = p.n_items;
    int4 *list = p.active ? p.d_compact : p.d_items;
    const int *cnt = p.d_count;
    void *args[] = {&p.d_inst, &list, (void *)&ni, (void *)&LX, (void *)&LY, (void *)&K,
                    (void *)&nblocks, (void *)&base, (void *)&rem, (void *)&cb, (void *)&cnt,
                    &p.d_bar, &p.d_err, (void *)&spin, (void *)&wall};
    hipError_t le = hipSuccess;
    int phase_grid = 8 * ((ni + 7) / 8);
    if (g_persistent) {
        le = hipLaunchKernel(kern, dim3(grid), dim3(threads), args, lds, cs);
    } else {
        const void *pk = select_phase_kernel(dtype, LX, body_kernel);
        set_lds_limit(pk, lds);
        for (int b = 0; b <= nblocks && le == hipSuccess; ++b) {
            const int copy = b == nblocks;
            if (copy && !cb) break;
            const int k = copy ? 0 : base + (b < rem ? 1 : 0);
            void *pargs[] = {&p.d_inst, &list, (void *)&ni, (void *)&LX, (void *)&LY, (void *)&K,
                             (void *)&k, (void *)&b, (void *)&copy, (void *)&cnt};
            le = hipLaunchKernel(pk, dim3(phase_grid), dim3(threads), pargs, lds, cs);
        }
    }
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    if (le != hipSuccess || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        release(p);
        return hip_fail(le != hipSuccess ? le : e, "capture batched launch");
    }
    p.graph = g;
    if ((e = hipGraphInstantiate(&p.exec, g, nullptr, nullptr, 0)) != hipSuccess) {
        release(p);
        return hip_fail(e, "instantiate batched graph");
    }
    p.info.grid = g_persistent ? grid : phase_grid;
    p.info.items = p.n_items;
    p.info.tb_depth = K;
    p.info.tile_x = wide ? 128 : LX;                    // wide: the tile of the wide instances
    p.info.tile_y = wide ? LY / 2 : LY;
    p.info.blocks = nblocks;
    p.info.copy_back = cb;
    p.info.lds_bytes = (int64_t)lds;
    return AC_OK;
}

bool same_inst3(const ac_instance3d &a, const ac_instance3d &b) {
    return a.phi == b.phi && a.work == b.work && a.nx == b.nx && a.ny == b.ny && a.nz == b.nz &&
           a.h == b.h && a.dt == b.dt && a.eps == b.eps;
}

bool key_equal3(const Plan &p, const ac_instance3d *inst, int32_t n, int64_t nsteps, int32_t dtype,
                const ac_tune &t, int dev) {
    if (p.dim != 3 || p.device != dev || p.nsteps != nsteps || p.dtype != dtype ||
        (int32_t)p.inst3.size() != n)
        return false;
    if (std::memcmp(&p.tune, &t, sizeof t) != 0) return false;
    for (int32_t i = 0; i < n; ++i)
        if (!same_inst3(p.inst3[i], inst[i])) return false;
    return true;
}

ac_status validate_batch3(const ac_instance3d *inst, int32_t n, int64_t nsteps, int32_t dtype,
                          std::vector<double> *alpha, std::vector<double> *r) {
    if (n < 0 || (n > 0 && !inst)) return fail(AC_ERR_INVALID_ARG, "bad instance array");
    alpha->resize(n);
    r->resize(n);
    std::vector<std::pair<uintptr_t, uintptr_t>> ranges;
    ranges.reserve(2 * (size_t)n);
    for (int32_t i = 0; i < n; ++i) {
        const ac_instance3d &I = inst[i];
        if (I.nx < 1 || I.ny < 1 || I.nz < 1)
            return fail(AC_ERR_INVALID_ARG, "instance %d: nx, ny, nz must be >= 1", i);
        const int64_t cells = (int64_t)I.nx * I.ny * I.nz;
        ac_status s = validate(I.phi, I.work, cells, 3, I.h, I.dt, I.eps, nsteps, dtype,
                               &(*alpha)[i], &(*r)[i]);
        if (s != AC_OK) {
            std::string m = g_err;
            return fail(s, "instance %d: %s", i, m.c_str());
        }
        const size_t bytes = (size_t)cells * elem_size(dtype);
        ranges.push_back({(uintptr_t)I.phi, (uintptr_t)I.phi + bytes});
        ranges.push_back({(uintptr_t)I.work, (uintptr_t)I.work + bytes});
    }
    std::sort(ranges.begin(), ranges.end());
    for (size_t i = 1; i < ranges.size(); ++i)
        if (ranges[i].first < ranges[i - 1].second)
            return fail(AC_ERR_INVALID_ARG, "instance buffers overlap");
    return AC_OK;
}

// REG: the batch has register-tile items (the kernel then carries both
// bodies; without them it keeps the LDS body's register count)
template <typename T, int K, bool REG>
const void *kernel3_cpt(int cpt) {
    if (cpt <= 1) return (const void *)batched3d_kernel<T, K, 1, REG>;
    if (cpt <= 2) return (const void *)batched3d_kernel<T, K, 2, REG>;
    if (cpt <= 4) return (const void *)batched3d_kernel<T, K, 4, REG>;
    return nullptr;
}

template <typename T, int K, bool REG>
const void *phase3_cpt(int cpt) {
    if (cpt <= 1) return (const void *)batched3d_phase_kernel<T, K, 1, REG>;
    if (cpt <= 2) return (const void *)batched3d_phase_kernel<T, K, 2, REG>;
    if (cpt <= 4) return (const void *)batched3d_phase_kernel<T, K, 4, REG>;
    return nullptr;
}

template <typename T, bool REG>
const void *phase3_of(int K, int cpt) {
    switch (K) {
    case 1: return phase3_cpt<T, 1, REG>(cpt);
    case 2: return phase3_cpt<T, 2, REG>(cpt);
    case 3: return phase3_cpt<T, 3, REG>(cpt);
    case 4: return phase3_cpt<T, 4, REG>(cpt);
    default: return nullptr;
    }
}

template <typename T, bool REG>
const void *kernel3_of(int K, int cpt) {
    switch (K) {
    case 1: return kernel3_cpt<T, 1, REG>(cpt);
    case 2: return kernel3_cpt<T, 2, REG>(cpt);
    case 3: return kernel3_cpt<T, 3, REG>(cpt);
    case 4: return kernel3_cpt<T, 4, REG>(cpt);
    default: return nullptr;
    }
}

// the kernels of a 3D batch: FP64 never has register items
const void *kernel3_sel(bool f64, bool reg, int K, int cpt) {
    return f64 ? kernel3_of<double, false>(K, cpt)
               : (reg ? kernel3_of<float, true>(K, cpt) : kernel3_of<float, false>(K, cpt));
}
const void *phase3_sel(bool f64, bool reg, int K, int cpt) {
    return f64 ? phase3_of<double, false>(K, cpt)
               : (reg ? phase3_of<float, true>(K, cpt) : phase3_of<float, false>(K, cpt));
}

ac_status build_plan3d(Plan &p, const ac_instance3d *inst, int32_t n, int64_t nsteps,
                       int32_t dtype, const ac_tune &tune, const std::vector<double> &alpha,
                       const std::vector<double> &r, const DevInfo &dev) {
    const size_t elem = elem_size(dtype);
    // kernel 0 or AC_KERNEL_3D_STREAM: the LDS body for every instance.
    // AC_KERNEL_3D_REG: FP32 instances at least 64 cells wide take the
    // register body on flush 64 x 32 tiles (z segments of kRegBatchLZ planes),
    // the others the LDS body.  On the 64-grid workload (sides 24..128) the
    // register items measured slower (591 against 697 GLUPS): at those widths
    // the flush 64-wide tiles recompute up to a third of their columns.
    ac_tune tl = tune;
    const bool mixed = tl.kernel == AC_KERNEL_3D_REG && dtype == AC_F32;
    tl.kernel = AC_KERNEL_3D_STREAM;
    // FP32 default: depth 2, per-instance tiles (below), segments of about 24
    // planes.  Measured on the 64-grid batch of sides 24..128: 915 GLUPS;
    // depth 2 with segments of 12..32 planes 800..915, depth 3 730..830 (one
    // fixed 32 x 32 tile at depth 3 with 16-plane segments: 692)
    if (dtype == AC_F32 && !tl.tb_depth && !tl.tile_x && !tl.tile_y && !tl.tile_z) {
        tl.tb_depth = 2;
        tl.tile_x = tl.tile_y = 32;
        tl.tile_z = 24;
    }
    if (tune.kernel != 0 && tune.kernel != AC_KERNEL_3D_STREAM && tune.kernel != AC_KERNEL_3D_REG)
        return fail(AC_ERR_UNSUPPORTED, "kernel %d is not a 3D kernel", tune.kernel);
    ac_plan tp;
    ac_status s = make_plan3d(256, 256, 256, nsteps, elem, &tl, dev, &tp);
    if (s != AC_OK) return s;
    const int LZ = tp.tile_z, K = tp.tb_depth, threads = tp.threads;
    if (K > 4) return fail(AC_ERR_UNSUPPORTED, "batched 3D supports tb_depth 1..4, got %d", K);
    // LDS tiles: the caller's shape for every instance, or (no shape given)
    // per instance the shape of at most kBatch3dCellsPerThread * threads cells
    // that computes the fewest cells over the instance's xy extent -- a tile
    // computes its K-cell halo too, and on grids of 24..128 cells a fixed
    // 32 x 32 tile computes about 2.7 cells per useful one
    const bool own_shape = tune.tile_x <= 0 && tune.tile_y <= 0;
    auto span = [&](int n, int L) { return (int64_t)((n + L - 2 * K - 1) / (L - 2 * K)) * L; };
    std::vector<int2> shape(n);
    int max_cells = tp.tile_x * tp.tile_y;
    for (int32_t i = 0; i < n; ++i) {
        int2 best{tp.tile_x, tp.tile_y};
        if (own_shape) {
            int64_t bc = span(inst[i].nx, best.x) * span(inst[i].ny, best.y);
            for (int lx = 64; lx >= std::max(16, 2 * K + 1); --lx)
                for (int ly = 64; ly >= 2 * K + 1; --ly) {
                    if (lx * ly > kBatch3dCellsPerThread * threads) continue;
                    const int64_t c = span(inst[i].nx, lx) * span(inst[i].ny, ly);
                    if (c < bc) {
                        bc = c;
                        best = int2{lx, ly};
                    }
                }
        }
        shape[i] = best;
        max_cells = std::max(max_cells, best.x * best.y);
    }
    const int LX = tp.tile_x, LY = (max_cells + LX - 1) / LX;   // LDS and cells per thread: the largest
    Tile3D t3{LX, LY, LZ, K, threads};
    const int cpt = stream3d_cells_per_thread(t3);
    // register items need the 512-thread workgroup of 8 waves x 4 rows
    const bool use_reg = mixed && threads == 64 * (32 / kReg3dRows);
    const int LZR = kRegBatchLZ;
    std::vector<BatchInst> hi(n);
    std::vector<int4> items;
    bool any_reg = false;
    for (int32_t i = 0; i < n; ++i) {
        const int OX = shape[i].x - 2 * K, OY = shape[i].y - 2 * K;
        const int tx = (inst[i].nx + OX - 1) / OX, ty = (inst[i].ny + OY - 1) / OY;
        // z segments: the instance's depth cut evenly into segments of about LZ
        // planes (no short remainder segment)
        const int segs = std::max(1, (inst[i].nz + LZ / 2) / LZ);
        const int lz = (inst[i].nz + segs - 1) / segs;
        const int tz = (inst[i].nz + lz - 1) / lz;
        const bool reg = use_reg && inst[i].nx >= 64;
        const int rtx = reg2d_tiles_1d(inst[i].nx, 64, K), rty = reg2d_tiles_1d(inst[i].ny, 32, K);
        hi[i] = BatchInst{inst[i].phi, inst[i].work, inst[i].nx, inst[i].ny, alpha[i], r[i],
                          inst[i].nz, tx, rtx, shape[i].x, shape[i].y, lz};
        if (reg) {
            any_reg = true;
            for (int z = 0; z < (inst[i].nz + LZR - 1) / LZR; ++z)
                for (int y = 0; y < rty; ++y)
                    for (int x = 0; x < rtx; ++x) items.push_back(int4{i, y * rtx + x, z, 1});
        } else {
            for (int z = 0; z < tz; ++z)
                for (int y = 0; y < ty; ++y)
                    for (int x = 0; x < tx; ++x) items.push_back(int4{i, y * tx + x, z, 0});
        }
    }
    // the phase kernels hand XCD x the x-th eighth of the items, in order:
    // within each eighth the full-length z segments go first and the short
    // last segments of the grids fill the tail
    {
        const size_t per = (items.size() + 7) / 8;
        auto planes = [&](const int4 &it) {
            const int L = it.w ? LZR : hi[it.x].lz;
            return std::min(L, inst[it.x].nz - it.z * L);
        };
        for (size_t b = 0; per > 0 && b < items.size(); b += per)
            std::stable_sort(items.begin() + b, items.begin() + std::min(items.size(), b + per),
                             [&](const int4 &u, const int4 &v) { return planes(u) > planes(v); });
    }
    // whole phases of K steps, then one phase of the remaining steps
    const int64_t q = nsteps / K, rem = nsteps % K;
    const int64_t phases = q + (rem ? 1 : 0);
    const int cb = (int)(phases & 1);                 // result in work: a final copy phase
    if (((double)phases + 2.0) * (double)items.size() + 1e6 > (double)INT_MAX)
        return fail(AC_ERR_UNSUPPORTED, "%zu tiles x %lld phases exceed the 32-bit work counters",
                    items.size(), (long long)phases);
    const bool f64 = dtype == AC_F64;
    const void *kA = kernel3_sel(f64, any_reg, K, cpt);
    const void *kB = rem ? kernel3_sel(f64, any_reg, (int)rem, cpt) : nullptr;
    if (!kA || (rem && !kB)) return fail(AC_ERR_UNSUPPORTED, "no batched 3D kernel for this shape");
    Tile3D tB{LX, LY, LZ, (int)(rem ? rem : K), threads};
    const size_t ldsA = std::max(stream3d_lds_bytes(t3, elem), any_reg ? reg3d_lds_bytes(K, 32, elem) : 0);
    const size_t ldsB = std::max(stream3d_lds_bytes(tB, elem),
                                 any_reg ? reg3d_lds_bytes(tB.K, 32, elem) : 0);
    set_lds_limit(kA, ldsA);
    if (kB) set_lds_limit(kB, ldsB);
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kA, threads, ldsA);
    if (e != hipSuccess) return hip_fail(e, "occupancy query");
    if (per_cu < 1) return fail(AC_ERR_UNSUPPORTED, "batched 3D kernel does not fit on a CU");
    int grid = per_cu * dev.cus;
    const int want = (int)std::min<size_t>((size_t)grid, (items.size() + 7) / 8 * 8);
    grid = std::max(8, want / 8 * 8);
    p.n_items = (int)items.size();
    p.grid = grid;
    if ((e = hipMalloc(&p.d_inst, sizeof(BatchInst) * std::max<int32_t>(n, 1))) != hipSuccess ||
        (e = hipMalloc(&p.d_items, sizeof(int4) * std::max<size_t>(items.size(), 1))) != hipSuccess ||
        (e = hipMalloc(&p.d_bar, sizeof(unsigned) * SYNC_WORDS)) != hipSuccess ||
        (e = hipMalloc(&p.d_err, sizeof(int))) != hipSuccess) {
        release(p);
        return fail(AC_ERR_NOMEM, "batched 3D plan allocation: %s", hipGetErrorString(e));
    }
    if (n > 0) e = hipMemcpy(p.d_inst, hi.data(), sizeof(BatchInst) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess && !items.empty())
        e = hipMemcpy(p.d_items, items.data(), sizeof(int4) * items.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(p.d_err, 0, sizeof(int));
    if (e != hipSuccess) { release(p); return hip_fail(e, "batched 3D plan upload"); }

    hipStream_t &cs = g_capture_stream[p.device];
    if (!cs && (e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess) {
        release(p);
        return hip_fail(e, "capture stream");
    }
    if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
        release(p);
        return hip_fail(e, "begin capture");
    }
    const long long spin = g_spin_limit;
    int clock_khz = 0;
    if (hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, p.device) != hipSuccess ||
        clock_khz <= 0)
        clock_khz = 100000;
    const long long wall = g_spin_limit == 0 ? 0 : 2000LL * clock_khz;
    const int ni = p.n_items;
    hipError_t le = hipSuccess;
    const int phase_grid = 8 * ((ni + 7) / 8);
    if (!g_persistent) {
        // one launch per phase: q of K steps, one of the remaining steps, a copy
        const void *pA = phase3_sel(f64, any_reg, K, cpt);
        const void *pB = rem ? phase3_sel(f64, any_reg, (int)rem, cpt) : nullptr;
        set_lds_limit(pA, ldsA);
        if (pB) set_lds_limit(pB, ldsB);
        for (int64_t b = 0; b < phases + cb && le == hipSuccess; ++b) {
            const int ph = (int)b, copy = b == phases;
            const bool last_rem = rem && b == phases - 1;
            void *pargs[] = {&p.d_inst, &p.d_items, (void *)&ni, (void *)&LX, (void *)&LY,
                             (void *)&LZ, (void *)&LZR, (void *)&ph, (void *)&copy};
            le = hipLaunchKernel(last_rem ? pB : pA, dim3(phase_grid), dim3(threads), pargs,
                                 last_rem ? ldsB : ldsA, cs);
        }
    }
    // launch A: q phases of K steps (+ the copy phase if nothing follows)
    if (g_persistent && q > 0) {
        hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, cs, p.d_bar);
        const int nph = (int)q, ph0 = 0, cbA = rem ? 0 : cb;
        void *args[] = {&p.d_inst, &p.d_items, (void *)&ni, (void *)&LX, (void *)&LY, (void *)&LZ,
                        (void *)&LZR, (void *)&nph, (void *)&ph0, (void *)&cbA, &p.d_bar, &p.d_err,
                        (void *)&spin, (void *)&wall};
        le = hipLaunchKernel(kA, dim3(grid), dim3(threads), args, ldsA, cs);
    }
    // launch B: one phase of the remaining steps (+ the copy phase)
    if (g_persistent && le == hipSuccess && rem) {
        hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, cs, p.d_bar);
        const int nph = 1, ph0 = (int)q, cbB = cb;
        void *args[] = {&p.d_inst, &p.d_items, (void *)&ni, (void *)&LX, (void *)&LY, (void *)&LZ,
                        (void *)&LZR, (void *)&nph, (void *)&ph0, (void *)&cbB, &p.d_bar, &p.d_err,
                        (void *)&spin, (void *)&wall};
        le = hipLaunchKernel(kB, dim3(grid), dim3(threads), args, ldsB, cs);
    }
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    if (le != hipSuccess || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        release(p);
        return hip_fail(le != hipSuccess ? le : e, "capture batched 3D launch");
    }
    p.graph = g;
    if ((e = hipGraphInstantiate(&p.exec, g, nullptr, nullptr, 0)) != hipSuccess) {
        release(p);
        return hip_fail(e, "instantiate batched 3D graph");
    }
    p.info.grid = g_persistent ? grid : phase_grid;
    p.info.items = p.n_items;
    p.info.tb_depth = K;
    p.info.tile_x = LX;
    p.info.tile_y = LY;
    p.info.blocks = (int32_t)phases;
    p.info.copy_back = cb;
    p.info.lds_bytes = (int64_t)ldsA;
    return AC_OK;
}

}  // namespace

// Reports (and clears) a barrier timeout of any cached batched plan on this
// device.  Called by ac_check after the stream has drained.
ac_status batched_check_errors() {
    std::lock_guard<std::mutex> lock(g_mu);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return AC_OK;
    for (Plan &p : g_plans) {
        if (p.device != dev || !p.d_err) continue;
        int v = 0;
        hipError_t e = hipMemcpy(&v, p.d_err, sizeof v, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "read batched error flag");
        if (v) {
            (void)hipMemset(p.d_err, 0, sizeof(int));
            return fail(AC_ERR_HIP, "batched grid barrier timed out; results of that call are "
                                    "incomplete");
        }
    }
    return AC_OK;
}

}  // namespace ac

using namespace ac;

extern "C" {

ac_status ac_step_batched_masked(const ac_instance2d *inst, int32_t n_inst, int64_t nsteps,
                                 int32_t dtype, const ac_tune *tune, const int32_t *active,
                                 ac_batch_info *info, void *stream) {
    g_err.clear();
    std::vector<double> alpha, r;
    ac_status s = validate_batch(inst, n_inst, nsteps, dtype, &alpha, &r);
    if (s != AC_OK) return s;
    // a graph holds one launch per temporal block: long calls run as repeated
    // chunks of kMaxGraphBlocks blocks (an even count, so each ends in phi)
    // and a remainder; the update of a cell does not depend on the blocking
    if (!g_persistent) {
        const int64_t depth = (tune && tune->tb_depth) ? tune->tb_depth : (dtype == AC_F64 ? 5 : 8);
        const int64_t chunk = kMaxGraphBlocks * depth;
        if (nsteps > chunk) {
            for (int64_t done = 0; done < nsteps;) {
                const int64_t n = nsteps - done > chunk ? chunk : nsteps - done;
                if ((s = ac_step_batched_masked(inst, n_inst, n, dtype, tune, active, info, stream)) != AC_OK)
                    return s;
                done += n;
            }
            return AC_OK;
        }
    }
    if (nsteps == 0 || n_inst == 0) {
        if (info) std::memset(info, 0, sizeof *info);
        return AC_OK;
    }
    DevInfo dev;
    hipError_t e = device_info(&dev);
    if (e != hipSuccess) return hip_fail(e, "device query");
    int device = 0;
    if ((e = hipGetDevice(&device)) != hipSuccess) return hip_fail(e, "hipGetDevice");
    ac_tune t{};
    if (tune) t = *tune;
    else {
        ac_tune tabled;
        if (tuned_lookup(AC_TUNE_BATCHED, dtype, 0, 0, 0, &tabled)) t = tabled;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_plans.begin();
    for (; it != g_plans.end(); ++it)
        if (key_equal(*it, inst, n_inst, nsteps, dtype, t, active, device)) break;
    if (it == g_plans.end()) {
        Plan p;
        p.inst.assign(inst, inst + n_inst);
        p.nsteps = nsteps;
        p.dtype = dtype;
        p.tune = t;
        p.active = active;
        p.device = device;
        if ((s = build_plan(p, inst, n_inst, nsteps, dtype, t, alpha, r, dev)) != AC_OK) return s;
        g_plans.push_front(std::move(p));
        while (g_plans.size() > kMaxPlans) {
            (void)hipDeviceSynchronize();   // the evicted graph may still be running
            release(g_plans.back());
            g_plans.pop_back();
        }
        it = g_plans.begin();
    } else if (it != g_plans.begin()) {
        g_plans.splice(g_plans.begin(), g_plans, it);
        it = g_plans.begin();
    }
    if (info) *info = it->info;
    if ((e = hipGraphLaunch(it->exec, reinterpret_cast<hipStream_t>(stream))) != hipSuccess)
        return hip_fail(e, "batched graph launch");
    return AC_OK;
}

ac_status ac_step_batched_tuned(const ac_instance2d *inst, int32_t n_inst, int64_t nsteps,
                                int32_t dtype, const ac_tune *tune, ac_batch_info *info,
                                void *stream) {
    return ac_step_batched_masked(inst, n_inst, nsteps, dtype, tune, nullptr, info, stream);
}

ac_status ac_step_batched(const ac_instance2d *inst, int32_t n_inst, int64_t nsteps,
                          int32_t dtype, void *stream) {
    return ac_step_batched_tuned(inst, n_inst, nsteps, dtype, nullptr, nullptr, stream);
}

ac_status ac_step_batched_3d(const ac_instance3d *inst, int32_t n_inst, int64_t nsteps,
                             int32_t dtype, const ac_tune *tune, ac_batch_info *info,
                             void *stream) {
    g_err.clear();
    std::vector<double> alpha, r;
    ac_status s = validate_batch3(inst, n_inst, nsteps, dtype, &alpha, &r);
    if (s != AC_OK) return s;
    if (!g_persistent) {       // bounded graphs, as for 2D batches
        const int64_t depth = (tune && tune->tb_depth) ? tune->tb_depth : (dtype == AC_F64 ? 3 : 4);
        const int64_t chunk = kMaxGraphBlocks * depth;
        if (nsteps > chunk) {
            for (int64_t done = 0; done < nsteps;) {
                const int64_t n = nsteps - done > chunk ? chunk : nsteps - done;
                if ((s = ac_step_batched_3d(inst, n_inst, n, dtype, tune, info, stream)) != AC_OK)
                    return s;
                done += n;
            }
            return AC_OK;
        }
    }
    if (nsteps == 0 || n_inst == 0) {
        if (info) std::memset(info, 0, sizeof *info);
        return AC_OK;
    }
    DevInfo dev;
    hipError_t e = device_info(&dev);
    if (e != hipSuccess) return hip_fail(e, "device query");
    int device = 0;
    if ((e = hipGetDevice(&device)) != hipSuccess) return hip_fail(e, "hipGetDevice");
    ac_tune t{};
    if (tune) t = *tune;
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_plans.begin();
    for (; it != g_plans.end(); ++it)
        if (key_equal3(*it, inst, n_inst, nsteps, dtype, t, device)) break;
    if (it == g_plans.end()) {
        Plan p;
        p.dim = 3;
        p.inst3.assign(inst, inst + n_inst);
        p.nsteps = nsteps;
        p.dtype = dtype;
        p.tune = t;
        p.active = nullptr;
        p.device = device;
        if ((s = build_plan3d(p, inst, n_inst, nsteps, dtype, t, alpha, r, dev)) != AC_OK) return s;
        g_plans.push_front(std::move(p));
        while (g_plans.size() > kMaxPlans) {
            (void)hipDeviceSynchronize();
            release(g_plans.back());
            g_plans.pop_back();
        }
        it = g_plans.begin();
    } else if (it != g_plans.begin()) {
        g_plans.splice(g_plans.begin(), g_plans, it);
        it = g_plans.begin();
    }
    if (info) *info = it->info;
    if ((e = hipGraphLaunch(it->exec, reinterpret_cast<hipStream_t>(stream))) != hipSuccess)
        return hip_fail(e, "batched 3D graph launch");
    return AC_OK;
}

ac_status ac_batched_release(void) {
    std::lock_guard<std::mutex> lock(g_mu);
    hipError_t e = hipDeviceSynchronize();
    for (Plan &p : g_plans) release(p);
    g_plans.clear();
    return e == hipSuccess ? AC_OK : hip_fail(e, "ac_batched_release");
}

void ac_batched_set_persistent(int32_t on) {
    std::lock_guard<std::mutex> lock(g_mu);
    g_persistent = on != 0;
    if (!g_plans.empty()) (void)hipDeviceSynchronize();
    for (Plan &p : g_plans) release(p);   // the mode is baked into captured graphs
    g_plans.clear();
}

void ac_batched_set_spin_limit(int64_t polls) {
    std::lock_guard<std::mutex> lock(g_mu);
    g_spin_limit = polls < 0 ? 20000000 : polls;
    if (!g_plans.empty()) (void)hipDeviceSynchronize();
    for (Plan &p : g_plans) release(p);   // the limit is baked into captured graphs
    g_plans.clear();
}

}  // extern "C"
