// Precision trace: the paper's Err (section 2, Eq. ERReq) between an FP32 and
// an FP64 run of the same explicit step, computed on the device.
//
// 2D: register tiles (reg2d.h) holding both precisions of every cell advance
// `depth` steps per launch; after each sub-step every wave adds the squared
// difference of the two states, in FP64, over the cells of its tile's output
// region -- exact at every sub-step, and each cell of the grid in exactly one
// output region -- and a workgroup adds its per-step sums to sq[t] with one
// FP64 atomic per step.  3D: one launch per step (the update of update3d,
// zero-Neumann by clamped neighbour indices) with the same per-step sums;
// rows are dealt to workgroups round-robin.  A final one-workgroup kernel
// turns the slots into rms[t] = sqrt(sq[t] / cells) and Err = mean over t of
// rms[t].  Both precisions are stepped by update2d / update3d, so the FP32
// path is bitwise the product stepper and the FP64 path the FP64 stepper.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <utility>

#include "ac_internal.h"
#include "reg2d.h"

namespace ac {

namespace {

constexpr int ERR_THREADS = 256;

// the four state buffers must be pairwise disjoint
ac_status check_disjoint(const void *p32, const void *w32, const void *p64, const void *w64,
                         int64_t cells) {
    const uintptr_t b[4] = {(uintptr_t)p32, (uintptr_t)w32, (uintptr_t)p64, (uintptr_t)w64};
    const size_t n[4] = {(size_t)cells * 4, (size_t)cells * 4, (size_t)cells * 8, (size_t)cells * 8};
    for (int i = 0; i < 4; ++i)
        for (int j = i + 1; j < 4; ++j)
            if (b[i] < b[j] + n[j] && b[j] < b[i] + n[i])
                return fail(AC_ERR_INVALID_ARG, "precision-trace buffers overlap");
    return AC_OK;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// workgroup sum of v added to *slot: one FP64 atomic per workgroup
__device__ inline void block_add(double v, double *slot) {
    __shared__ double part[ERR_THREADS / 64];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < ERR_THREADS / 64; ++w) s += part[w];
        atomicAdd(slot, s);
    }
}

// 2D trace tiles: 64 x ERR_ROWS * ERR_WAVES cells, depth up to ERR_DEPTH.
constexpr int ERR_ROWS = 16, ERR_WAVES = 8, ERR_DEPTH = 7;

// The fused steps of one trace tile for one x/y edge variant: both precisions
// advance together; after each sub-step every wave's sum of squared
// differences over the output cells goes to part[s][wave].
template <int EX, bool EY>
__device__ __forceinline__ void err_steps(float (&v32)[ERR_ROWS], double (&v64)[ERR_ROWS], int x,
                                          int nx, int y0, int ny, bool xout, int oy0, int oy1,
                                          float alpha32, float r32, double alpha64, double r64,
                                          int ksteps, float (*x32)[2][ERR_WAVES][64],
                                          double (*x64)[2][ERR_WAVES][64],
                                          double (*part)[ERR_WAVES])
{
    constexpr int RCH = ERR_ROWS, NW = ERR_WAVES;
    const int tx = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int s = 0; s < ksteps; ++s) {
        const int pb = s & 1;
        x32[pb][0][w][tx] = v32[0];
        x32[pb][1][w][tx] = v32[RCH - 1];
        x64[pb][0][w][tx] = v64[0];
        x64[pb][1][w][tx] = v64[RCH - 1];
        __syncthreads();
        const float hu32 = w > 0 ? x32[pb][1][w - 1][tx] : v32[0];
        const float hd32 = w + 1 < NW ? x32[pb][0][w + 1][tx] : v32[RCH - 1];
        const double hu64 = w > 0 ? x64[pb][1][w - 1][tx] : v64[0];
        const double hd64 = w + 1 < NW ? x64[pb][0][w + 1][tx] : v64[RCH - 1];
        float n32[RCH];
        double n64[RCH];
        reg2d_substep<float, RCH, EX, EY>(v32, n32, hu32, hd32, x, nx, y0, ny, alpha32, r32);
        reg2d_substep<double, RCH, EX, EY>(v64, n64, hu64, hd64, x, nx, y0, ny, alpha64, r64);
#pragma unroll
        for (int q = 0; q < RCH; ++q) {
            v32[q] = n32[q];
            v64[q] = n64[q];
        }
        double acc = 0.0;
        if (xout) {
#pragma unroll
            for (int q = 0; q < RCH; ++q) {
                const int y = y0 + q;
                const double e = (double)v32[q] - v64[q];
                acc += (y >= oy0 && y < oy1) ? e * e : 0.0;
            }
        }
        acc = wave_sum(acc);
        if (tx == 0) part[s][w] = acc;
    }
}

// Advance one register tile of both fields by ksteps <= halo steps, adding the
// per-step squared differences over its output region to sq[0 .. ksteps).
// The 1-D grid is XCD-banded as in the 2D register kernel.
__global__ void __launch_bounds__(64 * ERR_WAVES)
err_tile2d_kernel(const float *__restrict__ a32, float *__restrict__ b32,
                  const double *__restrict__ a64, double *__restrict__ b64, int nx, int ny,
                  float alpha32, float r32, double alpha64, double r64, int halo, int ksteps,
                  int tiles_x, int tiles, double *sq)
{
    constexpr int RCH = ERR_ROWS, NW = ERR_WAVES, LY = RCH * NW;
    __shared__ float x32[2][2][NW][64];
    __shared__ double x64[2][2][NW][64];
    __shared__ double part[ERR_DEPTH][NW];
    const int per = (tiles + 7) >> 3;
    const int t = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    if (t >= tiles) return;                         // whole workgroup
    const int tx = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tile_x = t % tiles_x, tile_y = t / tiles_x;
    int lx0, ox0, ox1, ly0, oy0, oy1;
    reg2d_tile_span(tile_x, tiles_x, nx, 64, halo, &lx0, &ox0, &ox1);
    reg2d_tile_span(tile_y, reg2d_tiles_1d(ny, LY, halo), ny, LY, halo, &ly0, &oy0, &oy1);
    const int x = lx0 + tx;
    const int y0 = ly0 + w * RCH;
    const int xc = min(x, nx - 1);
    float v32[RCH];
    double v64[RCH];
#pragma unroll
    for (int q = 0; q < RCH; ++q) {
        const size_t c = (size_t)min(y0 + q, ny - 1) * nx + xc;
        v32[q] = a32[c];
        v64[q] = a64[c];
    }
    const int ex = nx < 64 || tiles_x == 1 ? REG_X_SEL
                   : tile_x == 0           ? REG_X_LEFT
                   : tile_x == tiles_x - 1 ? REG_X_RIGHT
                                           : REG_X_IN;
    const bool edgeY = ny < LY && y0 <= ny - 1 && y0 + RCH - 1 >= ny - 1;
    const bool xout = x >= ox0 && x < ox1;
#define AC_ERR_STEPS(EX_, EY_)                                                                      \
    err_steps<EX_, EY_>(v32, v64, x, nx, y0, ny, xout, oy0, oy1, alpha32, r32, alpha64, r64,      \
                        ksteps, x32, x64, part)
    if (edgeY) {
        switch (ex) {
        case REG_X_IN: AC_ERR_STEPS(REG_X_IN, true); break;
        case REG_X_LEFT: AC_ERR_STEPS(REG_X_LEFT, true); break;
        case REG_X_RIGHT: AC_ERR_STEPS(REG_X_RIGHT, true); break;
        default: AC_ERR_STEPS(REG_X_SEL, true); break;
        }
    } else {
        switch (ex) {
        case REG_X_IN: AC_ERR_STEPS(REG_X_IN, false); break;
        case REG_X_LEFT: AC_ERR_STEPS(REG_X_LEFT, false); break;
        case REG_X_RIGHT: AC_ERR_STEPS(REG_X_RIGHT, false); break;
        default: AC_ERR_STEPS(REG_X_SEL, false); break;
        }
    }
#undef AC_ERR_STEPS
    __syncthreads();
    if ((int)threadIdx.x < ksteps) {
        double sum = 0.0;
#pragma unroll
        for (int i = 0; i < NW; ++i) sum += part[threadIdx.x][i];
        atomicAdd(sq + threadIdx.x, sum);
    }
    if (xout) {
#pragma unroll
        for (int q = 0; q < RCH; ++q) {
            const int y = y0 + q;
            if (y >= oy0 && y < oy1) {
                const size_t c = (size_t)y * nx + x;
                __builtin_nontemporal_store(v32[q], b32 + c);
                __builtin_nontemporal_store(v64[q], b64 + c);
            }
        }
    }
}

// 3D: (plane, row) pairs are dealt to workgroups round-robin; the lanes of a
// workgroup sweep a row in 256-wide strides.
__global__ void __launch_bounds__(ERR_THREADS)
err_step3d_kernel(const float *__restrict__ a32, float *__restrict__ b32,
                  const double *__restrict__ a64, double *__restrict__ b64, int nx, int ny, int nz,
                  float alpha32, float r32, double alpha64, double r64, double *sq_t)
{
    const long long plane = (long long)nx * ny;
    double acc = 0.0;
    for (long long q = blockIdx.x; q < (long long)ny * nz; q += gridDim.x) {
        const int z = (int)(q / ny), y = (int)(q - (long long)z * ny);
        const size_t row = (size_t)z * plane + (size_t)y * nx;
        const long long up = y > 0 ? -(long long)nx : 0, dn = y < ny - 1 ? (long long)nx : 0;
        const long long bk = z > 0 ? -plane : 0, fw = z < nz - 1 ? plane : 0;
        for (int x = threadIdx.x; x < nx; x += blockDim.x) {
            const size_t c = row + x;
            const long long l = x > 0 ? -1 : 0, rr = x < nx - 1 ? 1 : 0;
            const float f = update3d<float>(a32[c], a32[c + l], a32[c + rr], a32[c + up], a32[c + dn],
                                            a32[c + bk], a32[c + fw], alpha32, r32);
            const double d = update3d<double>(a64[c], a64[c + l], a64[c + rr], a64[c + up],
                                              a64[c + dn], a64[c + bk], a64[c + fw], alpha64, r64);
            b32[c] = f;
            b64[c] = d;
            const double e = (double)f - d;
            acc += e * e;
        }
    }
    block_add(acc, sq_t);
}

__global__ void err_zero_kernel(double *sq, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        sq[i] = 0.0;
}

// rms[t] = sqrt(sq[t] / cells) in place; *err = mean of rms (one workgroup)
__global__ void __launch_bounds__(ERR_THREADS)
err_finish_kernel(double *sq, long long n, double cells, double *err)
{
    __shared__ double part[ERR_THREADS / 64];
    double acc = 0.0;
    for (long long i = threadIdx.x; i < n; i += blockDim.x) {
        const double v = sqrt(sq[i] / cells);
        sq[i] = v;
        acc += v;
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < ERR_THREADS / 64; ++w) s += part[w];
        *err = n > 0 ? s / (double)n : 0.0;
    }
}

// Ping-pong both precisions through ceil(nsteps / depth) launches of up to
// `depth` steps; the final states end in phi32 / phi64 (a copy back when the
// launch count is odd).  step(s32, d32, s64, d64, k, slots) runs k steps.
template <typename Launch>
ac_status run_trace(float *phi32, float *work32, double *phi64, double *work64, long long cells,
                    int64_t nsteps, int depth, double *rms, double *err, hipStream_t st,
                    Launch step) {
    const unsigned zb = (unsigned)std::min<long long>((nsteps + 255) / 256 + 1, 1024);
    hipLaunchKernelGGL(err_zero_kernel, dim3(zb), dim3(256), 0, st, rms, (long long)nsteps);
    float *s32 = phi32, *d32 = work32;
    double *s64 = phi64, *d64 = work64;
    int64_t launches = 0;
    for (int64_t t = 0; t < nsteps; t += depth, ++launches) {
        const int k = (int)std::min<int64_t>(depth, nsteps - t);
        step(s32, d32, s64, d64, k, rms + t);
        std::swap(s32, d32);
        std::swap(s64, d64);
    }
    hipLaunchKernelGGL(err_finish_kernel, dim3(1), dim3(ERR_THREADS), 0, st, rms,
                       (long long)nsteps, (double)cells, err);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && (launches & 1)) {
        e = hipMemcpyAsync(phi32, s32, (size_t)cells * 4, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(phi64, s64, (size_t)cells * 8, hipMemcpyDeviceToDevice, st);
    }
    return e == hipSuccess ? AC_OK : hip_fail(e, "precision trace");
}

}  // namespace

}  // namespace ac

using namespace ac;

extern "C" {

ac_status ac_err_2d(float *phi32, float *work32, double *phi64, double *work64, int32_t nx,
                    int32_t ny, double h, double dt, double eps, int64_t nsteps, double *rms,
                    double *err, void *stream) {
    g_err.clear();
    if (nx < 1 || ny < 1) return fail(AC_ERR_INVALID_ARG, "nx, ny must be >= 1 (%d x %d)", nx, ny);
    const int64_t cells = (int64_t)nx * ny;
    double alpha = 0, r = 0;
    ac_status s;
    if ((s = validate(phi32, work32, cells, 2, h, dt, eps, nsteps, AC_F32, &alpha, &r)) != AC_OK) return s;
    if ((s = validate(phi64, work64, cells, 2, h, dt, eps, nsteps, AC_F64, &alpha, &r)) != AC_OK) return s;
    if (!err || (nsteps > 0 && !rms)) return fail(AC_ERR_INVALID_ARG, "rms and err must be non-null");
    if ((s = check_disjoint(phi32, work32, phi64, work64, cells)) != AC_OK) return s;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const float a32 = (float)alpha, r32 = (float)r;
    // depth-7 register tiles of 64 x 128 cells (the 2D stepper's plan on 2048^2)
    const int K = ERR_DEPTH;
    const int64_t tx = reg2d_tiles_1d(nx, 64, K),
                  tiles = tx * reg2d_tiles_1d(ny, ERR_ROWS * ERR_WAVES, K);
    if (tiles > INT_MAX - 8) return fail(AC_ERR_UNSUPPORTED, "grid too large for the trace tiles");
    const dim3 grid((unsigned)((tiles + 7) / 8 * 8));
    return run_trace(phi32, work32, phi64, work64, cells, nsteps, K, rms, err, st,
                     [&](const float *s32, float *d32, const double *s64, double *d64, int k,
                         double *slots) {
                         hipLaunchKernelGGL(err_tile2d_kernel, grid, dim3(64 * ERR_WAVES), 0, st,
                                            s32, d32, s64, d64, nx, ny, a32, r32, alpha, r, K, k,
                                            (int)tx, (int)tiles, slots);
                     });
}

ac_status ac_err_3d(float *phi32, float *work32, double *phi64, double *work64, int32_t nx,
                    int32_t ny, int32_t nz, double h, double dt, double eps, int64_t nsteps,
                    double *rms, double *err, void *stream) {
    g_err.clear();
    if (nx < 1 || ny < 1 || nz < 1)
        return fail(AC_ERR_INVALID_ARG, "nx, ny, nz must be >= 1 (%d x %d x %d)", nx, ny, nz);
    const int64_t cells = (int64_t)nx * ny * nz;
    double alpha = 0, r = 0;
    ac_status s;
    if ((s = validate(phi32, work32, cells, 3, h, dt, eps, nsteps, AC_F32, &alpha, &r)) != AC_OK) return s;
    if ((s = validate(phi64, work64, cells, 3, h, dt, eps, nsteps, AC_F64, &alpha, &r)) != AC_OK) return s;
    if (!err || (nsteps > 0 && !rms)) return fail(AC_ERR_INVALID_ARG, "rms and err must be non-null");
    if ((s = check_disjoint(phi32, work32, phi64, work64, cells)) != AC_OK) return s;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const float a32 = (float)alpha, r32 = (float)r;
    return run_trace(phi32, work32, phi64, work64, cells, nsteps, 1, rms, err, st,
                     [&](const float *s32, float *d32, const double *s64, double *d64, int,
                         double *slot) {
                         hipLaunchKernelGGL(err_step3d_kernel,
                                            dim3((unsigned)std::min<long long>((long long)ny * nz, 1024)), dim3(ERR_THREADS), 0, st,
                                            s32, d32, s64, d64, nx, ny, nz, a32, r32, alpha, r,
                                            slot);
                     });
}

}  // extern "C"
