// Precision trace: the paper's Err (section 2, Eq. ERReq) between an FP32 and
// an FP64 run of the same explicit step, computed on the device.
//
// One launch advances both fields by one step (the update of update2d /
// update3d, zero-Neumann by clamped neighbour indices) and adds the squared
// difference of the two new states, in FP64, to that step's slot of
// sq[nsteps]: per-lane sums, a workgroup reduction (cross-lane shuffles, then
// LDS), one FP64 atomic per workgroup and at most 1024 workgroups.  A final one-workgroup kernel turns the slots into
// rms[t] = sqrt(sq[t] / cells) and Err = mean over t of rms[t].  The fields are
// read from HBM every step (no temporal blocking): this is a verification
// path, its cost is two plain stencil passes per step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <utility>

#include "ac_internal.h"

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

// Rows (2D) or (plane, row) pairs (3D) are dealt to workgroups round-robin;
// the lanes of a workgroup sweep a row in 256-wide strides.
__global__ void __launch_bounds__(ERR_THREADS)
err_step2d_kernel(const float *__restrict__ a32, float *__restrict__ b32,
                  const double *__restrict__ a64, double *__restrict__ b64, int nx, int ny,
                  float alpha32, float r32, double alpha64, double r64, double *sq_t)
{
    double acc = 0.0;
    for (int y = blockIdx.x; y < ny; y += gridDim.x) {
        const size_t row = (size_t)y * nx;
        const long long up = y > 0 ? -(long long)nx : 0, dn = y < ny - 1 ? (long long)nx : 0;
        for (int x = threadIdx.x; x < nx; x += blockDim.x) {
            const size_t c = row + x;
            const long long l = x > 0 ? -1 : 0, rr = x < nx - 1 ? 1 : 0;
            const float f = update2d<float>(a32[c], a32[c + l], a32[c + rr], a32[c + up], a32[c + dn],
                                            alpha32, r32);
            const double d = update2d<double>(a64[c], a64[c + l], a64[c + rr], a64[c + up],
                                              a64[c + dn], alpha64, r64);
            b32[c] = f;
            b64[c] = d;
            const double e = (double)f - d;
            acc += e * e;
        }
    }
    block_add(acc, sq_t);
}

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

// Ping-pong both precisions through nsteps one-step launches; the final states
// end in phi32 / phi64 (a copy back when nsteps is odd).
template <typename Launch>
ac_status run_trace(float *phi32, float *work32, double *phi64, double *work64, long long cells,
                    int64_t nsteps, double *rms, double *err, hipStream_t st, Launch step) {
    const unsigned zb = (unsigned)std::min<long long>((nsteps + 255) / 256 + 1, 1024);
    hipLaunchKernelGGL(err_zero_kernel, dim3(zb), dim3(256), 0, st, rms, (long long)nsteps);
    (void)cells;
    float *s32 = phi32, *d32 = work32;
    double *s64 = phi64, *d64 = work64;
    for (int64_t t = 0; t < nsteps; ++t) {
        step(s32, d32, s64, d64, rms + t);
        std::swap(s32, d32);
        std::swap(s64, d64);
    }
    hipLaunchKernelGGL(err_finish_kernel, dim3(1), dim3(ERR_THREADS), 0, st, rms,
                       (long long)nsteps, (double)cells, err);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && (nsteps & 1)) {
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
    return run_trace(phi32, work32, phi64, work64, cells, nsteps, rms, err, st,
                     [&](const float *s32, float *d32, const double *s64, double *d64,
                         double *slot) {
                         hipLaunchKernelGGL(err_step2d_kernel, dim3((unsigned)std::min(ny, 1024)), dim3(ERR_THREADS), 0, st,
                                            s32, d32, s64, d64, nx, ny, a32, r32, alpha, r, slot);
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
    return run_trace(phi32, work32, phi64, work64, cells, nsteps, rms, err, st,
                     [&](const float *s32, float *d32, const double *s64, double *d64,
                         double *slot) {
                         hipLaunchKernelGGL(err_step3d_kernel,
                                            dim3((unsigned)std::min<long long>((long long)ny * nz, 1024)), dim3(ERR_THREADS), 0, st,
                                            s32, d32, s64, d64, nx, ny, nz, a32, r32, alpha, r,
                                            slot);
                     });
}

}  // extern "C"
