// Internal declarations shared by the libac translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "ac.h"
#include "update.h"

namespace ac {

// ----------------------------------------------------------- launchers ----
// 2D tiled kernel: each workgroup loads a (LX x LY) tile including a `halo`
// ring, advances it `ksteps` <= halo steps in LDS (or all steps if the tile is
// the whole grid), and stores the interior.
// rows a lane updates per chunk of a 2D tile sub-step (registers: about 4.5
// values per row per lane)
__host__ __device__ inline int rows_per_chunk(size_t elem) { return elem == 8 ? 8 : 16; }

struct Tile2D {
    int LX, LY, halo, threads;
};
template <typename T>
hipError_t launch_tile2d(const T *src, T *dst, int nx, int ny, T alpha, T r,
                         const Tile2D &t, int ksteps, hipStream_t stream);
size_t tile2d_lds_bytes(int LX, int LY, size_t elem);
// in-place variant (LX = 64, one LDS buffer, one row chunk per wave)
template <typename T>
hipError_t launch_tile2d_inplace(const T *src, T *dst, int nx, int ny, T alpha, T r,
                                 const Tile2D &t, int ksteps, hipStream_t stream);
size_t tile2d_inplace_lds_bytes(int LY, size_t elem);
int tile2d_inplace_threads(int LY, size_t elem);

// register-resident variant (LX = 64, kRegRows rows per wave held in VGPRs,
// LY / kRegRows waves of at most 16)
constexpr int kRegRows = 16;
template <typename T>
hipError_t launch_tile2d_reg(const T *src, T *dst, int nx, int ny, T alpha, T r, const Tile2D &t,
                             int ksteps, hipStream_t stream);
// LDS of the register kernel's row exchange: [2 parities][waves][2 rows][64]
inline size_t tile2d_reg_lds_bytes(int LY, size_t elem) {
    return (size_t)4 * (LY / kRegRows) * 64 * elem;
}

// register tiles two columns wide per lane (LX = 128, kRegWRows rows per wave,
// LY / kRegWRows waves of at most 16; nx >= 128)
constexpr int kRegWRows = 8;
template <typename T>
hipError_t launch_tile2d_regw(const T *src, T *dst, int nx, int ny, T alpha, T r, const Tile2D &t,
                              int ksteps, hipStream_t stream);
inline size_t tile2d_regw_lds_bytes(int LY, size_t elem) {
    return (size_t)8 * (LY / kRegWRows) * 64 * elem;
}

// 3D z-streaming kernel with K time levels pipelined along z.
struct Tile3D {
    int LX, LY, LZ, K, threads;
};
template <typename T>
hipError_t launch_stream3d(const T *src, T *dst, int nx, int ny, int nz, T alpha, T r,
                           const Tile3D &t, hipStream_t stream);
size_t stream3d_lds_bytes(const Tile3D &t, size_t elem);
int stream3d_cells_per_thread(const Tile3D &t);
// register-resident 3D variant: LX = 64, kReg3dRows rows per wave, at most
// kReg3dMaxWaves waves, depth 1..reg3d_max_depth; LDS row exchange
// [2][K][2 rows][waves][64]
constexpr int kReg3dRows = 4, kReg3dMaxWaves = 8;
inline int reg3d_max_depth(size_t elem) { return elem == 8 ? 6 : 8; }
inline size_t reg3d_lds_bytes(int K, int LY, size_t elem) {
    return (size_t)4 * K * (LY / kReg3dRows) * 64 * elem;
}
template <typename T>
hipError_t launch_reg3d(const T *src, T *dst, int nx, int ny, int nz, T alpha, T r,
                        const Tile3D &t, hipStream_t stream);
// the register kernel's read mode for a grid (reg3d_stream's SR) and its
// resident workgroups per CU in that mode
bool reg3d_select_reads(int nx, int ny, int nz, size_t elem);
int reg3d_blocks_per_cu(int K, int LY, size_t elem, bool sr);   // 0 if the query fails

// Raise a kernel's dynamic-LDS limit when it asks for more than 64 KiB; a
// runtime that rejects the attribute leaves the launch to report any problem.
inline void set_lds_limit(const void *kernel, size_t bytes) {
    if (bytes > 65536 &&
        hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess)
        (void)hipGetLastError();
}

// ----------------------------------------------------- host helpers ----
// (ac_api.hip) Status with a thread-local message; argument validation that
// makes no HIP call; the even-launch-count step split; per-call plans.
ac_status fail(ac_status s, const char *fmt, ...);
ac_status hip_fail(hipError_t e, const char *what);
extern thread_local std::string g_err;
size_t elem_size(int32_t dtype);
ac_status validate(const void *phi, const void *work, int64_t ncells, int dim, double h,
                   double dt, double eps, int64_t nsteps, int32_t dtype, double *alpha,
                   double *r);
struct Chunks {
    int64_t n, base, rem;  // n launches; launch i does base + (i < rem) steps
    bool copy_back;
};
Chunks plan_chunks(int64_t nsteps, int64_t k);
struct DevInfo;
ac_status make_plan2d(int nx, int ny, int64_t nsteps, size_t elem, const ac_tune *tune,
                      const DevInfo &dev, ac_plan *p);
ac_status make_plan3d(int nx, int ny, int nz, int64_t nsteps, size_t elem, const ac_tune *tune,
                      const DevInfo &dev, ac_plan *p);

// Autotuner table lookup (tune.hip); kind is AC_TUNE_*.
bool tuned_lookup(int kind, int32_t dtype, int64_t nx, int64_t ny, int64_t nz, ac_tune *out);
// Barrier-timeout flags of cached batched plans (batched.hip).
ac_status batched_check_errors();

// Device limits, cached per device.
struct DevInfo {
    int cus;
    size_t lds_per_block;
    int xcds;
};
hipError_t device_info(DevInfo *out);

}  // namespace ac
