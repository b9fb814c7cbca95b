// 3D Allen-Cahn 7-point stencil, streamed along z with K time levels
// pipelined in one pass (temporal blocking, gfx950 wave64).
//
// A workgroup owns an (LX - 2K) x (LY - 2K) column of output cells over the z
// segment [oz0, oz0 + LZ).  It streams planes t = oz0-K, oz0-K+1, ... through
// the kernel.  At iteration t, level 0 is plane t read from HBM, and level s
// (1 <= s <= K) advances plane t-s from time level s-1 to s.  The z
// neighbours of a level-s update come from registers (each thread keeps, per
// level, the last two planes of every cell it owns); the x/y neighbours come
// from an LDS copy of the level s-1 plane produced in the previous iteration.
// The level-K plane t-K is the output and goes back to HBM.  HBM traffic is
// therefore one read and one write per cell per K time steps, plus the halo.
//
// Level s is exact on the loaded tile shrunk by s cells on each side that is
// not a domain edge (and for planes at least s above the segment's first
// loaded plane, unless that is the domain bottom), so the level-K output tile
// is exact.  Cells outside the exact region compute values nobody reads.
//
// Zero-Neumann boundary (section 2): neighbour indices that fall outside the
// domain are replaced by the cell itself, in x, y and z, at every level.
//
// LDS holds two sets (even/odd iteration) of K planes of LX*LY values so one
// barrier per iteration separates producers from consumers.
//
// This file holds two kernels of that scheme: stream3d_kernel (stream3d.h),
// whose planes live in LDS, and reg3d_kernel (reg3d.h), whose planes live in
// registers with 64-wide tiles (x neighbours by cross-lane shifts, y edge
// rows through LDS).  The plan takes the register kernel for grids that give
// it enough workgroups and the LDS kernel for smaller ones.
#include "reg3d.h"
#include "stream3d.h"

namespace ac {

template <typename T, int K, int CPT>
__global__ void __launch_bounds__(512)
stream3d_kernel(const T *__restrict__ src, T *__restrict__ dst, int nx, int ny, int nz,
                T alpha, T r, int LX, int LY, int LZ, int tiles_x)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    stream3d_body<T, K, CPT>(src, dst, nx, ny, nz, alpha, r, LX, LY, LZ, tiles_x, blockIdx.x,
                             blockIdx.y, smem_raw);
}

size_t stream3d_lds_bytes(const Tile3D &t, size_t elem) {
    return 2 * (size_t)t.K * t.LX * t.LY * elem;
}

int stream3d_cells_per_thread(const Tile3D &t) {
    return (t.LX * t.LY + t.threads - 1) / t.threads;
}

template <typename T, int K, int CPT>
static hipError_t launch3(const T *src, T *dst, int nx, int ny, int nz, T alpha, T r,
                          const Tile3D &t, hipStream_t stream)
{
    const int OX = t.LX - 2 * K, OY = t.LY - 2 * K;
    const int tiles_x = (nx + OX - 1) / OX, tiles_y = (ny + OY - 1) / OY;
    dim3 grid(tiles_x * tiles_y, (nz + t.LZ - 1) / t.LZ);
    const size_t lds = stream3d_lds_bytes(t, sizeof(T));
    set_lds_limit((const void *)stream3d_kernel<T, K, CPT>, lds);
    hipLaunchKernelGGL((stream3d_kernel<T, K, CPT>), grid, dim3(t.threads), lds, stream,
                       src, dst, nx, ny, nz, alpha, r, t.LX, t.LY, t.LZ, tiles_x);
    return hipGetLastError();
}

template <typename T, int K>
static hipError_t launch3_cpt(const T *src, T *dst, int nx, int ny, int nz, T alpha, T r,
                              const Tile3D &t, hipStream_t stream)
{
    const int cpt = stream3d_cells_per_thread(t);
    if (cpt <= 1) return launch3<T, K, 1>(src, dst, nx, ny, nz, alpha, r, t, stream);
    if (cpt <= 2) return launch3<T, K, 2>(src, dst, nx, ny, nz, alpha, r, t, stream);
    if (cpt <= 4) return launch3<T, K, 4>(src, dst, nx, ny, nz, alpha, r, t, stream);
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_stream3d(const T *src, T *dst, int nx, int ny, int nz, T alpha, T r,
                           const Tile3D &t, hipStream_t stream)
{
    switch (t.K) {
    case 1: return launch3_cpt<T, 1>(src, dst, nx, ny, nz, alpha, r, t, stream);
    case 2: return launch3_cpt<T, 2>(src, dst, nx, ny, nz, alpha, r, t, stream);
    case 3: return launch3_cpt<T, 3>(src, dst, nx, ny, nz, alpha, r, t, stream);
    case 4: return launch3_cpt<T, 4>(src, dst, nx, ny, nz, alpha, r, t, stream);
    case 5: return launch3_cpt<T, 5>(src, dst, nx, ny, nz, alpha, r, t, stream);
    case 6: return launch3_cpt<T, 6>(src, dst, nx, ny, nz, alpha, r, t, stream);
    case 7: return launch3_cpt<T, 7>(src, dst, nx, ny, nz, alpha, r, t, stream);
    case 8: return launch3_cpt<T, 8>(src, dst, nx, ny, nz, alpha, r, t, stream);
    default: return hipErrorInvalidValue;
    }
}

// Register-resident variant (reg3d.h): 64-wide tiles, kReg3dRows rows per wave.
// SR: the rows beyond a wave are read at a selected LDS address rather than
// under a branch (reg3d_stream).
// The grid is one-dimensional over (z segment, xy tile), xy tiles fastest,
// numbered XCD-aware: workgroup b runs on XCD b % 8 and takes item
// (b % 8) * per + b / 8, so each XCD works through a contiguous range of
// neighbouring tiles and the halo the neighbours share (K columns, rows and
// planes around every tile) is read through one L2.
template <typename T, int K, bool SR>
__global__ void __launch_bounds__(512)
reg3d_kernel(const T *__restrict__ src, T *__restrict__ dst, int nx, int ny, int nz, T alpha, T r,
             int LZ, int tiles_x, int tiles_xy, int items)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int per = (items + 7) >> 3;
    const int item = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    if ((int)(blockIdx.x >> 3) >= per || item >= items) return;   // padding workgroup (whole group)
    reg3d_body<T, K, kReg3dRows, SR>(src, dst, nx, ny, nz, alpha, r, LZ, tiles_x, item % tiles_xy,
                                     item / tiles_xy, reinterpret_cast<T *>(smem_raw));
}

template <typename T, int K, bool SR>
static const void *reg3d_ptr() { return (const void *)reg3d_kernel<T, K, SR>; }

// Depths up to reg3d_max_depth: FP32 8 (169 VGPRs at depth 8), FP64 6 (211
// VGPRs; depth 8 would spill).
template <typename T, bool SR>
static const void *reg3d_kernel_k(int K) {
    switch (K) {
    case 1: return reg3d_ptr<T, 1, SR>();
    case 2: return reg3d_ptr<T, 2, SR>();
    case 3: return reg3d_ptr<T, 3, SR>();
    case 4: return reg3d_ptr<T, 4, SR>();
    case 5: return reg3d_ptr<T, 5, SR>();
    case 6: return reg3d_ptr<T, 6, SR>();
    default: break;
    }
    if constexpr (sizeof(T) == 4) {
        if (K == 7) return reg3d_ptr<T, 7, SR>();
        if (K == 8) return reg3d_ptr<T, 8, SR>();
    }
    return nullptr;
}

// The read mode per grid (measured on MI355X, A/B on one box): the selected
// address lets every level's cross-lane shifts fold into adds and wins in FP64
// (256^3 +5.5 %, 512^3 +4 %) and in FP32 up to 512^3 (256^3 +5 %, 512^3
// +2 %, 768^3 even), while FP32 1024^3 runs 5 % faster with the branch.
bool reg3d_select_reads(int nx, int ny, int nz, size_t elem) {
    return elem == 8 || (int64_t)nx * ny * nz <= (int64_t)512 * 512 * 512;
}

static const void *reg3d_kernel_of(int K, size_t elem, bool sr) {
    if (elem == 8) return reg3d_kernel_k<double, true>(K);
    return sr ? reg3d_kernel_k<float, true>(K) : reg3d_kernel_k<float, false>(K);
}

int reg3d_blocks_per_cu(int K, int LY, size_t elem, bool sr) {
    const void *k = reg3d_kernel_of(K, elem, sr);
    if (!k) return 0;
    const size_t lds = reg3d_lds_bytes(K, LY, elem);
    set_lds_limit(k, lds);
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, 64 * (LY / kReg3dRows), lds) !=
        hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return n;
}

template <typename T>
hipError_t launch_reg3d(const T *src, T *dst, int nx, int ny, int nz, T alpha, T r,
                        const Tile3D &t, hipStream_t stream)
{
    const void *k = reg3d_kernel_of(t.K, sizeof(T), reg3d_select_reads(nx, ny, nz, sizeof(T)));
    if (!k || t.LX != 64 || t.LY % kReg3dRows || t.LY / kReg3dRows > kReg3dMaxWaves)
        return hipErrorInvalidValue;
    // xy tiles flush against the domain edges (reg2d_tile_span)
    const int tiles_x = reg2d_tiles_1d(nx, 64, t.K), tiles_y = reg2d_tiles_1d(ny, t.LY, t.K);
    const int tiles_xy = tiles_x * tiles_y;
    const int64_t items64 = (int64_t)tiles_xy * ((nz + t.LZ - 1) / t.LZ);
    if (items64 > INT_MAX - 8) return hipErrorInvalidValue;
    int items = (int)items64;
    dim3 grid(8 * ((items + 7) / 8));
    const size_t lds = reg3d_lds_bytes(t.K, t.LY, sizeof(T));
    set_lds_limit(k, lds);
    void *args[] = {(void *)&src, (void *)&dst, (void *)&nx,   (void *)&ny,       (void *)&nz,
                    (void *)&alpha, (void *)&r, (void *)&t.LZ, (void *)&tiles_x, (void *)&tiles_xy,
                    (void *)&items};
    return hipLaunchKernel(k, grid, dim3(64 * (t.LY / kReg3dRows)), args, lds, stream);
}

template hipError_t launch_reg3d<float>(const float *, float *, int, int, int, float, float,
                                        const Tile3D &, hipStream_t);
template hipError_t launch_reg3d<double>(const double *, double *, int, int, int, double, double,
                                         const Tile3D &, hipStream_t);

template hipError_t launch_stream3d<float>(const float *, float *, int, int, int, float, float,
                                           const Tile3D &, hipStream_t);
template hipError_t launch_stream3d<double>(const double *, double *, int, int, int, double,
                                            double, const Tile3D &, hipStream_t);

}  // namespace ac
