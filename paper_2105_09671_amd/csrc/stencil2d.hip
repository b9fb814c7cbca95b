// 2D Allen-Cahn stencil with temporal blocking (gfx950, wave64): the register
// tile kernels, 64 wide with one column per lane (reg2d.h) and 128 wide with
// two (reg2w.h), one of which the default plan takes, and the LDS tile
// kernels described here (two LDS buffers, or one updated in place; tile2d.h).
//
// LDS tiles.  One workgroup owns an output tile of (LX - 2*halo) x (LY - 2*halo) cells.
// It loads the tile plus a `halo`-wide ring from HBM once, then advances the
// loaded region `ksteps` time steps inside LDS, ping-ponging between two LDS
// buffers, and finally stores the output tile.  After sub-step s only the
// region shrunk by s cells on every side that is not a domain edge is still
// exact, so each sub-step computes only that region.
//
// Zero-Neumann boundary (section 2): a neighbour that lies outside the domain
// is replaced by the cell itself, at every sub-step.  The test costs nothing
// on interior tiles: left/right edges are handled under a block-uniform
// branch (only tiles touching the domain's x edges take it) and top/bottom
// under a wave-uniform one (only the chunk holding row 0 or row ny-1).  A tile
// whose loaded region reaches a domain edge does not shrink on that side.
//
// When the tile covers the whole grid (halo = 0) one workgroup runs every time
// step of the call in a single launch.
//
// Thread layout: 64 lanes (one wave) along x, blockDim.x/64 waves along y.
// A sub-step deals chunks of rows (16 in FP32, 8 in FP64) round-robin to the
// waves; in a chunk each lane issues all LDS reads of its column before any
// arithmetic, and the 64 lanes of a wave touch 64 consecutive LDS words.
#include <climits>

#include "reg2d.h"
#include "reg2w.h"
#include "tile2d.h"

namespace ac {

template <typename T, int LXC>
__global__ void __launch_bounds__(1024)
tile2d_kernel(const T *src, T *dst, int nx, int ny, T alpha, T r,
              int LXr, int LY, int halo, int ksteps)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    tile2d_body<T, LXC>(src, dst, nx, ny, alpha, r, LXr, LY, halo, ksteps, blockIdx.x,
                        blockIdx.y, smem_raw);
}

// In-place variant for 64-wide tiles (parameters in tile2d.h).

template <typename T>
__global__ void __launch_bounds__(1024)
tile2d_inplace_kernel(const T *src, T *dst, int nx, int ny, T alpha, T r, int LY, int halo,
                      int ksteps)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    tile2d_body<T, 64, Rows<T>::value, true, INPLACE_LB, INPLACE_D>(
        src, dst, nx, ny, alpha, r, 64, LY, halo, ksteps, blockIdx.x, blockIdx.y, smem_raw);
}

size_t tile2d_inplace_lds_bytes(int LY, size_t elem) {
    return (size_t)lds_pitch(64) * lds_rows(LY, elem) * elem;
}

int tile2d_inplace_threads(int LY, size_t elem) {
    const int rch = rows_per_chunk(elem);
    return 64 * ((LY + rch - 1) / rch);
}

template <typename T>
hipError_t launch_tile2d_inplace(const T *src, T *dst, int nx, int ny, T alpha, T r,
                                 const Tile2D &t, int ksteps, hipStream_t stream)
{
    const int OX = 64 - 2 * t.halo, OY = t.LY - 2 * t.halo;
    dim3 grid((nx + OX - 1) / OX, (ny + OY - 1) / OY);
    const size_t lds = tile2d_inplace_lds_bytes(t.LY, sizeof(T));
    set_lds_limit((const void *)tile2d_inplace_kernel<T>, lds);
    hipLaunchKernelGGL(tile2d_inplace_kernel<T>, grid, dim3(t.threads), lds, stream, src, dst, nx,
                       ny, alpha, r, t.LY, t.halo, ksteps);
    return hipGetLastError();
}

template hipError_t launch_tile2d_inplace<float>(const float *, float *, int, int, float, float,
                                                 const Tile2D &, int, hipStream_t);
template hipError_t launch_tile2d_inplace<double>(const double *, double *, int, int, double,
                                                  double, const Tile2D &, int, hipStream_t);

// Register-resident variant (reg2d.h): 64-wide tiles, kRegRows rows per wave.
// A 1-D grid of ceil(tiles / 8) * 8 workgroups; the dispatcher places
// workgroup b on XCD b mod 8, and XCD x takes the x-th contiguous eighth of
// the row-major tile list, so a tile's halo neighbours mostly run on the same
// XCD and share its L2 (measured 5 % per launch on 2048^2).  Padding
// workgroups of the last eighth exit at once.
template <typename T>
__global__ void __launch_bounds__(1024)
tile2d_reg_kernel(const T *src, T *dst, int nx, int ny, T alpha, T r, int halo, int ksteps,
                  int tiles_x, int tiles)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int per = (tiles + 7) >> 3;
    const int t = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    if (t >= tiles) return;                         // whole workgroup
    reg2d_body<T, kRegRows>(src, dst, nx, ny, alpha, r, halo, ksteps, t % tiles_x, t / tiles_x,
                            reinterpret_cast<T *>(smem_raw));
}

template <typename T>
hipError_t launch_tile2d_reg(const T *src, T *dst, int nx, int ny, T alpha, T r, const Tile2D &t,
                             int ksteps, hipStream_t stream)
{
    const int nw = t.LY / kRegRows;
    const int64_t tx = reg2d_tiles_1d(nx, 64, t.halo),
                  tiles = tx * reg2d_tiles_1d(ny, t.LY, t.halo);
    if (tiles > INT_MAX - 8) return hipErrorInvalidValue;
    dim3 grid((unsigned)((tiles + 7) / 8 * 8));
    hipLaunchKernelGGL(tile2d_reg_kernel<T>, grid, dim3(64 * nw), tile2d_reg_lds_bytes(t.LY, sizeof(T)),
                       stream, src, dst, nx, ny, alpha, r, t.halo, ksteps, (int)tx, (int)tiles);
    return hipGetLastError();
}

template hipError_t launch_tile2d_reg<float>(const float *, float *, int, int, float, float,
                                             const Tile2D &, int, hipStream_t);
template hipError_t launch_tile2d_reg<double>(const double *, double *, int, int, double, double,
                                              const Tile2D &, int, hipStream_t);

// Register tiles two columns wide per lane (reg2w.h), grid as above.
template <typename T>
__global__ void __launch_bounds__(1024)
tile2d_regw_kernel(const T *src, T *dst, int nx, int ny, T alpha, T r, int halo, int ksteps,
                   int tiles_x, int tiles)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int per = (tiles + 7) >> 3;
    const int t = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    if (t >= tiles) return;                         // whole workgroup
    reg2w_body<T, kRegWRows>(src, dst, nx, ny, alpha, r, halo, ksteps, t % tiles_x, t / tiles_x,
                             reinterpret_cast<T *>(smem_raw));
}

template <typename T>
hipError_t launch_tile2d_regw(const T *src, T *dst, int nx, int ny, T alpha, T r, const Tile2D &t,
                              int ksteps, hipStream_t stream)
{
    const int nw = t.LY / kRegWRows;
    if (nx < 128 || t.LX != 128 || t.LY % kRegWRows || nw < 1 || nw > 16 || ksteps > t.halo ||
        t.LY < 2 * t.halo + 1)
        return hipErrorInvalidValue;
    const int64_t tx = reg2d_tiles_1d(nx, 128, t.halo),
                  tiles = tx * reg2d_tiles_1d(ny, t.LY, t.halo);
    if (tiles > INT_MAX - 8) return hipErrorInvalidValue;
    dim3 grid((unsigned)((tiles + 7) / 8 * 8));
    hipLaunchKernelGGL(tile2d_regw_kernel<T>, grid, dim3(64 * nw),
                       tile2d_regw_lds_bytes(t.LY, sizeof(T)), stream, src, dst, nx, ny, alpha, r,
                       t.halo, ksteps, (int)tx, (int)tiles);
    return hipGetLastError();
}

template hipError_t launch_tile2d_regw<float>(const float *, float *, int, int, float, float,
                                              const Tile2D &, int, hipStream_t);
template hipError_t launch_tile2d_regw<double>(const double *, double *, int, int, double, double,
                                               const Tile2D &, int, hipStream_t);

size_t tile2d_lds_bytes(int LX, int LY, size_t elem) {
    return 2 * (size_t)lds_pitch(LX) * lds_rows(LY, elem) * elem;
}

template <typename T, int LXC>
static void launch_lx(dim3 grid, size_t lds, hipStream_t stream, const T *src, T *dst, int nx,
                      int ny, T alpha, T r, const Tile2D &t, int ksteps) {
    set_lds_limit((const void *)tile2d_kernel<T, LXC>, lds);
    hipLaunchKernelGGL((tile2d_kernel<T, LXC>), grid, dim3(t.threads), lds, stream,
                       src, dst, nx, ny, alpha, r, t.LX, t.LY, t.halo, ksteps);
}

template <typename T>
hipError_t launch_tile2d(const T *src, T *dst, int nx, int ny, T alpha, T r,
                         const Tile2D &t, int ksteps, hipStream_t stream)
{
    const int OX = t.LX - 2 * t.halo, OY = t.LY - 2 * t.halo;
    dim3 grid((nx + OX - 1) / OX, (ny + OY - 1) / OY);
    const size_t lds = tile2d_lds_bytes(t.LX, t.LY, sizeof(T));
    switch (t.LX) {
    case 64: launch_lx<T, 64>(grid, lds, stream, src, dst, nx, ny, alpha, r, t, ksteps); break;
    case 128: launch_lx<T, 128>(grid, lds, stream, src, dst, nx, ny, alpha, r, t, ksteps); break;
    case 256: launch_lx<T, 256>(grid, lds, stream, src, dst, nx, ny, alpha, r, t, ksteps); break;
    default: launch_lx<T, 0>(grid, lds, stream, src, dst, nx, ny, alpha, r, t, ksteps); break;
    }
    return hipGetLastError();
}

template hipError_t launch_tile2d<float>(const float *, float *, int, int, float, float,
                                         const Tile2D &, int, hipStream_t);
template hipError_t launch_tile2d<double>(const double *, double *, int, int, double, double,
                                          const Tile2D &, int, hipStream_t);

}  // namespace ac
