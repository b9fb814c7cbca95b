// 2D Allen-Cahn stencil with temporal blocking in LDS (gfx950, wave64).
//
// One workgroup owns an output tile of (LX - 2*halo) x (LY - 2*halo) cells.
// It loads the tile plus a `halo`-wide ring from HBM once, then advances the
// whole loaded region `ksteps` time steps inside LDS, ping-ponging between two
// LDS buffers, and finally stores the output tile.  After sub-step s only the
// region shrunk by s cells on every side that is not a domain edge is still
// exact, so each sub-step computes only that region.
//
// The zero-Neumann ghost layer (section 2) is never stored: a neighbour index
// that falls outside the domain is replaced by the cell itself, at every
// sub-step.  A tile whose loaded region reaches a domain edge therefore does
// not shrink on that side.
//
// When the tile covers the whole grid (halo = 0, LX = nx, LY = ny) one
// workgroup runs every time step of the call in a single launch.
//
// Thread layout: 64 lanes (one wave) along x, blockDim.x/64 waves along y.
// Each lane walks down a column of its strip, carrying the cell above and the
// cell itself in registers, and reads the cell below, left and right from LDS;
// the 64 lanes of a wave touch 64 consecutive LDS words (no bank conflicts).
#include "ac_internal.h"

namespace ac {

template <typename T>
__global__ void __launch_bounds__(1024)
tile2d_kernel(const T *src, T *dst, int nx, int ny, T alpha, T r,
              int LX, int LY, int halo, int ksteps)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *bufA = reinterpret_cast<T *>(smem_raw);
    T *bufB = bufA + (size_t)LX * LY;

    const int tx = threadIdx.x & 63;
    const int ty = threadIdx.x >> 6;
    const int BY = blockDim.x >> 6;

    const int OX = LX - 2 * halo, OY = LY - 2 * halo;
    const int ox0 = blockIdx.x * OX, oy0 = blockIdx.y * OY;
    const int ox1 = min(ox0 + OX, nx), oy1 = min(oy0 + OY, ny);
    const int lx0 = ox0 - halo, ly0 = oy0 - halo;          // global coords of local (0,0)
    const int gx0 = max(lx0, 0), gx1 = min(ox1 + halo, nx); // loaded region
    const int gy0 = max(ly0, 0), gy1 = min(oy1 + halo, ny);
    const bool edgeL = lx0 <= 0, edgeR = ox1 + halo >= nx;
    const bool edgeT = ly0 <= 0, edgeB = oy1 + halo >= ny;

    // HBM -> LDS, rows spread over waves, 64 consecutive x per wave access
    for (int y = gy0 + ty; y < gy1; y += BY) {
        const T *row = src + (size_t)y * nx;
        const int lrow = (y - ly0) * LX - lx0;
        for (int x = gx0 + tx; x < gx1; x += 64)
            bufA[lrow + x] = row[x];
    }
    __syncthreads();

    T *A = bufA, *B = bufB;
    for (int s = 1; s <= ksteps; ++s) {
        const int sh = s < halo ? s : halo;
        const int cx0 = edgeL ? gx0 : gx0 + sh;
        const int cx1 = edgeR ? gx1 : gx1 - sh;
        const int cy0 = edgeT ? gy0 : gy0 + sh;
        const int cy1 = edgeB ? gy1 : gy1 - sh;
        const int rows = cy1 - cy0;
        const int per = (rows + BY - 1) / BY;
        const int ys = cy0 + ty * per;
        const int ye = min(ys + per, cy1);
        if (ys < ye) {
            for (int x = cx0 + tx; x < cx1; x += 64) {
                const bool atL = (x == 0), atR = (x == nx - 1);
                int li = (ys - ly0) * LX + (x - lx0);   // LDS index of (x, y)
                T c = A[li];
                T up = (ys == 0) ? c : A[li - LX];
                for (int y = ys; y < ye; ++y, li += LX) {
                    const T dn = (y == ny - 1) ? c : A[li + LX];
                    const T lf = atL ? c : A[li - 1];
                    const T rt = atR ? c : A[li + 1];
                    B[li] = update2d<T>(c, lf, rt, up, dn, alpha, r);
                    up = c;
                    c = dn;
                }
            }
        }
        __syncthreads();
        T *t = A; A = B; B = t;
    }

    // LDS -> HBM, output tile only
    for (int y = oy0 + ty; y < oy1; y += BY) {
        T *row = dst + (size_t)y * nx;
        const int lrow = (y - ly0) * LX - lx0;
        for (int x = ox0 + tx; x < ox1; x += 64)
            row[x] = A[lrow + x];
    }
}

size_t tile2d_lds_bytes(int LX, int LY, size_t elem) { return 2 * (size_t)LX * LY * elem; }

template <typename T>
hipError_t launch_tile2d(const T *src, T *dst, int nx, int ny, T alpha, T r,
                         const Tile2D &t, int ksteps, hipStream_t stream)
{
    const int OX = t.LX - 2 * t.halo, OY = t.LY - 2 * t.halo;
    dim3 grid((nx + OX - 1) / OX, (ny + OY - 1) / OY);
    const size_t lds = tile2d_lds_bytes(t.LX, t.LY, sizeof(T));
    set_lds_limit((const void *)tile2d_kernel<T>, lds);
    hipLaunchKernelGGL(tile2d_kernel<T>, grid, dim3(t.threads), lds, stream,
                       src, dst, nx, ny, alpha, r, t.LX, t.LY, t.halo, ksteps);
    return hipGetLastError();
}

template hipError_t launch_tile2d<float>(const float *, float *, int, int, float, float,
                                         const Tile2D &, int, hipStream_t);
template hipError_t launch_tile2d<double>(const double *, double *, int, int, double, double,
                                          const Tile2D &, int, hipStream_t);

}  // namespace ac
