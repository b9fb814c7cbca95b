// 2D Allen-Cahn stencil with temporal blocking in LDS (gfx950, wave64).
//
// One workgroup owns an output tile of (LX - 2*halo) x (LY - 2*halo) cells.
// It loads the tile plus a `halo`-wide ring from HBM once, then advances the
// loaded region `ksteps` time steps inside LDS, ping-ponging between two LDS
// buffers, and finally stores the output tile.  After sub-step s only the
// region shrunk by s cells on every side that is not a domain edge is still
// exact, so each sub-step computes only that region.
//
// Zero-Neumann boundary (section 2): the LDS tile has a one-cell frame.  Where
// the tile touches a domain edge the frame holds the ghost layer, i.e. a copy
// of the adjacent interior cell, exactly as in the paper's extended grid.  The
// ghosts are written when the tile is loaded and again by every edge cell each
// time it is updated, so the stencil reads its four neighbours from LDS with no
// boundary test at all.  A tile whose loaded region reaches a domain edge does
// not shrink on that side.
//
// When the tile covers the whole grid (halo = 0) one workgroup runs every time
// step of the call in a single launch.
//
// Thread layout: 64 lanes (one wave) along x, blockDim.x/64 waves along y.
// A sub-step deals chunks of RCH rows round-robin to the waves; in a chunk each
// lane issues all 3*RCH+2 LDS reads of its column before any arithmetic, and
// the 64 lanes of a wave touch 64 consecutive LDS words (no bank conflicts).
#include "ac_internal.h"

namespace ac {

constexpr int RCH = 8;   // rows per chunk in a sub-step
constexpr int LB = 8;    // global loads in flight per lane while filling the tile

// LDS geometry: pitch LX+2 (one frame column each side), LY + RCH + 2 rows
// (one frame row above, the frame row below plus RCH rows of slack for the
// unconditional reads of a chunk that ends at the bottom of the tile).
__host__ __device__ inline int lds_pitch(int LX) { return LX + 2; }
__host__ __device__ inline int lds_rows(int LY) { return LY + RCH + 2; }

template <typename T, int LXC>
__global__ void __launch_bounds__(1024)
tile2d_kernel(const T *src, T *dst, int nx, int ny, T alpha, T r,
              int LXr, int LY, int halo, int ksteps)
{
    const int LX = LXC > 0 ? LXC : LXr;
    const int P = lds_pitch(LX);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *bufA = reinterpret_cast<T *>(smem_raw);
    T *bufB = bufA + (size_t)P * lds_rows(LY);

    const int tx = threadIdx.x & 63;
    const int ty = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave index
    const int BY = blockDim.x >> 6;

    const int OX = LX - 2 * halo, OY = LY - 2 * halo;
    const int ox0 = blockIdx.x * OX, oy0 = blockIdx.y * OY;
    const int ox1 = min(ox0 + OX, nx), oy1 = min(oy0 + OY, ny);
    const int lx0 = ox0 - halo, ly0 = oy0 - halo;          // global coords of tile (0,0)
    const int gx0 = max(lx0, 0), gx1 = min(ox1 + halo, nx); // loaded region
    const int gy0 = max(ly0, 0), gy1 = min(oy1 + halo, ny);
    const bool edgeL = lx0 <= 0, edgeR = ox1 + halo >= nx;
    const bool edgeT = ly0 <= 0, edgeB = oy1 + halo >= ny;
    // LDS index of global (x, y): (y - ly0 + 1) * P + (x - lx0 + 1)
    const int base = (1 - ly0) * P + (1 - lx0);

    // HBM -> LDS, 64 consecutive x per wave access; edge cells also fill ghosts.
    // Loads are issued in batches of LB per lane, all in flight together.
    {
        const int W = gx1 - gx0;
        const int cpr = (W + 63) >> 6;                      // 64-wide pieces per row
        const int nr = (gy1 - gy0 - ty + BY - 1) / BY;      // rows handled by this wave
        const int items = max(nr, 0) * cpr;
        for (int w0 = 0; w0 < items; w0 += LB) {
            T v[LB];
            int xs[LB], ys[LB];
#pragma unroll
            for (int b = 0; b < LB; ++b) {
                const int w = w0 + b;
                const int i = w / cpr, j = w - i * cpr;
                xs[b] = gx0 + tx + 64 * j;
                ys[b] = gy0 + ty + BY * i;
                const bool ok = w < items && xs[b] < gx1;
                v[b] = ok ? src[(size_t)ys[b] * nx + xs[b]] : T(0);
                if (!ok) xs[b] = -1;
            }
#pragma unroll
            for (int b = 0; b < LB; ++b) {
                const int x = xs[b], y = ys[b];
                if (x >= 0) {
                    const int li = base + y * P + x;
                    bufA[li] = v[b];
                    if (x == 0) bufA[li - 1] = v[b];
                    if (x == nx - 1) bufA[li + 1] = v[b];
                    if (y == 0) bufA[li - P] = v[b];
                    if (y == ny - 1) bufA[li + P] = v[b];
                }
            }
        }
    }
    __syncthreads();

    T *A = bufA, *B = bufB;
    for (int s = 1; s <= ksteps; ++s) {
        const int sh = s < halo ? s : halo;
        const int cx0 = edgeL ? gx0 : gx0 + sh;
        const int cx1 = edgeR ? gx1 : gx1 - sh;
        const int cy0 = edgeT ? gy0 : gy0 + sh;
        const int cy1 = edgeB ? gy1 : gy1 - sh;
        for (int y0 = cy0 + ty * RCH; y0 < cy1; y0 += BY * RCH) {
            const int nrow = min(RCH, cy1 - y0);              // wave-uniform
            // ghost rows are only touched by chunks that hold a domain edge row
            const bool ghostY = (y0 == 0) || (y0 + nrow == ny);
            for (int x = cx0 + tx; x < cx1; x += 64) {
                const int li0 = base + y0 * P + x;
                T col[RCH + 2], lf[RCH], rt[RCH];
#pragma unroll
                for (int q = 0; q < RCH + 2; ++q) col[q] = A[li0 + (q - 1) * P];
#pragma unroll
                for (int q = 0; q < RCH; ++q) {
                    lf[q] = A[li0 + q * P - 1];
                    rt[q] = A[li0 + q * P + 1];
                }
                T v[RCH];
#pragma unroll
                for (int q = 0; q < RCH; ++q)
                    v[q] = update2d<T>(col[q + 1], lf[q], rt[q], col[q], col[q + 2], alpha, r);
                if (nrow == RCH) {
#pragma unroll
                    for (int q = 0; q < RCH; ++q) B[li0 + q * P] = v[q];
                } else {
#pragma unroll
                    for (int q = 0; q < RCH; ++q)
                        if (q < nrow) B[li0 + q * P] = v[q];
                }
                // Neumann ghosts: block-uniform tests first, so interior tiles
                // skip them with a scalar branch
                if (edgeL | edgeR) {
                    if (x == 0 || x == nx - 1) {
                        const int o = (x == 0) ? -1 : 1;
#pragma unroll
                        for (int q = 0; q < RCH; ++q)
                            if (q < nrow) {
                                B[li0 + q * P + o] = v[q];
                                if (nx == 1) B[li0 + q * P + 1] = v[q];
                            }
                    }
                }
                if (ghostY) {
                    if (y0 == 0) B[li0 - P] = v[0];
#pragma unroll
                    for (int q = 0; q < RCH; ++q)
                        if (q < nrow && y0 + q == ny - 1) B[li0 + (q + 1) * P] = v[q];
                }
            }
        }
        __syncthreads();
        T *t = A; A = B; B = t;
    }

    // LDS -> HBM, output tile only
    for (int y = oy0 + ty; y < oy1; y += BY) {
        T *row = dst + (size_t)y * nx;
        const int lrow = base + y * P;
        for (int x = ox0 + tx; x < ox1; x += 64)
            row[x] = A[lrow + x];
    }
}

size_t tile2d_lds_bytes(int LX, int LY, size_t elem) {
    return 2 * (size_t)lds_pitch(LX) * lds_rows(LY) * elem;
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
