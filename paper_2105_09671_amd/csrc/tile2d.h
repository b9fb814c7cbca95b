// Device code of the 2D LDS tile: shared by the single-grid tiled kernel and
// the batched persistent kernel.  Algorithm notes are in stencil2d.hip.
#pragma once

#include "ac_internal.h"

namespace ac {

constexpr int RCH = 8;   // rows per chunk in a sub-step
constexpr int LB = 8;    // global loads in flight per lane while filling the tile

// LDS geometry: pitch LX+2 (one frame column each side), LY + RCH + 2 rows
// (one frame row above, the frame row below plus RCH rows of slack for the
// unconditional reads of a chunk that ends at the bottom of the tile).
__host__ __device__ inline int lds_pitch(int LX) { return LX + 2; }
__host__ __device__ inline int lds_rows(int LY) { return LY + RCH + 2; }

// Advance output tile (tile_x, tile_y) of one grid by ksteps; the whole
// workgroup participates.  smem holds the two LDS buffers.
template <typename T, int LXC>
__device__ __forceinline__ void tile2d_body(const T *src, T *dst, int nx, int ny, T alpha, T r,
                                            int LXr, int LY, int halo, int ksteps, int tile_x,
                                            int tile_y, unsigned char *smem)
{
    const int LX = LXC > 0 ? LXC : LXr;
    const int P = lds_pitch(LX);
    T *bufA = reinterpret_cast<T *>(smem);
    T *bufB = bufA + (size_t)P * lds_rows(LY);

    const int tx = threadIdx.x & 63;
    const int ty = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave index
    const int BY = blockDim.x >> 6;

    const int OX = LX - 2 * halo, OY = LY - 2 * halo;
    const int ox0 = tile_x * OX, oy0 = tile_y * OY;
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

}  // namespace ac
