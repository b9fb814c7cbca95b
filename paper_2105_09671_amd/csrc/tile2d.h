// Device code of the 2D LDS tile: shared by the single-grid tiled kernel and
// the batched persistent kernel.  Algorithm notes are in stencil2d.hip.
#pragma once

#include "ac_internal.h"

namespace ac {

// rows per chunk in a sub-step (registers: about 4.5 values per row per lane)
template <typename T> struct Rows { static constexpr int value = 16; };
template <> struct Rows<double> { static constexpr int value = 8; };
__host__ __device__ inline int rows_per_chunk(size_t elem) { return elem == 8 ? 8 : 16; }
constexpr int LB = 8;    // global loads in flight per lane while filling the tile

// LDS geometry: pitch LX+2 and LY + RCH + 2 rows -- a one-cell frame plus
// slack rows, so that the unconditional reads and writes of a chunk at the
// edge of the tile or of the domain stay inside the allocation.  Frame and
// slack values never reach an exact cell: a Neumann neighbour is replaced by
// the cell itself with a select, and only exact cells go back to HBM.
__host__ __device__ inline int lds_pitch(int LX) { return LX + 2; }
__host__ __device__ inline int lds_rows(int LY, size_t elem) { return LY + rows_per_chunk(elem) + 2; }

// Advance output tile (tile_x, tile_y) of one grid by ksteps; the whole
// workgroup participates.  smem holds the two LDS buffers.
template <typename T, int LXC>
__device__ __forceinline__ void tile2d_body(const T *src, T *dst, int nx, int ny, T alpha, T r,
                                            int LXr, int LY, int halo, int ksteps, int tile_x,
                                            int tile_y, unsigned char *smem)
{
    constexpr int RCH = Rows<T>::value;
    const int LX = LXC > 0 ? LXC : LXr;
    const int P = lds_pitch(LX);
    T *bufA = reinterpret_cast<T *>(smem);
    T *bufB = bufA + (size_t)P * lds_rows(LY, sizeof(T));

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
    const bool edgeX = edgeL | edgeR;
    // LDS index of global (x, y): (y - ly0 + 1) * P + (x - lx0 + 1)
    const int base = (1 - ly0) * P + (1 - lx0);

    // HBM -> LDS, 64 consecutive x per wave access, LB loads in flight per lane
    {
        const int W = gx1 - gx0;
        const int cpr = (W + 63) >> 6;                      // 64-wide pieces per row
        const int nr = (gy1 - gy0 - ty + BY - 1) / BY;      // rows handled by this wave
        const int items = max(nr, 0) * cpr;
        for (int w0 = 0; w0 < items; w0 += LB) {
            T v[LB];
            int li[LB];
#pragma unroll
            for (int b = 0; b < LB; ++b) {
                const int w = w0 + b;
                const int i = w / cpr, j = w - i * cpr;
                const int x = gx0 + tx + 64 * j, y = gy0 + ty + BY * i;
                const bool ok = w < items && x < gx1;
                v[b] = ok ? src[(size_t)y * nx + x] : T(0);
                li[b] = ok ? base + y * P + x : -1;
            }
#pragma unroll
            for (int b = 0; b < LB; ++b)
                if (li[b] >= 0) bufA[li[b]] = v[b];
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
                // zero-Neumann: a neighbour outside the domain is the cell itself
                if (edgeX) {                                  // block-uniform
                    const bool atL = x == 0, atR = x == nx - 1;
#pragma unroll
                    for (int q = 0; q < RCH; ++q) {
                        lf[q] = atL ? col[q + 1] : lf[q];
                        rt[q] = atR ? col[q + 1] : rt[q];
                    }
                }
                if (y0 == 0) col[0] = col[1];                 // wave-uniform
                if (y0 + nrow == ny) {                        // chunk holds the last row
#pragma unroll
                    for (int q = 0; q < RCH; ++q)
                        if (q == nrow - 1) col[q + 2] = col[q + 1];
                }
                // Whole chunk, also rows at or past cy1: those are never read by
                // an exact cell of the next sub-step (the exact region shrinks, and
                // rows past the domain are replaced by the Neumann select), and
                // the LDS has slack rows for them.
#pragma unroll
                for (int q = 0; q < RCH; ++q)
                    B[li0 + q * P] =
                        update2d<T>(col[q + 1], lf[q], rt[q], col[q], col[q + 2], alpha, r);
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
