// Device code of the 2D LDS tile: shared by the single-grid tiled kernel and
// the batched persistent kernel.  Algorithm notes are in stencil2d.hip.
#pragma once

#include "ac_internal.h"

namespace ac {

// default rows per chunk in a sub-step (registers: about 4.5 values per row
// per lane)
template <typename T> struct Rows { static constexpr int value = 16; };
template <> struct Rows<double> { static constexpr int value = 8; };
constexpr int LB = 8;    // default global loads in flight per lane while filling the tile

// The in-place variant for 64-wide tiles: one LDS buffer, every wave owns one
// row chunk per sub-step and computes it as a rolling window (three rows of
// reads in flight), sixteen global loads in flight per lane in the fill.
// Half the LDS and about 55 registers per lane: seven tiles fit on a CU.
constexpr int INPLACE_LB = 16, INPLACE_D = 3;

// LDS geometry: pitch LX+2 and LY + RCH + 2 rows per buffer -- a one-cell
// frame plus slack rows, so that the unconditional reads and writes of a
// chunk at the edge of the tile or of the domain stay inside the allocation.
// Frame and slack values never reach an exact cell: a Neumann neighbour is
// replaced by the cell itself with a select, and only exact cells go back to
// HBM.
__host__ __device__ inline int lds_pitch(int LX) { return LX + 2; }
__host__ __device__ inline int lds_rows_rch(int LY, int rch) { return LY + rch + 2; }
__host__ __device__ inline int lds_rows(int LY, size_t elem) { return lds_rows_rch(LY, rows_per_chunk(elem)); }

// One lane's chunk of a sub-step: column x, rows y0 .. y0+RCH-1 of the tile
// (LDS index li0 for row y0), read from A; the RCH new values go to out.
// EX: the tile touches an x edge of the domain; EY: the chunk holds row 0 or
// row ny-1.  Zero-Neumann: a neighbour outside the domain is the cell itself.
// The whole chunk is computed, also rows at or past the exact region: those
// are never read by an exact cell of the next sub-step (the exact region
// shrinks, and rows past the domain are replaced by the Neumann select), and
// the LDS has slack rows for them.
template <typename T, int RCH, bool EX, bool EY>
__device__ __forceinline__ void chunk_compute(const T *A, int li0, int P, int x, int nx, int y0,
                                              int ny, int nrow, T alpha, T r, T out[RCH])
{
    T col[RCH + 2], lf[RCH], rt[RCH];
#pragma unroll
    for (int q = 0; q < RCH + 2; ++q) col[q] = A[li0 + (q - 1) * P];
#pragma unroll
    for (int q = 0; q < RCH; ++q) {
        lf[q] = A[li0 + q * P - 1];
        rt[q] = A[li0 + q * P + 1];
    }
    if (EX) {
        const bool atL = x == 0, atR = x == nx - 1;
#pragma unroll
        for (int q = 0; q < RCH; ++q) {
            lf[q] = atL ? col[q + 1] : lf[q];
            rt[q] = atR ? col[q + 1] : rt[q];
        }
    }
    if (EY) {
        if (y0 == 0) col[0] = col[1];
        if (y0 + nrow == ny) {
#pragma unroll
            for (int q = 0; q < RCH; ++q)
                if (q == nrow - 1) col[q + 2] = col[q + 1];
        }
    }
#pragma unroll
    for (int q = 0; q < RCH; ++q)
        out[q] = update2d<T>(col[q + 1], lf[q], rt[q], col[q], col[q + 2], alpha, r);
}

// The same chunk as a rolling window: the LDS reads of row q + D are issued
// before row q is computed, and a scheduling barrier after each row keeps the
// compiler from hoisting every read of the chunk to the top.  About 3 D + 20
// registers instead of 4.5 per row, so more waves fit on a SIMD.
template <typename T, int RCH, bool EX, bool EY, int D>
__device__ __forceinline__ void chunk_compute_pipe(const T *A, int li0, int P, int x, int nx,
                                                   int y0, int ny, int nrow, T alpha, T r,
                                                   T out[RCH])
{
    T col[RCH + 2], lf[RCH], rt[RCH];                 // col[j] holds row j - 1
#pragma unroll
    for (int j = 0; j < D + 2 && j < RCH + 2; ++j) col[j] = A[li0 + (j - 1) * P];
#pragma unroll
    for (int q = 0; q < D && q < RCH; ++q) {
        lf[q] = A[li0 + q * P - 1];
        rt[q] = A[li0 + q * P + 1];
    }
    const bool atL = EX && x == 0, atR = EX && x == nx - 1;
    const bool top = EY && y0 == 0, bot = EY && y0 + nrow == ny;
#pragma unroll
    for (int q = 0; q < RCH; ++q) {
        if (q + D + 2 <= RCH + 1) col[q + D + 2] = A[li0 + (q + D + 1) * P];
        if (q + D < RCH) {
            lf[q + D] = A[li0 + (q + D) * P - 1];
            rt[q + D] = A[li0 + (q + D) * P + 1];
        }
        const T c = col[q + 1];
        T up = col[q], dn = col[q + 2], l = lf[q], rr = rt[q];
        if (EX) {
            l = atL ? c : l;
            rr = atR ? c : rr;
        }
        if (EY) {
            if (q == 0) up = top ? c : up;
            dn = (bot && q == nrow - 1) ? c : dn;
        }
        out[q] = update2d<T>(c, l, rr, up, dn, alpha, r);
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Separate code for edge and interior chunks: interior tiles (most of a large
// grid) then carry no Neumann selects at all.  edgeX is block-uniform, edgeY
// wave-uniform.
template <typename T, int RCH, int D, bool EX, bool EY>
__device__ __forceinline__ void chunk_variant(const T *A, int li0, int P, int x, int nx, int y0,
                                              int ny, int nrow, T alpha, T r, T out[RCH])
{
    if constexpr (D > 0)
        chunk_compute_pipe<T, RCH, EX, EY, D>(A, li0, P, x, nx, y0, ny, nrow, alpha, r, out);
    else
        chunk_compute<T, RCH, EX, EY>(A, li0, P, x, nx, y0, ny, nrow, alpha, r, out);
}

template <typename T, int RCH, int D>
__device__ __forceinline__ void chunk_dispatch(bool edgeX, bool edgeY, const T *A, int li0, int P,
                                               int x, int nx, int y0, int ny, int nrow, T alpha,
                                               T r, T out[RCH])
{
    if (edgeX) {
        if (edgeY) chunk_variant<T, RCH, D, true, true>(A, li0, P, x, nx, y0, ny, nrow, alpha, r, out);
        else       chunk_variant<T, RCH, D, true, false>(A, li0, P, x, nx, y0, ny, nrow, alpha, r, out);
    } else {
        if (edgeY) chunk_variant<T, RCH, D, false, true>(A, li0, P, x, nx, y0, ny, nrow, alpha, r, out);
        else       chunk_variant<T, RCH, D, false, false>(A, li0, P, x, nx, y0, ny, nrow, alpha, r, out);
    }
}

// Advance output tile (tile_x, tile_y) of one grid by ksteps; the whole
// workgroup participates.  smem holds the LDS buffer(s).
//
// RCH: rows per chunk.  SINGLE: one LDS buffer updated in place -- every
// wave computes its chunk into registers, the workgroup meets at a barrier,
// then writes back -- which halves the LDS of a tile and so doubles the tiles
// a CU holds; it needs at most one chunk per wave per sub-step, i.e. LX <= 64
// and at least ceil(LY / RCH) waves.  Otherwise two buffers ping-pong, one
// barrier per sub-step.  LBT: global loads in flight per lane in the fill.
// D > 0: rolling-window chunks with D rows of reads in flight.
template <typename T, int LXC, int RCH = Rows<T>::value, bool SINGLE = false, int LBT = LB,
          int D = 0>
__device__ __forceinline__ void tile2d_body(const T *src, T *dst, int nx, int ny, T alpha, T r,
                                            int LXr, int LY, int halo, int ksteps, int tile_x,
                                            int tile_y, unsigned char *smem)
{
    const int LX = LXC > 0 ? LXC : LXr;
    const int P = lds_pitch(LX);
    T *bufA = reinterpret_cast<T *>(smem);
    T *bufB = SINGLE ? bufA : bufA + (size_t)P * lds_rows_rch(LY, RCH);

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

    // HBM -> LDS, 64 consecutive x per wave access, LBT loads in flight per lane
    {
        const int W = gx1 - gx0;
        const int cpr = (W + 63) >> 6;                      // 64-wide pieces per row
        const int nr = (gy1 - gy0 - ty + BY - 1) / BY;      // rows handled by this wave
        const int items = max(nr, 0) * cpr;
        for (int w0 = 0; w0 < items; w0 += LBT) {
            T v[LBT];
            int li[LBT];
#pragma unroll
            for (int b = 0; b < LBT; ++b) {
                const int w = w0 + b;
                const int i = w / cpr, j = w - i * cpr;
                const int x = gx0 + tx + 64 * j, y = gy0 + ty + BY * i;
                const bool ok = w < items && x < gx1;
                v[b] = ok ? src[(size_t)y * nx + x] : T(0);
                li[b] = ok ? base + y * P + x : -1;
            }
#pragma unroll
            for (int b = 0; b < LBT; ++b)
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
        T out[RCH];
        int lw = -1;                                          // LDS index of the held chunk
        for (int y0 = cy0 + ty * RCH; y0 < cy1; y0 += BY * RCH) {
            const int nrow = min(RCH, cy1 - y0);              // wave-uniform
            // chunk holds the first or the last row of the domain (wave-uniform)
            const bool edgeY = y0 == 0 || y0 + nrow == ny;
            for (int x = cx0 + tx; x < cx1; x += 64) {
                const int li0 = base + y0 * P + x;
                chunk_dispatch<T, RCH, D>(edgeX, edgeY, A, li0, P, x, nx, y0, ny, nrow, alpha, r, out);
                if (SINGLE) {
                    lw = li0;
                } else {
#pragma unroll
                    for (int q = 0; q < RCH; ++q) B[li0 + q * P] = out[q];
                }
            }
        }
        __syncthreads();
        if (SINGLE) {
            if (lw >= 0) {
#pragma unroll
                for (int q = 0; q < RCH; ++q) A[lw + q * P] = out[q];
            }
            __syncthreads();
        } else {
            T *t = A; A = B; B = t;
        }
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
