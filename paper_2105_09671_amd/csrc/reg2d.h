// Register-resident 2D tiles with temporal blocking (gfx950, wave64).
//
// A workgroup of NW waves owns a tile 64 cells wide and NW*RCH rows tall,
// including a `halo`-wide ring.  Lane l of wave w holds column l of rows
// w*RCH .. w*RCH+RCH-1 in VGPRs for all the fused steps:
//   * the x neighbours of a cell are the same row in lanes l-1 and l+1, read
//     with a whole-wave DPP shift (no LDS traffic);
//   * the y neighbours are the lane's own registers, except for the first and
//     last row of a wave, whose outer neighbours come from the adjacent waves
//     through a small LDS exchange buffer (two rows per wave per step, double
//     buffered by step parity, so one barrier per step suffices).
// The tile is loaded once from HBM and its exact interior stored once per
// launch, as in the LDS-tiled kernels; after s fused steps the cells within s
// of a non-domain tile edge are no longer exact, hence the halo >= steps.  The
// interior is written with non-temporal stores: nothing in the launch reads it
// again, and streaming it out shortens the cache write-back at the kernel
// boundary.
//
// Zero-Neumann boundary (section 2): where a neighbour lies outside the domain
// the cell itself is used.  The selects exist only in the edge variants: EX
// for tiles that reach x = 0 or x = nx-1 (block-uniform), EY for waves whose
// rows reach y = 0 or y = ny-1 (wave-uniform).  Cells outside the domain are
// loaded from the clamped address, so every load stays in bounds and every
// value stays finite; no exact cell ever reads them.
//
// Every cell is updated by update2d from the same neighbour values as in the
// LDS kernels, so the result is bitwise that of any other 2D plan.
#pragma once

#include "ac_internal.h"

namespace ac {

// DPP controls of the whole-wave shifts by one lane (gfx9 encoding).
constexpr int kDppWaveShr1 = 0x138;   // lane l receives lane l-1
constexpr int kDppWaveShl1 = 0x130;   // lane l receives lane l+1

template <int CTRL>
__device__ __forceinline__ float wave_shift(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xf,
                                                               0xf, true));
}

template <int CTRL>
__device__ __forceinline__ double wave_shift(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)u, CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), CTRL, 0xf, 0xf, true);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// One step of a wave's RCH rows, in place.  hu / hd: the rows just above and
// below the wave's rows (old values).  x: this lane's column; y0: the wave's
// first row.
template <typename T, int RCH, bool EX, bool EY>
__device__ __forceinline__ void reg2d_substep(T v[RCH], T hu, T hd, int x, int nx, int y0, int ny,
                                              T alpha, T r)
{
    const bool atL = EX && x == 0, atR = EX && x == nx - 1;
    T prev = hu;
#pragma unroll
    for (int q = 0; q < RCH; ++q) {
        const T c = v[q];
        T up = prev, dn = q + 1 < RCH ? v[q + 1] : hd;
        T l = wave_shift<kDppWaveShr1>(c), rr = wave_shift<kDppWaveShl1>(c);
        if (EX) {
            l = atL ? c : l;
            rr = atR ? c : rr;
        }
        if (EY) {
            up = y0 + q == 0 ? c : up;
            dn = y0 + q == ny - 1 ? c : dn;
        }
        prev = c;
        v[q] = update2d<T>(c, l, rr, up, dn, alpha, r);
    }
}

// Advance tile (tile_x, tile_y) of one grid by ksteps <= halo steps (any
// number if the tile covers the whole grid).  The workgroup has NW =
// blockDim.x / 64 waves; the tile is 64 x NW*RCH cells including the halo.
// xb: the LDS row exchange, [2 parities][2 rows][NW waves][64 lanes].
template <typename T, int RCH>
__device__ __forceinline__ void reg2d_body(const T *__restrict__ src, T *__restrict__ dst, int nx,
                                           int ny, T alpha, T r, int halo, int ksteps, int tile_x,
                                           int tile_y, T *xb)
{
    const int tx = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int NW = blockDim.x >> 6;
    const int OX = 64 - 2 * halo, OY = NW * RCH - 2 * halo;
    const int ox0 = tile_x * OX, oy0 = tile_y * OY;
    const int lx0 = ox0 - halo;
    const int x = lx0 + tx;
    const int y0 = oy0 - halo + w * RCH;
    const int xc = min(max(x, 0), nx - 1);
    T v[RCH];
#pragma unroll
    for (int q = 0; q < RCH; ++q) {
        const int yc = min(max(y0 + q, 0), ny - 1);
        v[q] = src[(size_t)yc * nx + xc];
    }
    const bool edgeX = lx0 <= 0 || lx0 + 63 >= nx - 1;
    const bool edgeY = y0 <= 0 || y0 + RCH - 1 >= ny - 1;
    for (int s = 0; s < ksteps; ++s) {
        T *b = xb + (s & 1) * 2 * NW * 64;
        b[w * 64 + tx] = v[0];
        b[(NW + w) * 64 + tx] = v[RCH - 1];
        __syncthreads();
        const T hu = w > 0 ? b[(NW + w - 1) * 64 + tx] : v[0];
        const T hd = w + 1 < NW ? b[(w + 1) * 64 + tx] : v[RCH - 1];
        if (edgeX) {
            if (edgeY) reg2d_substep<T, RCH, true, true>(v, hu, hd, x, nx, y0, ny, alpha, r);
            else       reg2d_substep<T, RCH, true, false>(v, hu, hd, x, nx, y0, ny, alpha, r);
        } else {
            if (edgeY) reg2d_substep<T, RCH, false, true>(v, hu, hd, x, nx, y0, ny, alpha, r);
            else       reg2d_substep<T, RCH, false, false>(v, hu, hd, x, nx, y0, ny, alpha, r);
        }
    }
    const int ox1 = min(ox0 + OX, nx), oy1 = min(oy0 + OY, ny);
    if (x >= ox0 && x < ox1) {
#pragma unroll
        for (int q = 0; q < RCH; ++q) {
            const int y = y0 + q;
            if (y >= oy0 && y < oy1) __builtin_nontemporal_store(v[q], dst + (size_t)y * nx + x);
        }
    }
}

}  // namespace ac
