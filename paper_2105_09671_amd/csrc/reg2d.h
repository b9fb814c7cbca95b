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
// Tiling (reg2d_tile_span): along each axis the first tile starts at the
// domain's first cell and, when the domain is longer than a tile, the last
// one ends at its last cell; the tiles between step by L - 2 halo.  So a
// domain edge always falls on a tile edge, and the zero-Neumann boundary
// (section 2: a neighbour outside the domain is the cell itself) costs almost
// nothing:
//   * y: the first row of a tile's first wave, or the last row of its last
//     wave, takes the row itself as its outer neighbour, which is the
//     Neumann value at y = 0 and y = ny-1;
//   * x: at x = 0 (lane 0 of a first tile) and x = nx-1 (lane 63 of a last
//     tile) the DPP shift keeps the lane's own value instead of a neighbour's,
//     one move that cannot fold into the add (10 VALU instructions per cell
//     there against 9).
// Only a domain smaller than one tile (nx < 64, or ny shorter than the tile)
// has cells beyond its edge inside the tile; there the edge variant replaces
// the neighbour by a select.  Cells outside the domain are loaded from the
// clamped address, so every load stays in bounds and every value stays
// finite; no exact cell ever reads them.
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

// The same shift, but the lane with no source lane (lane 0 for a right shift,
// lane 63 for a left one) keeps its own value: the Neumann neighbour of a
// domain edge that sits on the wave's first or last lane.
template <int CTRL>
__device__ __forceinline__ float wave_shift_keep(float v) {
    const int i = __builtin_bit_cast(int, v);
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(i, i, CTRL, 0xf, 0xf, false));
}

template <int CTRL>
__device__ __forceinline__ double wave_shift_keep(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const int l = (int)(unsigned)u, h = (int)(unsigned)(u >> 32);
    const int lo = __builtin_amdgcn_update_dpp(l, l, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(h, h, CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Placement of tile i of nt along an axis of n cells, tiles of L cells with a
// `halo`-wide ring: loaded cells [*ld, *ld + L), exact output [*o0, *o1).
__host__ __device__ inline int reg2d_tiles_1d(int n, int L, int halo) {
    return n <= L ? 1 : 1 + (n - L + (L - 2 * halo) - 1) / (L - 2 * halo);
}

__host__ __device__ inline void reg2d_tile_span(int i, int nt, int n, int L, int halo, int *ld,
                                                int *o0, int *o1) {
    const int O = L - 2 * halo;
    *ld = i == 0 ? 0 : (i == nt - 1 ? n - L : i * O);
    *o0 = i == 0 ? 0 : i * O + halo;
    *o1 = i == nt - 1 ? n : i * O + halo + O;
}

// x-edge handling of a tile: none, its lane 0 is x = 0, its lane 63 is
// x = nx-1, or the domain is narrower than the tile (selects).
enum { REG_X_IN = 0, REG_X_LEFT = 1, REG_X_RIGHT = 2, REG_X_SEL = 3 };

// Row q of one step of a wave's RCH rows, from `in` to `out` (distinct
// registers, so rows can go in any order).  hu / hd: the rows just above and
// below the wave's rows (old values).  x: this lane's column; y0: the wave's
// first row.  EY: the domain ends inside the wave's rows at y = ny-1.
template <typename T, int RCH, int EX, bool EY>
__device__ __forceinline__ void reg2d_row(int q, const T (&in)[RCH], T (&out)[RCH], T hu, T hd,
                                          int x, int nx, int y0, int ny, T alpha, T r)
{
    const T c = in[q];
    const T up = q > 0 ? in[q - 1] : hu;
    T dn = q + 1 < RCH ? in[q + 1] : hd;
    T l = EX == REG_X_LEFT ? wave_shift_keep<kDppWaveShr1>(c) : wave_shift<kDppWaveShr1>(c);
    T rr = EX == REG_X_RIGHT ? wave_shift_keep<kDppWaveShl1>(c) : wave_shift<kDppWaveShl1>(c);
    if (EX == REG_X_SEL) {
        l = x == 0 ? c : l;
        rr = x == nx - 1 ? c : rr;
    }
    if (EY) dn = y0 + q == ny - 1 ? c : dn;
    out[q] = update2d<T>(c, l, rr, up, dn, alpha, r);
}

// One step of all RCH rows of a wave, top to bottom.
template <typename T, int RCH, int EX, bool EY>
__device__ __forceinline__ void reg2d_substep(const T (&in)[RCH], T (&out)[RCH], T hu, T hd, int x,
                                              int nx, int y0, int ny, T alpha, T r)
{
#pragma unroll
    for (int q = 0; q < RCH; ++q) reg2d_row<T, RCH, EX, EY>(q, in, out, hu, hd, x, nx, y0, ny, alpha, r);
}

// The LDS row exchange of a tile: [2 parities][NW waves][first, last row][64
// lanes] (the 128-wide tile's blocks hold four rows).  A lane addresses it
// through `own`, its slot in its wave's block for one parity: the previous
// wave's block sits one block (per_wave values) below, the next wave's one
// above, so every access is an immediate offset from an address the step
// loop keeps (no address arithmetic per step).
template <typename T>
struct RowExchange {
    T *own0, *own1;               // per parity
    const T *prev0, *prev1;       // own - per_wave, or own for the tile's first wave
    bool has_prev, has_next;
    __device__ RowExchange(T *xb, int per_wave) {
        const int tx = threadIdx.x & 63;
        const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const int NW = blockDim.x >> 6;
        has_prev = w > 0;
        has_next = w + 1 < NW;
        own0 = xb + w * per_wave + tx;
        own1 = own0 + NW * per_wave;
        prev0 = has_prev ? own0 - per_wave : own0;
        prev1 = has_prev ? own1 - per_wave : own1;
    }
    // selects, not an indexed array: a runtime parity stays in registers
    __device__ T *own(int p) const { return p ? own1 : own0; }
    __device__ const T *prev(int p) const { return p ? prev1 : prev0; }
};

// One fused step of a tile: publish the wave's first and last row to the row
// exchange (parity p), meet at the barrier, read the neighbours' rows (the
// tile's first and last wave use their own edge rows there: the Neumann
// mirror where the tile edge is the domain edge), step `in` into `out`.
template <typename T, int RCH, int EX, bool EY>
__device__ __forceinline__ void reg2d_step(const T (&in)[RCH], T (&out)[RCH], const RowExchange<T> &xe,
                                           int p, int x, int nx, int y0, int ny, T alpha, T r)
{
    T *own = xe.own(p);
    own[0] = in[0];
    own[64] = in[RCH - 1];
    __syncthreads();
    const T hu = xe.has_prev ? xe.prev(p)[64] : in[0];
    const T hd = xe.has_next ? own[128] : in[RCH - 1];
    reg2d_substep<T, RCH, EX, EY>(in, out, hu, hd, x, nx, y0, ny, alpha, r);
}

// The fused steps of one tile for one x/y edge variant (chosen once per tile,
// so the step loop carries no dispatch).  FP32 takes two steps per trip, v ->
// u -> v: the two register sets alternate and no value is moved.  FP64 steps
// through one spare set and copies back, since a second full set of 16 double
// rows would not fit the 128 VGPRs a 1024-thread workgroup allows.  xb: the
// LDS row exchange, 4 * NW * 64 values.
template <typename T, int RCH, int EX, bool EY>
__device__ __forceinline__ void reg2d_steps(T (&v)[RCH], int x, int nx, int y0, int ny, T alpha, T r,
                                            int ksteps, T *xb)
{
    const RowExchange<T> xe(xb, 128);
    T u[RCH];
    int s = 0;
    if constexpr (sizeof(T) == 4) {
        for (; s + 1 < ksteps; s += 2) {
            reg2d_step<T, RCH, EX, EY>(v, u, xe, 0, x, nx, y0, ny, alpha, r);
            reg2d_step<T, RCH, EX, EY>(u, v, xe, 1, x, nx, y0, ny, alpha, r);
        }
    }
    for (; s < ksteps; ++s) {
        reg2d_step<T, RCH, EX, EY>(v, u, xe, s & 1, x, nx, y0, ny, alpha, r);
#pragma unroll
        for (int q = 0; q < RCH; ++q) v[q] = u[q];
    }
}

template <typename T, int RCH, bool EY>
__device__ __forceinline__ void reg2d_steps_x(int ex, T (&v)[RCH], int x, int nx, int y0, int ny,
                                              T alpha, T r, int ksteps, T *xb)
{
    switch (ex) {
    case REG_X_IN: reg2d_steps<T, RCH, REG_X_IN, EY>(v, x, nx, y0, ny, alpha, r, ksteps, xb); break;
    case REG_X_LEFT: reg2d_steps<T, RCH, REG_X_LEFT, EY>(v, x, nx, y0, ny, alpha, r, ksteps, xb); break;
    case REG_X_RIGHT: reg2d_steps<T, RCH, REG_X_RIGHT, EY>(v, x, nx, y0, ny, alpha, r, ksteps, xb); break;
    default: reg2d_steps<T, RCH, REG_X_SEL, EY>(v, x, nx, y0, ny, alpha, r, ksteps, xb); break;
    }
}

// Advance tile (tile_x, tile_y) of one grid by ksteps <= halo steps (any
// number if the tile covers the whole grid).  The workgroup has NW =
// blockDim.x / 64 waves; the tile is 64 x NW*RCH cells including the halo.
template <typename T, int RCH>
__device__ __forceinline__ void reg2d_body(const T *__restrict__ src, T *__restrict__ dst, int nx,
                                           int ny, T alpha, T r, int halo, int ksteps, int tile_x,
                                           int tile_y, T *xb)
{
    const int tx = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int NW = blockDim.x >> 6;
    const int LY = NW * RCH;
    const int ntx = reg2d_tiles_1d(nx, 64, halo), nty = reg2d_tiles_1d(ny, LY, halo);
    int lx0, ox0, ox1, ly0, oy0, oy1;
    reg2d_tile_span(tile_x, ntx, nx, 64, halo, &lx0, &ox0, &ox1);
    reg2d_tile_span(tile_y, nty, ny, LY, halo, &ly0, &oy0, &oy1);
    const int x = lx0 + tx;
    const int y0 = ly0 + w * RCH;
    const int xc = min(x, nx - 1);
    T v[RCH];
#pragma unroll
    for (int q = 0; q < RCH; ++q) {
        const int yc = min(y0 + q, ny - 1);
        v[q] = src[(size_t)yc * nx + xc];
    }
    // x edges: a domain narrower than the tile needs selects; otherwise the
    // first tile's lane 0 is x = 0 and the last tile's lane 63 is x = nx-1
    // (both for nx = 64 exactly, which takes the select path too)
    const int ex = nx < 64 || (ntx == 1) ? REG_X_SEL
                   : tile_x == 0         ? REG_X_LEFT
                   : tile_x == ntx - 1   ? REG_X_RIGHT
                                         : REG_X_IN;
    // y: a domain shorter than the tile ends inside the wave holding ny-1
    const bool edgeY = ny < LY && y0 <= ny - 1 && y0 + RCH - 1 >= ny - 1;
    if (edgeY) reg2d_steps_x<T, RCH, true>(ex, v, x, nx, y0, ny, alpha, r, ksteps, xb);
    else       reg2d_steps_x<T, RCH, false>(ex, v, x, nx, y0, ny, alpha, r, ksteps, xb);
    if (x >= ox0 && x < ox1) {
#pragma unroll
        for (int q = 0; q < RCH; ++q) {
            const int y = y0 + q;
            if (y >= oy0 && y < oy1) __builtin_nontemporal_store(v[q], dst + (size_t)y * nx + x);
        }
    }
}

}  // namespace ac
