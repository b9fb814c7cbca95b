// 2D Allen-Cahn register tiles two columns wide per lane: 128-wide tiles on
// gfx950 wave64, temporal blocking as in reg2d.h (section 2.1 update,
// zero-Neumann edges of section 2).
//
// Lane l of a wave holds columns x0 + 2l (`a`) and x0 + 2l + 1 (`b`) of RCH
// consecutive rows.  The x neighbours of a are lane l-1's b and the lane's own
// b; those of b are its own a and lane l+1's a.  So a cell needs one
// cross-lane shift instead of two, and the shift folds into the add of the
// neighbour pair: one VALU operation per cell less than the 64-wide tile, and
// the 128-wide tile loses half as large a share of its columns to the halo.
//
// The y direction (waves stacked along y, edge rows exchanged through LDS with
// one barrier per step), the flush tile placement and the update itself are
// those of reg2d.h, so both tiles round identically.  The tile needs nx >= 128
// (every column it loads lies in the domain); narrower domains take the
// 64-wide tile.
#pragma once

#include <cstdint>

#include "reg2d.h"

namespace ac {

// Whole-wave shift by one lane whose lane without a source lane (lane 0 for a
// right shift, lane 63 for a left one) takes `old` instead.
template <int CTRL>
__device__ __forceinline__ float wave_shift_or(float src, float old) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old),
                                                                  __builtin_bit_cast(int, src), CTRL,
                                                                  0xf, 0xf, false));
}

template <int CTRL>
__device__ __forceinline__ double wave_shift_or(double src, double old) {
    const unsigned long long s = __builtin_bit_cast(unsigned long long, src);
    const unsigned long long o = __builtin_bit_cast(unsigned long long, old);
    const int lo = __builtin_amdgcn_update_dpp((int)(unsigned)o, (int)(unsigned)s, CTRL, 0xf, 0xf,
                                               false);
    const int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(o >> 32), (int)(unsigned)(s >> 32),
                                               CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// x edges of a wide tile: REG_X_IN, REG_X_LEFT (lane 0's a is x = 0),
// REG_X_RIGHT (lane 63's b is x = nx-1) or REG_X_SEL (both: the tile spans
// the whole width).
template <typename T, int RCH, int EX, bool EY>
__device__ __forceinline__ void reg2w_row(int q, const T (&ia)[RCH], const T (&ib)[RCH],
                                          T (&oa)[RCH], T (&ob)[RCH], T hua, T hub, T hda, T hdb,
                                          int y0, int ny, T alpha, T r)
{
    constexpr bool keepL = EX == REG_X_LEFT || EX == REG_X_SEL;
    constexpr bool keepR = EX == REG_X_RIGHT || EX == REG_X_SEL;
    const T a = ia[q], b = ib[q];
    const T ua = q > 0 ? ia[q - 1] : hua, ub = q > 0 ? ib[q - 1] : hub;
    T da = q + 1 < RCH ? ia[q + 1] : hda, db = q + 1 < RCH ? ib[q + 1] : hdb;
    // Neumann at x = 0 / nx-1: the missing neighbour is the cell itself
    const T al = keepL ? wave_shift_or<kDppWaveShr1>(b, a) : wave_shift<kDppWaveShr1>(b);
    const T br = keepR ? wave_shift_or<kDppWaveShl1>(a, b) : wave_shift<kDppWaveShl1>(a);
    if (EY) {
        const bool last = y0 + q == ny - 1;
        da = last ? a : da;
        db = last ? b : db;
    }
    oa[q] = update2d<T>(a, al, b, ua, da, alpha, r);
    ob[q] = update2d<T>(b, a, br, ub, db, alpha, r);
}

// One fused step of a wide tile, (ia, ib) -> (oa, ob): publish the wave's
// first and last rows to the row exchange (reg2d.h's RowExchange with blocks
// of four rows: first a, first b, last a, last b; parity p), meet at the
// barrier, read the rows next to the wave's own (the tile's first and last
// wave use their own edge rows there: the Neumann mirror where the tile edge
// is the domain edge), step every row.
template <typename T, int RCH, int EX, bool EY>
__device__ __forceinline__ void reg2w_step(const T (&ia)[RCH], const T (&ib)[RCH], T (&oa)[RCH],
                                           T (&ob)[RCH], const RowExchange<T> &xe, int p, int y0,
                                           int ny, T alpha, T r)
{
    T *own = xe.own(p);
    own[0] = ia[0];
    own[64] = ib[0];
    own[128] = ia[RCH - 1];
    own[192] = ib[RCH - 1];
    __syncthreads();
    T hua = ia[0], hub = ib[0], hda = ia[RCH - 1], hdb = ib[RCH - 1];
    if (xe.has_prev) {
        hua = xe.prev(p)[128];
        hub = xe.prev(p)[192];
    }
    if (xe.has_next) {
        hda = own[256];
        hdb = own[320];
    }
#pragma unroll
    for (int q = 0; q < RCH; ++q)
        reg2w_row<T, RCH, EX, EY>(q, ia, ib, oa, ob, hua, hub, hda, hdb, y0, ny, alpha, r);
}

// The fused steps of one wide tile for one edge variant, two per trip so the
// two register sets alternate and no value is moved.  xb: the row exchange,
// 8 * NW * 64 values.
template <typename T, int RCH, int EX, bool EY>
__device__ __forceinline__ void reg2w_steps(T (&va)[RCH], T (&vb)[RCH], int y0, int ny, T alpha,
                                            T r, int ksteps, T *xb)
{
    const RowExchange<T> xe(xb, 256);
    T ua[RCH], ub[RCH];
    int s = 0;
    for (; s + 1 < ksteps; s += 2) {
        reg2w_step<T, RCH, EX, EY>(va, vb, ua, ub, xe, 0, y0, ny, alpha, r);
        reg2w_step<T, RCH, EX, EY>(ua, ub, va, vb, xe, 1, y0, ny, alpha, r);
    }
    if (s < ksteps) {
        // the last step follows an odd one (or is the only step)
        reg2w_step<T, RCH, EX, EY>(va, vb, ua, ub, xe, 0, y0, ny, alpha, r);
#pragma unroll
        for (int q = 0; q < RCH; ++q) {
            va[q] = ua[q];
            vb[q] = ub[q];
        }
    }
}

template <typename T, int RCH, bool EY>
__device__ __forceinline__ void reg2w_steps_x(int ex, T (&va)[RCH], T (&vb)[RCH], int y0, int ny,
                                              T alpha, T r, int ksteps, T *xb)
{
    switch (ex) {
    case REG_X_IN: reg2w_steps<T, RCH, REG_X_IN, EY>(va, vb, y0, ny, alpha, r, ksteps, xb); break;
    case REG_X_LEFT: reg2w_steps<T, RCH, REG_X_LEFT, EY>(va, vb, y0, ny, alpha, r, ksteps, xb); break;
    case REG_X_RIGHT: reg2w_steps<T, RCH, REG_X_RIGHT, EY>(va, vb, y0, ny, alpha, r, ksteps, xb); break;
    default: reg2w_steps<T, RCH, REG_X_SEL, EY>(va, vb, y0, ny, alpha, r, ksteps, xb); break;
    }
}

// Advance wide tile (tile_x, tile_y) of one grid by ksteps <= halo steps
// (src -> dst, exact output region only).  nx >= 128.  Rows beyond ny-1 (a
// domain shorter than the tile) load row ny-1 and are never stored.  Rows go
// in and out as pairs of adjacent values when nx and both pointers allow it
// (every pair then starts at an even column: tiles start at multiples of
// 128 - 2*halo or at nx - 128).
template <typename T, int RCH>
__device__ __forceinline__ void reg2w_body(const T *__restrict__ src, T *__restrict__ dst, int nx,
                                           int ny, T alpha, T r, int halo, int ksteps, int tile_x,
                                           int tile_y, T *xb)
{
    typedef T T2 __attribute__((ext_vector_type(2)));
    const int tx = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int NW = blockDim.x >> 6;
    const int LY = NW * RCH;
    const int ntx = reg2d_tiles_1d(nx, 128, halo), nty = reg2d_tiles_1d(ny, LY, halo);
    int lx0, ox0, ox1, ly0, oy0, oy1;
    reg2d_tile_span(tile_x, ntx, nx, 128, halo, &lx0, &ox0, &ox1);
    reg2d_tile_span(tile_y, nty, ny, LY, halo, &ly0, &oy0, &oy1);
    const int xa = lx0 + 2 * tx;
    const int y0 = ly0 + w * RCH;
    const bool pairs = (nx & 1) == 0 && ((reinterpret_cast<uintptr_t>(src) |
                                          reinterpret_cast<uintptr_t>(dst)) & (sizeof(T2) - 1)) == 0;
    T va[RCH], vb[RCH];
    if (pairs) {
#pragma unroll
        for (int q = 0; q < RCH; ++q) {
            const int yc = min(y0 + q, ny - 1);
            const T2 p = *reinterpret_cast<const T2 *>(src + (size_t)yc * nx + xa);
            va[q] = p.x;
            vb[q] = p.y;
        }
    } else {
#pragma unroll
        for (int q = 0; q < RCH; ++q) {
            const int yc = min(y0 + q, ny - 1);
            va[q] = src[(size_t)yc * nx + xa];
            vb[q] = src[(size_t)yc * nx + xa + 1];
        }
    }
    const int ex = ntx == 1         ? REG_X_SEL
                   : tile_x == 0       ? REG_X_LEFT
                   : tile_x == ntx - 1 ? REG_X_RIGHT
                                       : REG_X_IN;
    const bool edgeY = ny < LY && y0 <= ny - 1 && y0 + RCH - 1 >= ny - 1;
    if (edgeY) reg2w_steps_x<T, RCH, true>(ex, va, vb, y0, ny, alpha, r, ksteps, xb);
    else       reg2w_steps_x<T, RCH, false>(ex, va, vb, y0, ny, alpha, r, ksteps, xb);
    const bool ina = xa >= ox0 && xa < ox1, inb = xa + 1 >= ox0 && xa + 1 < ox1;
#pragma unroll
    for (int q = 0; q < RCH; ++q) {
        const int y = y0 + q;
        if (y < oy0 || y >= oy1) continue;
        T *row = dst + (size_t)y * nx + xa;
        if (pairs && ina && inb) {
            T2 p;
            p.x = va[q];
            p.y = vb[q];
            __builtin_nontemporal_store(p, reinterpret_cast<T2 *>(row));
        } else {
            if (ina) __builtin_nontemporal_store(va[q], row);
            if (inb) __builtin_nontemporal_store(vb[q], row + 1);
        }
    }
}

}  // namespace ac
