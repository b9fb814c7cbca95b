// Register-resident 3D z-streaming tiles with K time levels pipelined along z
// (gfx950, wave64).
//
// A workgroup of NW waves owns an xy tile 64 cells wide and NW*RCH rows tall,
// including a K-wide halo, and streams it through a segment of z planes.
// Lane l of wave w holds, for each level s < K, column l of its RCH rows of
// two consecutive planes (`prv`, `cur`) in VGPRs; level s+1 of plane p is
// computed as soon as level s of plane p+1 exists, so one pass over the planes
// advances the segment K steps (the scheme of the LDS z-streaming kernel,
// with the planes held in registers instead of LDS):
//   * x neighbours: the same register in lanes l-1 / l+1 (DPP wave shifts);
//   * y neighbours: the lane's own registers, except beyond a wave's first and
//     last row, where they come from the adjacent waves through an LDS
//     exchange of 2 rows x K levels per wave per plane, double-buffered by
//     plane parity so one barrier per plane suffices;
//   * z neighbours: the previous and next plane of the same level, in
//     registers.
// Level-0 planes are loaded PD planes ahead.  Every load uses a clamped
// address; cells outside the domain are never exact and never read by an
// exact cell.
//
// Zero-Neumann boundary (section 2): the xy tiles sit flush against the
// domain edges (reg2d_tile_span), so the x and y edges cost what they cost
// in the 2D register kernel (nothing in y, one DPP move that keeps the lane's
// own value in x; selects only for a domain smaller than one tile); the z
// edges p = 0 and p = nz-1 are a uniform branch per plane and level, so
// interior planes carry no selects.  In-plane offsets are 32-bit (the plan
// requires nx * ny < 2^31).  update3d pairs the neighbour sum per axis, so
// the result is bitwise that of the LDS 3D kernel.
#pragma once

#include <type_traits>

#include "reg2d.h"

namespace ac {

constexpr int kReg3dPD = 2;   // level-0 planes loaded ahead of use

// Level s of plane p for the wave's RCH rows: c = cur (level s-1 of plane p),
// zm = prv (plane p-1), zp = nw (plane p+1), hu / hd the rows beyond the wave.
// EX: x-edge handling as in the 2D register kernel (REG_X_*); EY: the domain
// ends inside the wave's rows at y = ny-1; EZ: plane p is a z edge.
template <typename T, int RCH, int EX, bool EY, bool EZ>
__device__ __forceinline__ void reg3d_level(const T cur[RCH], const T prv[RCH], const T nw[RCH],
                                            T hu, T hd, T res[RCH], int x, int nx, int y0, int ny,
                                            bool zlo, bool zhi, T alpha, T r)
{
    const bool atL = EX == REG_X_SEL && x == 0, atR = EX == REG_X_SEL && x == nx - 1;
#pragma unroll
    for (int q = 0; q < RCH; ++q) {
        const T c = cur[q];
        T up = q > 0 ? cur[q - 1] : hu, dn = q + 1 < RCH ? cur[q + 1] : hd;
        T zm = prv[q], zp = nw[q];
        T l = EX == REG_X_LEFT ? wave_shift_keep<kDppWaveShr1>(c) : wave_shift<kDppWaveShr1>(c);
        T rr = EX == REG_X_RIGHT ? wave_shift_keep<kDppWaveShl1>(c) : wave_shift<kDppWaveShl1>(c);
        if (EX == REG_X_SEL) {
            l = atL ? c : l;
            rr = atR ? c : rr;
        }
        if (EY) dn = y0 + q == ny - 1 ? c : dn;
        if (EZ) {
            zm = zlo ? c : zm;
            zp = zhi ? c : zp;
        }
        res[q] = update3d<T>(c, l, rr, up, dn, zm, zp, alpha, r);
    }
}

// The plane loop of one tile for one x/y edge variant (chosen once per tile,
// so the loop carries no per-level dispatch): K levels pipelined along the z
// segment [oz0, oz1).  xb: the LDS row exchange (below), 4 * K * NW * 64
// values.  SR: how a wave reads the rows beyond its own (below).
template <typename T, int K, int RCH, int EX, bool EY, bool SR>
__device__ __forceinline__ void reg3d_stream(const T *__restrict__ src, T *__restrict__ dst, int nx,
                                             int ny, int nz, T alpha, T r, int x, int y0, bool xout,
                                             int oy0, int oy1, int oz0, int oz1,
                                             const int (&gxy)[RCH], T *xb)
{
    constexpr int PD = kReg3dPD;
    const int tx = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int NW = blockDim.x >> 6;
    const size_t pstride = (size_t)nx * ny;
    T cur[K][RCH], prv[K][RCH], pf[PD][RCH];
#pragma unroll
    for (int s = 0; s < K; ++s)
#pragma unroll
        for (int q = 0; q < RCH; ++q) cur[s][q] = prv[s][q] = T(0);

    const int t0 = max(oz0 - K, 0);
    const int t1 = oz1 - 1 + K;           // last iteration: level K emits plane oz1-1
#pragma unroll
    for (int d = 0; d < PD; ++d) {
        const size_t zo = (size_t)min(t0 + d, nz - 1) * pstride;
#pragma unroll
        for (int q = 0; q < RCH; ++q) pf[d][q] = src[zo + gxy[q]];
    }
    // the row exchange.  SR: [2 parities][NW waves][K levels][first, last
    // row][64 lanes], and per parity a lane keeps three addresses, so that
    // every access is an immediate offset: `own` (its slot in its wave's
    // block), `up` (row 2s of it is the row above the wave at level s: the
    // previous wave's last row, or for the tile's first wave its own first
    // row, the Neumann mirror at a domain edge) and `dn` (row 2s: the next
    // wave's first row, or the last wave's own last row).  Else [2 parities]
    // [K levels][first, last row][NW waves][64 lanes], addressed per access
    // (measured at 1024^3, where this variant runs: 9 % faster than the
    // per-wave blocks there, which gain 2-3 % at 256^3 and 512^3 and 25 % in
    // FP64 at 256^3)
    constexpr int BS = 2 * K * 64;                      // one wave's block
    T *own0 = xb + w * BS + tx, *own1 = own0 + NW * BS;
    const T *up0 = w > 0 ? own0 - BS + 64 : own0, *up1 = w > 0 ? own1 - BS + 64 : own1;
    const T *dn0 = w + 1 < NW ? own0 + BS : own0 + 64, *dn1 = w + 1 < NW ? own1 + BS : own1 + 64;
    const int row = NW * 64;                            // one exchanged row of all waves
    // one pass over plane t; ZC: some level of this iteration may sit on a z
    // edge (then each level tests its plane), else no level does
    auto iteration = [&](int t, auto zc) {
        constexpr bool ZC = decltype(zc)::value;
        const bool odd = t & 1;
        T *own = odd ? own1 : own0;
        const T *up = odd ? up1 : up0, *dn = odd ? dn1 : dn0;
        T *b = xb + (size_t)(t & 1) * K * 2 * row;
        // publish the wave's edge rows of every level (level s: plane t-1-s)
#pragma unroll
        for (int s = 0; s < K; ++s) {
            if constexpr (SR) {
                own[(2 * s) * 64] = cur[s][0];
                own[(2 * s + 1) * 64] = cur[s][RCH - 1];
            } else {
                b[(2 * s) * row + w * 64 + tx] = cur[s][0];
                b[(2 * s + 1) * row + w * 64 + tx] = cur[s][RCH - 1];
            }
        }
        T nw[RCH];
#pragma unroll
        for (int q = 0; q < RCH; ++q) nw[q] = pf[0][q];
#pragma unroll
        for (int d = 0; d + 1 < PD; ++d)
#pragma unroll
            for (int q = 0; q < RCH; ++q) pf[d][q] = pf[d + 1][q];
        {
            const size_t zo = (size_t)min(t + PD, nz - 1) * pstride;
#pragma unroll
            for (int q = 0; q < RCH; ++q) pf[PD - 1][q] = src[zo + gxy[q]];
        }
        __syncthreads();
#pragma unroll
        for (int s = 1; s <= K; ++s) {
            const int p = t - s;                        // plane advanced to level s
            // the rows beyond the wave; the tile's first (last) wave uses its
            // own first (last) row there, the Neumann mirror at a domain edge.
            // SR: it reads it back from the exchange at a selected address, so
            // no branch splits the iteration and the cross-lane shifts can
            // fold into adds; else it takes the value under a branch, which
            // lets the compiler start the shifts while the reads are in flight
            T hu, hd;
            if constexpr (SR) {
                hu = up[(2 * (s - 1)) * 64];
                hd = dn[(2 * (s - 1)) * 64];
            } else {
                hu = w > 0 ? b[(2 * (s - 1) + 1) * row + (w - 1) * 64 + tx] : cur[s - 1][0];
                hd = w + 1 < NW ? b[(2 * (s - 1)) * row + (w + 1) * 64 + tx] : cur[s - 1][RCH - 1];
            }
            T res[RCH];
            if constexpr (ZC) {
                const bool zlo = p == 0, zhi = p == nz - 1;
                if (zlo || zhi)
                    reg3d_level<T, RCH, EX, EY, true>(cur[s - 1], prv[s - 1], nw, hu, hd, res, x,
                                                      nx, y0, ny, zlo, zhi, alpha, r);
                else
                    reg3d_level<T, RCH, EX, EY, false>(cur[s - 1], prv[s - 1], nw, hu, hd, res, x,
                                                       nx, y0, ny, false, false, alpha, r);
            } else {
                reg3d_level<T, RCH, EX, EY, false>(cur[s - 1], prv[s - 1], nw, hu, hd, res, x, nx,
                                                   y0, ny, false, false, alpha, r);
            }
#pragma unroll
            for (int q = 0; q < RCH; ++q) {
                prv[s - 1][q] = cur[s - 1][q];
                cur[s - 1][q] = nw[q];
                nw[q] = res[q];
            }
        }
        const int pout = t - K;
        if (pout >= oz0 && pout < oz1 && xout) {
#pragma unroll
            for (int q = 0; q < RCH; ++q) {
                const int y = y0 + q;
                if (y >= oy0 && y < oy1) dst[(size_t)pout * pstride + (size_t)y * nx + x] = nw[q];
            }
        }
    };
    // iterations t in [K+1, nz-1] advance only planes 1 .. nz-2: no z edge, so
    // the middle loop carries no branch; the few iterations before and after
    // it test each level's plane
    const int fa = max(t0, K + 1), fb = min(t1, nz - 1);
    const int e1 = min(t1, fa - 1);
    for (int t = t0; t <= e1; ++t) iteration(t, std::true_type{});
    int t = fa;
    // three iterations per trip: the (prv, cur, incoming) rotation of every
    // level then returns to the same registers, so it costs no moves
    for (; t + 2 <= fb; t += 3) {
        iteration(t, std::false_type{});
        iteration(t + 1, std::false_type{});
        iteration(t + 2, std::false_type{});
    }
    for (; t <= fb; ++t) iteration(t, std::false_type{});
    for (int t = max(fb + 1, fa); t <= t1; ++t) iteration(t, std::true_type{});
}

template <typename T, int K, int RCH, bool EY, bool SR>
__device__ __forceinline__ void reg3d_stream_x(int ex, const T *__restrict__ src, T *__restrict__ dst,
                                               int nx, int ny, int nz, T alpha, T r, int x, int y0,
                                               bool xout, int oy0, int oy1, int oz0, int oz1,
                                               const int (&gxy)[RCH], T *xb)
{
    switch (ex) {
    case REG_X_IN:
        reg3d_stream<T, K, RCH, REG_X_IN, EY, SR>(src, dst, nx, ny, nz, alpha, r, x, y0, xout, oy0, oy1,
                                              oz0, oz1, gxy, xb);
        break;
    case REG_X_LEFT:
        reg3d_stream<T, K, RCH, REG_X_LEFT, EY, SR>(src, dst, nx, ny, nz, alpha, r, x, y0, xout, oy0,
                                                oy1, oz0, oz1, gxy, xb);
        break;
    case REG_X_RIGHT:
        reg3d_stream<T, K, RCH, REG_X_RIGHT, EY, SR>(src, dst, nx, ny, nz, alpha, r, x, y0, xout, oy0,
                                                 oy1, oz0, oz1, gxy, xb);
        break;
    default:
        reg3d_stream<T, K, RCH, REG_X_SEL, EY, SR>(src, dst, nx, ny, nz, alpha, r, x, y0, xout, oy0,
                                               oy1, oz0, oz1, gxy, xb);
        break;
    }
}

// Advance xy tile `tile` (row-major over tiles_x columns) of z segment `zseg`
// (LZ planes) by K steps.  xb: the LDS row exchange of reg3d_stream.
template <typename T, int K, int RCH, bool SR>
__device__ __forceinline__ void reg3d_body(const T *__restrict__ src, T *__restrict__ dst, int nx,
                                           int ny, int nz, T alpha, T r, int LZ, int tiles_x,
                                           int tile, int zseg, T *xb)
{
    const int tx = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int NW = blockDim.x >> 6;
    const int LY = NW * RCH;
    // xy tiles sit flush against the domain edges as in the 2D register kernel
    const int tile_x = tile % tiles_x, tile_y = tile / tiles_x;
    const int nty = reg2d_tiles_1d(ny, LY, K);
    int lx0, ox0, ox1, ly0, oy0, oy1;
    reg2d_tile_span(tile_x, tiles_x, nx, 64, K, &lx0, &ox0, &ox1);
    reg2d_tile_span(tile_y, nty, ny, LY, K, &ly0, &oy0, &oy1);
    const int oz0 = zseg * LZ, oz1 = min(oz0 + LZ, nz);
    const int x = lx0 + tx;
    const int y0 = ly0 + w * RCH;
    const int xc = min(x, nx - 1);
    const int ex = nx < 64 || tiles_x == 1 ? REG_X_SEL
                   : tile_x == 0           ? REG_X_LEFT
                   : tile_x == tiles_x - 1 ? REG_X_RIGHT
                                           : REG_X_IN;
    const bool edgeY = ny < LY && y0 <= ny - 1 && y0 + RCH - 1 >= ny - 1;
    const bool xout = x >= ox0 && x < ox1;
    int gxy[RCH];
#pragma unroll
    for (int q = 0; q < RCH; ++q) gxy[q] = min(y0 + q, ny - 1) * nx + xc;
    if (edgeY)
        reg3d_stream_x<T, K, RCH, true, SR>(ex, src, dst, nx, ny, nz, alpha, r, x, y0, xout, oy0, oy1,
                                        oz0, oz1, gxy, xb);
    else
        reg3d_stream_x<T, K, RCH, false, SR>(ex, src, dst, nx, ny, nz, alpha, r, x, y0, xout, oy0, oy1,
                                         oz0, oz1, gxy, xb);
}

}  // namespace ac
