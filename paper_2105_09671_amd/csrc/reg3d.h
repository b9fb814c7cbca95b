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
// Zero-Neumann boundary (section 2): x and y edges as in the 2D register
// kernel (EX block-uniform, EY wave-uniform variants); the z edges p = 0 and
// p = nz-1 are a uniform branch per plane and level, so interior planes carry
// no selects.  update3d pairs the neighbour sum per axis, so the result is
// bitwise that of the LDS 3D kernel.
#pragma once

#include "reg2d.h"

namespace ac {

constexpr int kReg3dPD = 2;   // level-0 planes loaded ahead of use

// Level s of plane p for the wave's RCH rows: c = cur (level s-1 of plane p),
// zm = prv (plane p-1), zp = nw (plane p+1), hu / hd the rows beyond the wave.
template <typename T, int RCH, bool EX, bool EY, bool EZ>
__device__ __forceinline__ void reg3d_level(const T cur[RCH], const T prv[RCH], const T nw[RCH],
                                            T hu, T hd, T res[RCH], int x, int nx, int y0, int ny,
                                            bool zlo, bool zhi, T alpha, T r)
{
    const bool atL = EX && x == 0, atR = EX && x == nx - 1;
#pragma unroll
    for (int q = 0; q < RCH; ++q) {
        const T c = cur[q];
        T up = q > 0 ? cur[q - 1] : hu, dn = q + 1 < RCH ? cur[q + 1] : hd;
        T zm = prv[q], zp = nw[q];
        T l = wave_shift<kDppWaveShr1>(c), rr = wave_shift<kDppWaveShl1>(c);
        if (EX) {
            l = atL ? c : l;
            rr = atR ? c : rr;
        }
        if (EY) {
            up = y0 + q == 0 ? c : up;
            dn = y0 + q == ny - 1 ? c : dn;
        }
        if (EZ) {
            zm = zlo ? c : zm;
            zp = zhi ? c : zp;
        }
        res[q] = update3d<T>(c, l, rr, up, dn, zm, zp, alpha, r);
    }
}

// Advance xy tile `tile` (row-major over tiles_x columns) of z segment `zseg`
// (LZ planes) by K steps.  xb: LDS exchange, [2 parities][K levels][2 rows]
// [NW waves][64 lanes].
template <typename T, int K, int RCH>
__device__ __forceinline__ void reg3d_body(const T *__restrict__ src, T *__restrict__ dst, int nx,
                                           int ny, int nz, T alpha, T r, int LZ, int tiles_x,
                                           int tile, int zseg, T *xb)
{
    constexpr int PD = kReg3dPD;
    const int tx = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int NW = blockDim.x >> 6;
    const int OX = 64 - 2 * K, OY = NW * RCH - 2 * K;
    const int ox0 = (tile % tiles_x) * OX, oy0 = (tile / tiles_x) * OY;
    const int ox1 = min(ox0 + OX, nx), oy1 = min(oy0 + OY, ny);
    const int oz0 = zseg * LZ, oz1 = min(oz0 + LZ, nz);
    const int lx0 = ox0 - K;
    const int x = lx0 + tx;
    const int y0 = oy0 - K + w * RCH;
    const int xc = min(max(x, 0), nx - 1);
    const bool edgeX = lx0 <= 0 || lx0 + 63 >= nx - 1;
    const bool edgeY = y0 <= 0 || y0 + RCH - 1 >= ny - 1;
    const bool xout = x >= ox0 && x < ox1;
    const size_t pstride = (size_t)nx * ny;
    int gxy[RCH];
#pragma unroll
    for (int q = 0; q < RCH; ++q) gxy[q] = min(max(y0 + q, 0), ny - 1) * nx + xc;

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
    const int row = NW * 64;                            // one exchanged row of all waves
    for (int t = t0; t <= t1; ++t) {
        T *b = xb + (size_t)(t & 1) * K * 2 * row;
        // publish the wave's edge rows of every level (level s: plane t-1-s)
#pragma unroll
        for (int s = 0; s < K; ++s) {
            b[(2 * s) * row + w * 64 + tx] = cur[s][0];
            b[(2 * s + 1) * row + w * 64 + tx] = cur[s][RCH - 1];
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
            const T hu = w > 0 ? b[(2 * (s - 1) + 1) * row + (w - 1) * 64 + tx] : cur[s - 1][0];
            const T hd = w + 1 < NW ? b[(2 * (s - 1)) * row + (w + 1) * 64 + tx]
                                    : cur[s - 1][RCH - 1];
            const bool zlo = p == 0, zhi = p == nz - 1;
            T res[RCH];
#define AC_REG3D_LEVEL(EX_, EY_)                                                                   \
    if (zlo || zhi)                                                                                \
        reg3d_level<T, RCH, EX_, EY_, true>(cur[s - 1], prv[s - 1], nw, hu, hd, res, x, nx, y0,    \
                                            ny, zlo, zhi, alpha, r);                               \
    else                                                                                           \
        reg3d_level<T, RCH, EX_, EY_, false>(cur[s - 1], prv[s - 1], nw, hu, hd, res, x, nx, y0,   \
                                             ny, false, false, alpha, r);
            if (edgeX) {
                if (edgeY) { AC_REG3D_LEVEL(true, true) } else { AC_REG3D_LEVEL(true, false) }
            } else {
                if (edgeY) { AC_REG3D_LEVEL(false, true) } else { AC_REG3D_LEVEL(false, false) }
            }
#undef AC_REG3D_LEVEL
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
    }
}

}  // namespace ac
