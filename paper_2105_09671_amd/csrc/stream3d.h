// Device code of the 3D z-streaming tile: shared by the single-grid kernel and
// the batched persistent kernel.  Algorithm notes are in stencil3d.hip.
#pragma once

#include "ac_internal.h"

namespace ac {

constexpr int PD = 4;   // level-0 planes prefetched ahead of use

// Advance xy tile `tile` (row-major over tiles_x columns) of z segment `zseg`
// by K steps; the whole workgroup participates.  smem holds 2 K LX LY values.
template <typename T, int K, int CPT>
__device__ __forceinline__ void stream3d_body(const T *__restrict__ src, T *__restrict__ dst, int nx,
                                              int ny, int nz, T alpha, T r, int LX, int LY, int LZ,
                                              int tiles_x, int tile, int zseg,
                                              unsigned char *smem_raw)
{
    T *slots = reinterpret_cast<T *>(smem_raw);        // [2][K][LX*LY]
    const int NT = blockDim.x;
    const int plane_l = LX * LY;

    const int OX = LX - 2 * K, OY = LY - 2 * K;
    const int ox0 = (tile % tiles_x) * OX, oy0 = (tile / tiles_x) * OY;
    const int ox1 = min(ox0 + OX, nx), oy1 = min(oy0 + OY, ny);
    const int oz0 = zseg * LZ, oz1 = min(oz0 + LZ, nz);
    const int lx0 = ox0 - K, ly0 = oy0 - K;

    // per owned cell: LDS index, neighbour offsets (Neumann folded), global index
    int li[CPT], oxm[CPT], oxp[CPT], oym[CPT], oyp[CPT];
    long gxy[CPT];
    bool ow[CPT], ld[CPT], st[CPT];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int l = threadIdx.x + j * NT;
        const bool own = l < plane_l;
        const int lx = own ? l % LX : 0, ly = own ? l / LX : 0;
        const int gx = lx0 + lx, gy = ly0 + ly;
        const bool in = own && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        li[j] = own ? l : 0;
        ow[j] = own;
        // a neighbour outside the domain (Neumann) or outside the tile
        // (inexact cell, value unused) reads the cell itself
        oxm[j] = (gx > 0 && lx > 0) ? -1 : 0;
        oxp[j] = (gx < nx - 1 && lx < LX - 1) ? 1 : 0;
        oym[j] = (gy > 0 && ly > 0) ? -LX : 0;
        oyp[j] = (gy < ny - 1 && ly < LY - 1) ? LX : 0;
        ld[j] = in;
        st[j] = in && gx >= ox0 && gx < ox1 && gy >= oy0 && gy < oy1;
        gxy[j] = in ? (long)gy * nx + gx : 0;
    }

    T cur[K][CPT], prv[K][CPT], pf[PD][CPT];   // pf: level-0 planes t .. t+PD-1 in flight
#pragma unroll
    for (int s = 0; s < K; ++s)
#pragma unroll
        for (int j = 0; j < CPT; ++j) { cur[s][j] = T(0); prv[s][j] = T(0); }

    const long pstride = (long)nx * ny;
    const int t0 = max(oz0 - K, 0);
    const int t1 = oz1 - 1 + K;           // last iteration: level K emits plane oz1-1

#pragma unroll
    for (int d = 0; d < PD; ++d)
#pragma unroll
        for (int j = 0; j < CPT; ++j)
            pf[d][j] = (ld[j] && t0 + d < nz) ? src[(long)(t0 + d) * pstride + gxy[j]] : T(0);

    for (int t = t0; t <= t1; ++t) {
        T *set = slots + (size_t)(t & 1) * K * plane_l;
        // publish the planes produced in iteration t-1 (level s: plane t-1-s)
#pragma unroll
        for (int s = 0; s < K; ++s)
#pragma unroll
            for (int j = 0; j < CPT; ++j)
                if (ow[j]) set[s * plane_l + li[j]] = cur[s][j];

        T nw[CPT];
#pragma unroll
        for (int j = 0; j < CPT; ++j) nw[j] = pf[0][j];
        // keep PD planes of level 0 in flight
#pragma unroll
        for (int d = 0; d + 1 < PD; ++d)
#pragma unroll
            for (int j = 0; j < CPT; ++j) pf[d][j] = pf[d + 1][j];
#pragma unroll
        for (int j = 0; j < CPT; ++j)
            pf[PD - 1][j] = (ld[j] && t + PD < nz) ? src[(long)(t + PD) * pstride + gxy[j]] : T(0);
        __syncthreads();

#pragma unroll
        for (int s = 1; s <= K; ++s) {
            const int p = t - s;              // plane advanced to level s
            const T *pl = set + (s - 1) * plane_l;
            T res[CPT];
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                const T c = cur[s - 1][j];
                const T zp = (p == nz - 1) ? c : nw[j];
                const T zm = (p == 0) ? c : prv[s - 1][j];
                const int i = li[j];
                res[j] = update3d<T>(c, pl[i + oxm[j]], pl[i + oxp[j]], pl[i + oym[j]],
                                     pl[i + oyp[j]], zm, zp, alpha, r);
            }
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                prv[s - 1][j] = cur[s - 1][j];
                cur[s - 1][j] = nw[j];
                nw[j] = res[j];
            }
        }
        const int pout = t - K;
        if (pout >= oz0 && pout < oz1) {
#pragma unroll
            for (int j = 0; j < CPT; ++j)
                if (st[j]) dst[(long)pout * pstride + gxy[j]] = nw[j];
        }
    }
}

}  // namespace ac
