// 3D Allen-Cahn 7-point stencil, streamed along z with K time levels
// pipelined in one pass (temporal blocking, gfx950 wave64).
//
// A workgroup owns an (LX - 2K) x (LY - 2K) column of output cells over the z
// segment [oz0, oz0 + LZ).  It streams planes t = oz0-K, oz0-K+1, ... through
// the kernel.  At iteration t, level 0 is plane t read from HBM, and level s
// (1 <= s <= K) advances plane t-s from time level s-1 to s.  The z
// neighbours of a level-s update come from registers (each thread keeps, per
// level, the last two planes of every cell it owns); the x/y neighbours come
// from an LDS copy of the level s-1 plane produced in the previous iteration.
// The level-K plane t-K is the output and goes back to HBM.  HBM traffic is
// therefore one read and one write per cell per K time steps, plus the halo.
//
// Level s is exact on the loaded tile shrunk by s cells on each side that is
// not a domain edge (and for planes at least s above the segment's first
// loaded plane, unless that is the domain bottom), so the level-K output tile
// is exact.  Cells outside the exact region compute values nobody reads.
//
// Zero-Neumann boundary (section 2): neighbour indices that fall outside the
// domain are replaced by the cell itself, in x, y and z, at every level.
//
// LDS holds two sets (even/odd iteration) of K planes of LX*LY values so one
// barrier per iteration separates producers from consumers.
#include "ac_internal.h"

namespace ac {

constexpr int PD = 4;   // level-0 planes prefetched ahead of use

template <typename T, int K, int CPT>
__global__ void __launch_bounds__(512)
stream3d_kernel(const T *__restrict__ src, T *__restrict__ dst, int nx, int ny, int nz,
                T alpha, T r, int LX, int LY, int LZ, int tiles_x)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *slots = reinterpret_cast<T *>(smem_raw);        // [2][K][LX*LY]
    const int NT = blockDim.x;
    const int plane_l = LX * LY;

    const int OX = LX - 2 * K, OY = LY - 2 * K;
    const int tile = blockIdx.x;
    const int ox0 = (tile % tiles_x) * OX, oy0 = (tile / tiles_x) * OY;
    const int ox1 = min(ox0 + OX, nx), oy1 = min(oy0 + OY, ny);
    const int oz0 = blockIdx.y * LZ, oz1 = min(oz0 + LZ, nz);
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

size_t stream3d_lds_bytes(const Tile3D &t, size_t elem) {
    return 2 * (size_t)t.K * t.LX * t.LY * elem;
}

int stream3d_cells_per_thread(const Tile3D &t) {
    return (t.LX * t.LY + t.threads - 1) / t.threads;
}

template <typename T, int K, int CPT>
static hipError_t launch3(const T *src, T *dst, int nx, int ny, int nz, T alpha, T r,
                          const Tile3D &t, hipStream_t stream)
{
    const int OX = t.LX - 2 * K, OY = t.LY - 2 * K;
    const int tiles_x = (nx + OX - 1) / OX, tiles_y = (ny + OY - 1) / OY;
    dim3 grid(tiles_x * tiles_y, (nz + t.LZ - 1) / t.LZ);
    const size_t lds = stream3d_lds_bytes(t, sizeof(T));
    set_lds_limit((const void *)stream3d_kernel<T, K, CPT>, lds);
    hipLaunchKernelGGL((stream3d_kernel<T, K, CPT>), grid, dim3(t.threads), lds, stream,
                       src, dst, nx, ny, nz, alpha, r, t.LX, t.LY, t.LZ, tiles_x);
    return hipGetLastError();
}

template <typename T, int K>
static hipError_t launch3_cpt(const T *src, T *dst, int nx, int ny, int nz, T alpha, T r,
                              const Tile3D &t, hipStream_t stream)
{
    const int cpt = stream3d_cells_per_thread(t);
    if (cpt <= 1) return launch3<T, K, 1>(src, dst, nx, ny, nz, alpha, r, t, stream);
    if (cpt <= 2) return launch3<T, K, 2>(src, dst, nx, ny, nz, alpha, r, t, stream);
    if (cpt <= 4) return launch3<T, K, 4>(src, dst, nx, ny, nz, alpha, r, t, stream);
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_stream3d(const T *src, T *dst, int nx, int ny, int nz, T alpha, T r,
                           const Tile3D &t, hipStream_t stream)
{
    switch (t.K) {
    case 1: return launch3_cpt<T, 1>(src, dst, nx, ny, nz, alpha, r, t, stream);
    case 2: return launch3_cpt<T, 2>(src, dst, nx, ny, nz, alpha, r, t, stream);
    case 3: return launch3_cpt<T, 3>(src, dst, nx, ny, nz, alpha, r, t, stream);
    case 4: return launch3_cpt<T, 4>(src, dst, nx, ny, nz, alpha, r, t, stream);
    case 5: return launch3_cpt<T, 5>(src, dst, nx, ny, nz, alpha, r, t, stream);
    case 6: return launch3_cpt<T, 6>(src, dst, nx, ny, nz, alpha, r, t, stream);
    case 7: return launch3_cpt<T, 7>(src, dst, nx, ny, nz, alpha, r, t, stream);
    case 8: return launch3_cpt<T, 8>(src, dst, nx, ny, nz, alpha, r, t, stream);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_stream3d<float>(const float *, float *, int, int, int, float, float,
                                           const Tile3D &, hipStream_t);
template hipError_t launch_stream3d<double>(const double *, double *, int, int, int, double,
                                            double, const Tile3D &, hipStream_t);

}  // namespace ac
