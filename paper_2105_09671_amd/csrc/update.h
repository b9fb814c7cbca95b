// The explicit Allen-Cahn update of one cell, shared by every kernel.
#pragma once

#include <hip/hip_runtime.h>

namespace ac {

// ---------------------------------------------------------------------------
// The explicit Allen-Cahn update of one cell (section 2.1, Eq. pytorchACeq):
//   phi' = phi + alpha*(phi - phi^3) + r*(S - 2d*phi),
//   alpha = dt/eps^2, r = dt/h^2, S = sum of the axis neighbours.
// The neighbour sum is paired per axis, (x- + x+) + (y- + y+) [+ (z- + z+)],
// and the remaining products are fused multiply-adds written out explicitly,
// so every kernel (any tile shape, any temporal-blocking depth) rounds
// identically.  phi = +-1 and phi = 0 are bitwise fixed points:
//   c = +-1: c*c = 1, fma(-1, c, c) = 0, and S = 2d*c exactly.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
__device__ __forceinline__ T react_and_diffuse(T c, T s, T two_d, T alpha, T r) {
    const T lap = fma_(-two_d, c, s);      // S - 2d*c, rounded once
    const T c2 = c * c;
    const T re = fma_(-c2, c, c);          // c - c^3
    const T t = fma_(alpha, re, c);        // c + alpha*(c - c^3)
    return fma_(r, lap, t);                // + r*(S - 2d*c)
}

template <typename T>
__device__ __forceinline__ T update2d(T c, T xm, T xp, T ym, T yp, T alpha, T r) {
    const T s = (xm + xp) + (ym + yp);
    return react_and_diffuse<T>(c, s, T(4), alpha, r);
}

template <typename T>
__device__ __forceinline__ T update3d(T c, T xm, T xp, T ym, T yp, T zm, T zp, T alpha, T r) {
    const T s = ((xm + xp) + (ym + yp)) + (zm + zp);
    return react_and_diffuse<T>(c, s, T(6), alpha, r);
}

}  // namespace ac
