// The explicit Allen-Cahn update of one cell, shared by every kernel.
#pragma once

#include <hip/hip_runtime.h>

namespace ac {

// ---------------------------------------------------------------------------
// The explicit Allen-Cahn update of one cell (section 2.1, Eq. pytorchACeq):
//   phi' = phi + alpha*(phi - phi^3) + r*(S - 2d*phi),
//   alpha = dt/eps^2, r = dt/h^2, S = sum of the axis neighbours.
// The neighbour sum is paired per axis, (x- + x+) + (y- + y+) [+ (z- + z+)],
// and every product is written out explicitly, so every kernel (any tile
// shape, any temporal-blocking depth) rounds identically in each precision.
//
// FP32 evaluates the increment form above in five operations: S - 2d*phi is
// exact where S ~ 2d*phi (one rounding of a small value), and phi only meets
// the rounding of the final sum, so a smooth field loses little per step.
// FP64 evaluates the equal form
//   phi' = phi * (k1 + alpha*(1 - phi^2)) + r*S,   k1 = 1 - 2d*r,
// in four: it rounds phi*k1 and r*S as whole values (about one ulp of phi
// per step instead of one ulp of the increment), which in FP64 stays far
// below every bar, while in FP32 it measured 2-13x the FP32-vs-FP64 error
// of the increment form.  k1 = fma(-2d, r, 1) is loop-invariant (hoisted).
//
// phi = +-1 and phi = 0 are bitwise fixed points in both forms:
//   increment form, c = +-1: c*c = 1, fma(-1, c, c) = 0, S = 2d*c exactly;
//   product form, c = +-1: 1 - c^2 = 0 exactly, so w = k1, and r*2d + k1
//   rounds to 1 because k1 is 1 - 2d*r rounded once to a value below 1
//   (|error| <= ulp(1)/4), the stability bound keeping 1 - 2d*r >= 0;
//   c = 0 (with zero neighbours): every term is 0.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
__device__ __forceinline__ T react_and_diffuse(T c, T s, T two_d, T alpha, T r) {
    if constexpr (sizeof(T) == 8) {
        const T k1 = fma_(-two_d, r, T(1));    // 1 - 2d*r (loop-invariant)
        const T u = fma_(-c, c, T(1));         // 1 - c^2, rounded once
        const T w = fma_(alpha, u, k1);        // k1 + alpha*(1 - c^2)
        return fma_(r, s, w * c);              // c*w + r*S
    } else {
        const T lap = fma_(-two_d, c, s);      // S - 2d*c, rounded once
        const T c2 = c * c;
        const T re = fma_(-c2, c, c);          // c - c^3
        const T t = fma_(alpha, re, c);        // c + alpha*(c - c^3)
        return fma_(r, lap, t);                // + r*(S - 2d*c)
    }
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
