// BF16 MFMA building blocks of the surrogate network (gfx950).
//
// Activations are NHWC bf16.  A tensor view is (ptr, channel stride Cs,
// channel offset Co): element (n, y, x, c) lives at ((n*H + y)*W + x)*Cs + Co + c,
// so a concatenation is two views into one buffer and costs no copy.
//
// Every convolution is an implicit GEMM on a (32 WM) x (32 WN) output tile
// with K stepped by 32.  A workgroup of 256 threads (WM x WN = 4 waves) stages
// one A tile and one B tile in LDS per K step (both stored with the K index
// contiguous), then each wave issues 2 x 2 v_mfma_f32_16x16x32_bf16 with FP32
// accumulation on its 32 x 32 block.  Operand layout of that
// instruction (wave64): lane l supplies A[l % 16][8*(l/16) .. +7] and
// B[8*(l/16) .. +7][l % 16]; it receives D[4*(l/16) + r][l % 16], r = 0..3.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ac {
namespace sur {

typedef unsigned short bf16_t;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 32, LP = BK + 8;   // LDS pitch (bf16 units)

// float -> bf16, round to nearest even (NaN stays NaN)
__host__ __device__ inline bf16_t f2bf(float f) {
    unsigned u;
    __builtin_memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (bf16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}
__host__ __device__ inline float bf2f(bf16_t h) {
    unsigned u = (unsigned)h << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

struct View {
    bf16_t *p;
    int Cs, Co;
};

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Generalised tile: WM x WN waves (WM * WN = 4), each owning a 32 x 32 block
// (2 x 2 MFMA tiles); the workgroup tile is (32 WM) x (32 WN).
template <int WM, int WN>
__device__ inline void mma_step_t(const bf16_t *As, const bf16_t *Bs, floatx4 acc[2][2]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm = w % WM, wn = w / WM;
    const int r = lane & 15, kc = (lane >> 4) * 8;
    bf16x8 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        a[i] = *reinterpret_cast<const bf16x8 *>(As + (wm * 32 + i * 16 + r) * LP + kc);
        b[i] = *reinterpret_cast<const bf16x8 *>(Bs + (wn * 32 + i * 16 + r) * LP + kc);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
}

// M tile of a GEMM launched with ceil(n/8)*8 workgroups along x.  The
// dispatcher places workgroup g on XCD g mod 8; XCD x gets the x-th contiguous
// eighth of the M tiles, so output rows that read the same input rows through
// a 3x3 window run on one XCD and share its L2 (round-robin tiles would have
// every XCD fetch every input row).  Returns n or more for the padding
// workgroups of the last eighth.
__device__ inline int xcd_tile(int n) {
    const int per = (n + 7) >> 3;
    return (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
}

inline unsigned xcd_grid(int n) { return 8u * (unsigned)((n + 7) >> 3); }

template <int WM, int WN>
__device__ inline void acc_coord_t(int i, int j, int r, int *row, int *col) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    *row = (w % WM) * 32 + i * 16 + (lane >> 4) * 4 + r;
    *col = (w / WM) * 32 + j * 16 + (lane & 15);
}

}  // namespace sur
}  // namespace ac
