// Learned K-step surrogate: a 3-level U-Net (32-64-128 channels, replicate
// padding) mapping phi to phi + U(phi), trained and run with hand-written
// BF16 MFMA kernels (FP32 accumulation, FP32 master weights and Adam).
//
// Network (a 3x3 conv is replicate padded, the discrete zero-Neumann
// boundary; every conv has a bias; relu where marked):
//   e1a = relu conv3(phi)            e1 = relu conv3(e1a)          H x W, 32 ch
//   e2a = relu conv3(pool e1)        e2 = relu conv3(e2a)          H/2,   64 ch
//   bt  = relu conv3(pool e2)                                      H/4,  128 ch
//   u2  = conv1(up bt)   d2 = relu conv3(cat(u2, e2))              H/2,   64 ch
//   u1  = conv1(up d2)   d1 = relu conv3(cat(u1, e1))              H,     32 ch
//   out = phi + conv1(d1)
// A 1x1 conv commutes with nearest upsampling, so u2 and u1 are computed at
// the low resolution (4x fewer flops), in the epilogue of the 3x3 layer that
// produces their input.  cat(u, e) is one buffer in training: a copy kernel
// writes each u value to its 2x2 block of channels [0, C), the encoder
// writes e straight into [C, 2C); inference keeps u at the low resolution and
// the next 3x3 layer reads it through the upsampling.
//
// Backward of a replicate-padded conv: with X_pad[p] = X[clamp(p - 1)] the
// forward is a valid correlation over X_pad, so dX_pad is the full (zero
// padded) correlation of dZ with the flipped kernel -- an implicit GEMM -- and
// dX adds the pad ring onto the border cells it was copied from (fold kernel).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "ac_internal.h"
#include "conv_patch.h"
#include "sur_kernels.h"

namespace ac {
namespace sur {

// ------------------------------------------------------- input gradient ----
// dX_pad at (y+1, x+1) = sum_{tap, co} dZ[y+1-ky][x+1-kx][co] * W[co][tap][ci]
// (zero outside the image); 1x1: dX = dZ W.  Rows = pixels, cols = input
// channels, K = (tap, co) with the weights pre-transposed to [tap][Cin][Cout].
// Epilogue: channels >= mask_c0 are multiplied by [mask > 0] (the relu of the
// layer that produced X); accumulate adds to what dX holds.
template <int KS, int WM, int WN>
__global__ void __launch_bounds__(256)
conv_dgrad_kernel(View dZ, int lgCout, int B, int H, int W, const bf16_t *__restrict__ Wt,
                  int Cin, View dX, View mask, int mask_c0, int accumulate)
{
    constexpr int TBM = 32 * WM, TBN = 32 * WN;
    constexpr int NA = (TBM * 4 + 255) / 256, NB = (TBN * 4 + 255) / 256;
    __shared__ __align__(16) bf16_t As[TBM * LP];
    __shared__ __align__(16) bf16_t Bs[TBN * LP];
    const int Cout = 1 << lgCout, K = KS * KS * Cout, M = B * H * W;
    const int mt = xcd_tile((M + TBM - 1) / TBM);
    if (mt * TBM >= M) return;                      // padding workgroup (whole group)
    const int m0 = mt * TBM, n0 = blockIdx.y * TBN;
    const int t = threadIdx.x;
    int arow[NA], akc[NA], pn[NA], py[NA], px[NA];
    bool aok[NA];
#pragma unroll
    for (int u = 0; u < NA; ++u) {
        const int c = t + 256 * u;
        arow[u] = c >> 2;
        akc[u] = (c & 3) * 8;
        const int m = m0 + arow[u];
        aok[u] = c < TBM * 4 && m < M;
        pn[u] = py[u] = px[u] = 0;
        if (aok[u]) {
            pn[u] = m / (H * W);
            const int rem = m - pn[u] * H * W;
            py[u] = rem / W;
            px[u] = rem - py[u] * W;
        }
    }
    auto loadA = [&](int u, int k0) -> uint4 {
        const int k = k0 + akc[u];
        if (!aok[u] || k >= K) return uint4{0, 0, 0, 0};
        const int tap = k >> lgCout, co = k & (Cout - 1);
        int yy = py[u], xx = px[u];
        if (KS == 3) {
            yy = py[u] + 1 - tap / 3;
            xx = px[u] + 1 - tap % 3;
            if (yy < 0 || yy >= H || xx < 0 || xx >= W) return uint4{0, 0, 0, 0};
        }
        return *reinterpret_cast<const uint4 *>(dZ.p + ((size_t)(pn[u] * H + yy) * W + xx) * dZ.Cs + dZ.Co + co);
    };
    auto loadB = [&](int u, int k0) -> uint4 {
        const int c = t + 256 * u, ci = n0 + (c >> 2), k = k0 + (c & 3) * 8;
        if (c >= TBN * 4 || ci >= Cin || k >= K) return uint4{0, 0, 0, 0};
        const int tap = k >> lgCout, co = k & (Cout - 1);
        return *reinterpret_cast<const uint4 *>(Wt + ((size_t)tap * Cin + ci) * Cout + co);
    };
    floatx4 acc[2][2] = {};
    uint4 ra[NA], rb[NB];
#pragma unroll
    for (int u = 0; u < NA; ++u) ra[u] = loadA(u, 0);
#pragma unroll
    for (int u = 0; u < NB; ++u) rb[u] = loadB(u, 0);
    for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
        for (int u = 0; u < NA; ++u)
            if (t + 256 * u < TBM * 4) *reinterpret_cast<uint4 *>(As + arow[u] * LP + akc[u]) = ra[u];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int c = t + 256 * u;
            if (c < TBN * 4) *reinterpret_cast<uint4 *>(Bs + (c >> 2) * LP + (c & 3) * 8) = rb[u];
        }
        __syncthreads();
        if (k0 + BK < K) {
#pragma unroll
            for (int u = 0; u < NA; ++u) ra[u] = loadA(u, k0 + BK);
#pragma unroll
            for (int u = 0; u < NB; ++u) rb[u] = loadB(u, k0 + BK);
        }
        mma_step_t<WM, WN>(As, Bs, acc);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                int row, col;
                acc_coord_t<WM, WN>(i, j, q, &row, &col);
                const int mg = m0 + row, cg = n0 + col;
                if (mg >= M || cg >= Cin) continue;
                float v = acc[i][j][q];
                if (mask.p && cg >= mask_c0 && !(bf2f(mask.p[(size_t)mg * mask.Cs + mask.Co + cg]) > 0.f))
                    v = 0.f;
                bf16_t *dst = dX.p + (size_t)mg * dX.Cs + dX.Co + cg;
                if (accumulate) v += bf2f(*dst);
                *dst = f2bf(v);
            }
}

// The pad ring of dX_pad, folded onto the border cells (3x3 only).  One thread
// per (border cell, input channel).  W is the forward layout [Cout][tap][Cin].
__global__ void dgrad_fold_kernel(View dZ, int Cout, int B, int H, int W,
                                  const bf16_t *__restrict__ Wk, int Cin, View dX, View mask,
                                  int mask_c0)
{
    const int nb = (H == 1 || W == 1) ? H * W : 2 * W + 2 * (H - 2);
    const long long total = (long long)B * nb * Cin;
    for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < total;
         id += (long long)gridDim.x * blockDim.x) {
        const int ci = (int)(id % Cin);
        const long long pb = id / Cin;
        const int n = (int)(pb / nb), b = (int)(pb % nb);
        int y, x;
        if (H == 1 || W == 1) { y = b / W; x = b % W; }
        else if (b < W) { y = 0; x = b; }
        else if (b < 2 * W) { y = H - 1; x = b - W; }
        else { const int q = b - 2 * W; y = 1 + (q >> 1); x = (q & 1) ? W - 1 : 0; }
        int P[3], Q[3], np = 0, nq = 0;
        P[np++] = y + 1;
        if (y == 0) P[np++] = 0;
        if (y == H - 1) P[np++] = H + 1;
        Q[nq++] = x + 1;
        if (x == 0) Q[nq++] = 0;
        if (x == W - 1) Q[nq++] = W + 1;
        float s = 0.f;
        for (int a = 0; a < np; ++a)
            for (int c = 0; c < nq; ++c) {
                if (a == 0 && c == 0) continue;   // the main kernel's position
                for (int ky = 0; ky < 3; ++ky) {
                    const int yy = P[a] - ky;
                    if (yy < 0 || yy >= H) continue;
                    for (int kx = 0; kx < 3; ++kx) {
                        const int xx = Q[c] - kx;
                        if (xx < 0 || xx >= W) continue;
                        const bf16_t *g = dZ.p + ((size_t)(n * H + yy) * W + xx) * dZ.Cs + dZ.Co;
                        const bf16_t *w = Wk + (size_t)(ky * 3 + kx) * Cin + ci;
                        for (int co = 0; co < Cout; ++co)
                            s += bf2f(g[co]) * bf2f(w[(size_t)co * 9 * Cin]);
                    }
                }
            }
        if (s == 0.f) continue;
        const size_t pix = (size_t)(n * H + y) * W + x;
        if (mask.p && ci >= mask_c0 && !(bf2f(mask.p[pix * mask.Cs + mask.Co + ci]) > 0.f)) continue;
        bf16_t *dst = dX.p + pix * dX.Cs + dX.Co + ci;
        *dst = f2bf(bf2f(*dst) + s);
    }
}

// ------------------------------------------------------ weight gradient ----
// dW[co][(tap, ci)] += sum over pixels dZ[p][co] * X[shift_tap(p)][ci].  Rows =
// output channels, cols = (tap, ci), K = pixels.  Both operands are read 8
// channels at a time and transposed into LDS (K contiguous).  Each workgroup
// owns one pixel range (split K) and adds its tile into dW with FP32 atomics.
template <int KS, int WM, int WN>
__global__ void __launch_bounds__(256)
conv_wgrad_kernel(View dZ, int Cout, View X, int lgCin, int B, int H, int W,
                  float *__restrict__ dW, int pix_per_split)
{
    constexpr int TBM = 32 * WM, TBN = 32 * WN;
    constexpr int CA = TBM / 8, CB = TBN / 8;                  // 8-channel chunks per pixel
    constexpr int NA = (32 * CA + 255) / 256, NB = (32 * CB + 255) / 256;
    __shared__ __align__(16) bf16_t As[TBM * LP];
    __shared__ __align__(16) bf16_t Bs[TBN * LP];
    const int Cin = 1 << lgCin, Kw = KS * KS * Cin, M = B * H * W;
    const int m0 = blockIdx.x * TBM, n0 = blockIdx.y * TBN;     // M tiles over Cout here
    const int p_begin = blockIdx.z * pix_per_split;
    const int p_end = min(M, p_begin + pix_per_split);
    if (p_begin >= p_end) return;
    const int t = threadIdx.x;
    auto loadA = [&](int u, int p0) -> uint4 {
        const int c = t + 256 * u, pl = c / CA, co = m0 + (c % CA) * 8, p = p0 + pl;
        if (c >= 32 * CA || p >= p_end || co >= Cout) return uint4{0, 0, 0, 0};
        return *reinterpret_cast<const uint4 *>(dZ.p + (size_t)p * dZ.Cs + dZ.Co + co);
    };
    auto loadB = [&](int u, int p0) -> uint4 {
        const int c = t + 256 * u, pl = c / CB, kk = n0 + (c % CB) * 8, p = p0 + pl;
        if (c >= 32 * CB || p >= p_end || kk >= Kw) return uint4{0, 0, 0, 0};
        const int tap = kk >> lgCin, ci = kk & (Cin - 1);
        const int n = p / (H * W), rem = p - n * H * W;
        int y = rem / W, x = rem - y * W;
        if (KS == 3) {
            y = clampi(y + tap / 3 - 1, 0, H - 1);
            x = clampi(x + tap % 3 - 1, 0, W - 1);
        }
        return *reinterpret_cast<const uint4 *>(X.p + ((size_t)(n * H + y) * W + x) * X.Cs + X.Co + ci);
    };
    floatx4 acc[2][2] = {};
    uint4 ra[NA], rb[NB];
#pragma unroll
    for (int u = 0; u < NA; ++u) ra[u] = loadA(u, p_begin);
#pragma unroll
    for (int u = 0; u < NB; ++u) rb[u] = loadB(u, p_begin);
    for (int p0 = p_begin; p0 < p_end; p0 += BK) {
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            const int c = t + 256 * u;
            if (c < 32 * CA) {
                const bf16_t *v = reinterpret_cast<const bf16_t *>(&ra[u]);
                const int pl = c / CA, cc = (c % CA) * 8;
#pragma unroll
                for (int e = 0; e < 8; ++e) As[(cc + e) * LP + pl] = v[e];
            }
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int c = t + 256 * u;
            if (c < 32 * CB) {
                const bf16_t *v = reinterpret_cast<const bf16_t *>(&rb[u]);
                const int pl = c / CB, cc = (c % CB) * 8;
#pragma unroll
                for (int e = 0; e < 8; ++e) Bs[(cc + e) * LP + pl] = v[e];
            }
        }
        __syncthreads();
        if (p0 + BK < p_end) {
#pragma unroll
            for (int u = 0; u < NA; ++u) ra[u] = loadA(u, p0 + BK);
#pragma unroll
            for (int u = 0; u < NB; ++u) rb[u] = loadB(u, p0 + BK);
        }
        mma_step_t<WM, WN>(As, Bs, acc);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                int row, col;
                acc_coord_t<WM, WN>(i, j, q, &row, &col);
                const int rg = m0 + row, cg = n0 + col;
                if (rg < Cout && cg < Kw) atomicAdd(dW + (size_t)rg * Kw + cg, acc[i][j][q]);
            }
}

// db[c] += sum over pixels dZ[p][c]
__global__ void bias_grad_kernel(View dZ, int C, int M, float *db)
{
    const int groups = blockDim.x / C;
    const int c = threadIdx.x % C, gi = threadIdx.x / C;
    if (gi >= groups) return;
    float s = 0.f;
    for (long long p = (long long)blockIdx.x * groups + gi; p < M; p += (long long)gridDim.x * groups)
        s += bf2f(dZ.p[(size_t)p * dZ.Cs + dZ.Co + c]);
    atomicAdd(db + c, s);
}

// ------------------------------------------------------- point-wise ops ----
// phi [n] FP32 -> X0 NHWC with 8 channels, channel 0 = phi, 1..7 = 0
__global__ void pack_input_kernel(const float *phi, bf16_t *x0, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        uint4 v{(unsigned)f2bf(phi[i]), 0u, 0u, 0u};
        reinterpret_cast<uint4 *>(x0)[i] = v;
    }
}

// 2x2 average, 8 channels per thread
__global__ void pool_kernel(View X, int C, int B, int H, int W, View Y)
{
    const int Ho = H / 2, Wo = W / 2, c8 = C / 8;
    const long long total = (long long)B * Ho * Wo * c8;
    for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < total;
         id += (long long)gridDim.x * blockDim.x) {
        const int cq = (int)(id % c8);
        const long long pix = id / c8;
        const int n = (int)(pix / (Ho * Wo)), rem = (int)(pix % (Ho * Wo)), y = rem / Wo, x = rem % Wo;
        float s[8] = {};
        for (int d = 0; d < 4; ++d) {
            const size_t ip = ((size_t)n * H + 2 * y + (d >> 1)) * W + 2 * x + (d & 1);
            const uint4 v = *reinterpret_cast<const uint4 *>(X.p + ip * X.Cs + X.Co + cq * 8);
            const bf16_t *e = reinterpret_cast<const bf16_t *>(&v);
            for (int k = 0; k < 8; ++k) s[k] += bf2f(e[k]);
        }
        uint4 o;
        bf16_t *oe = reinterpret_cast<bf16_t *>(&o);
        for (int k = 0; k < 8; ++k) oe[k] = f2bf(0.25f * s[k]);
        *reinterpret_cast<uint4 *>(Y.p + (size_t)pix * Y.Cs + Y.Co + cq * 8) = o;
    }
}

// dX (H x W) += 0.25 * dP(y/2, x/2) * [mask > 0]
__global__ void pool_bwd_kernel(View dP, int C, int B, int H, int W, View dX, View mask)
{
    const long long total = (long long)B * H * W * C;
    for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < total;
         id += (long long)gridDim.x * blockDim.x) {
        const int c = (int)(id % C);
        const long long pix = id / C;
        const int n = (int)(pix / (H * W)), rem = (int)(pix % (H * W)), y = rem / W, x = rem % W;
        if (!(bf2f(mask.p[(size_t)pix * mask.Cs + mask.Co + c]) > 0.f)) continue;
        const size_t lp = ((size_t)n * (H / 2) + y / 2) * (W / 2) + x / 2;
        const float g = 0.25f * bf2f(dP.p[lp * dP.Cs + dP.Co + c]);
        bf16_t *dst = dX.p + (size_t)pix * dX.Cs + dX.Co + c;
        *dst = f2bf(bf2f(*dst) + g);
    }
}

// dLow (Hl x Wl) = sum of the 2x2 block of dHigh
__global__ void up_bwd_kernel(View dHigh, int C, int B, int Hl, int Wl, View dLow)
{
    const long long total = (long long)B * Hl * Wl * C;
    for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < total;
         id += (long long)gridDim.x * blockDim.x) {
        const int c = (int)(id % C);
        const long long pix = id / C;
        const int n = (int)(pix / (Hl * Wl)), rem = (int)(pix % (Hl * Wl)), y = rem / Wl, x = rem % Wl;
        float s = 0.f;
        for (int d = 0; d < 4; ++d) {
            const size_t hp = ((size_t)n * 2 * Hl + 2 * y + (d >> 1)) * 2 * Wl + 2 * x + (d & 1);
            s += bf2f(dHigh.p[hp * dHigh.Cs + dHigh.Co + c]);
        }
        dLow.p[(size_t)pix * dLow.Cs + dLow.Co + c] = f2bf(s);
    }
}

// dHigh (2 Hl x 2 Wl) = nearest 2x upsampling of dLow; C a multiple of 8,
// 16 bytes per thread
__global__ void up_copy_kernel(View low, int C, int B, int Hl, int Wl, View high)
{
    const int q8 = C >> 3;
    const long long total = (long long)B * 4 * Hl * Wl * q8;
    for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < total;
         id += (long long)gridDim.x * blockDim.x) {
        const int q = (int)(id % q8);
        const long long pix = id / q8;
        const int Wh = 2 * Wl, Hh = 2 * Hl;
        const int n = (int)(pix / ((long long)Hh * Wh)), rem = (int)(pix % ((long long)Hh * Wh));
        const int y = rem / Wh, x = rem % Wh;
        const size_t lp = ((size_t)n * Hl + (y >> 1)) * Wl + (x >> 1);
        *reinterpret_cast<uint4 *>(high.p + (size_t)pix * high.Cs + high.Co + 8 * q) =
            *reinterpret_cast<const uint4 *>(low.p + lp * low.Cs + low.Co + 8 * q);
    }
}

// out = phi + b + sum_c d1[c] w[c]   (the 1x1 head, C = 32)
__global__ void head_fwd_kernel(View d1, const float *wh, const float *bh, const float *phi,
                                float *out, int M)
{
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < M; p += gridDim.x * blockDim.x) {
        const bf16_t *a = d1.p + (size_t)p * d1.Cs + d1.Co;
        float s = bh[0];
        for (int c = 0; c < 32; ++c) s += bf2f(a[c]) * wh[c];
        out[p] = phi[p] + s;
    }
}

// r = out - target; dU = 2 r / M; loss += sum r^2 / M
__global__ void mse_kernel(const float *out, const float *tgt, float *dU, int M, float *loss)
{
    __shared__ float red[256];
    float s = 0.f;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < M; p += gridDim.x * blockDim.x) {
        const float r = out[p] - tgt[p];
        dU[p] = 2.f * r / (float)M;
        s += r * r;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = blockDim.x / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(loss, red[0] / (float)M);
}

// head backward: dd1 = dU w [d1 > 0]; dw += dU d1; db += dU
__global__ void head_bwd_kernel(View d1, const float *dU, const float *wh, int M, View dd1,
                                float *dwh, float *dbh)
{
    __shared__ float red[33][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    float sw[32] = {}, sb = 0.f;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < M; p += gridDim.x * blockDim.x) {
        const bf16_t *a = d1.p + (size_t)p * d1.Cs + d1.Co;
        bf16_t *g = dd1.p + (size_t)p * dd1.Cs + dd1.Co;
        const float u = dU[p];
        sb += u;
        for (int c = 0; c < 32; ++c) {
            const float av = bf2f(a[c]);
            sw[c] += u * av;
            g[c] = f2bf(av > 0.f ? u * wh[c] : 0.f);
        }
    }
    // reduce over the block: wave-wise through LDS
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
        if (wv == w) {
            for (int c = 0; c < 32; ++c) red[c][lane] = (w == 0 ? 0.f : red[c][lane]) + sw[c];
            red[32][lane] = (w == 0 ? 0.f : red[32][lane]) + sb;
        }
        __syncthreads();
    }
    if (threadIdx.x < 33) {
        float s = 0.f;
        for (int l = 0; l < 64; ++l) s += red[threadIdx.x][l];
        atomicAdd(threadIdx.x < 32 ? dwh + threadIdx.x : dbh, s);
    }
}

// FP32 canonical weights -> bf16 [Cout][K] (cin_pad > cin zero-pads the input
// channels, used for the 1-channel first layer)
__global__ void pack_weights_kernel(const float *w, int Cout, int taps, int cin, int cin_pad,
                                    bf16_t *out)
{
    const int total = Cout * taps * cin_pad;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const int c = i % cin_pad, rest = i / cin_pad;
        out[i] = c < cin ? f2bf(w[(size_t)rest * cin + c]) : (bf16_t)0;
    }
}

// w -> bf16(w) held as FP32 (the first layer's weights for its VALU form)
__global__ void round_first_weights_kernel(const float *w, int n, float *out)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) out[i] = bf2f(f2bf(w[i]));
}

// [Cout][taps][Cin] -> [taps][Cin][Cout]
__global__ void transpose_w_kernel(const bf16_t *w, int Cout, int taps, int Cin, bf16_t *wt)
{
    const int total = Cout * taps * Cin;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const int co = i % Cout, rest = i / Cout, ci = rest % Cin, tap = rest / Cin;
        wt[i] = w[((size_t)co * taps + tap) * Cin + ci];
    }
}

// first-layer weight gradient [Cout][9][8] -> canonical [Cout][9][1]
__global__ void unpack_first_grad_kernel(const float *g8, int Cout, float *g)
{
    const int total = Cout * 9;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x)
        g[i] = g8[(size_t)i * 8];
}

__global__ void adam_kernel(float *w, float *m, float *v, const float *g, int n, float lr,
                            float b1, float b2, float eps, float bc1, float bc2)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        w[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    }
}

}  // namespace sur
}  // namespace ac

// =================================================================== host ====
using namespace ac;
using namespace ac::sur;

namespace {

enum { L_E1A, L_E1B, L_E2A, L_E2B, L_BT, L_U2, L_D2, L_U1, L_D1, L_HEAD, NL };
struct LayerDef {
    int cin, cout, k;
};
const LayerDef kLayers[NL] = {{1, 32, 3},  {32, 32, 3}, {32, 64, 3}, {64, 64, 3},  {64, 128, 3},
                              {128, 64, 1}, {128, 64, 3}, {64, 32, 1}, {64, 32, 3}, {32, 1, 1}};

int lg2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

}  // namespace

struct ac_sur {
    int Bmax = 0, H = 0, W = 0;
    hipStream_t st = nullptr;
    int64_t nparam = 0;
    int64_t woff[NL], boff[NL];     // canonical flat offsets (weights, bias)
    int64_t kwoff[NL];              // offsets into the bf16 kernel-layout weights
    float *w32 = nullptr, *m = nullptr, *v = nullptr, *g = nullptr, *g_first = nullptr;
    bf16_t *wb = nullptr, *wt = nullptr, *wf = nullptr;   // wf: fragment order (Cin >= 32, Cout >= 16)
    bf16_t *u2lo = nullptr, *u1lo = nullptr;             // decoder 1x1 outputs at low resolution (inference)
    float *w1f = nullptr;                                // first-layer weights rounded to BF16, [32][9]
    float *out = nullptr, *dU = nullptr, *loss = nullptr;
    bf16_t *x0, *e1a, *cat1, *p1, *e2a, *cat2, *p2, *bt, *d2, *d1;
    bf16_t *dd1, *dcat1, *du1, *dd2, *dcat2, *du2, *dbt, *dp2, *de2a, *dp1, *de1a;
    std::vector<void *> allocs;
    bool have_fwd = false, have_loss = false;
    int last_batch = 0;
    const float *last_phi = nullptr;
};

namespace {

ac_status sur_alloc(ac_sur *s, void **p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes ? bytes : 16);
    if (e != hipSuccess) return fail(AC_ERR_NOMEM, "surrogate allocation of %zu B: %s", bytes, hipGetErrorString(e));
    s->allocs.push_back(*p);
    return AC_OK;
}

dim3 grid1(long long n, int per = 256) {
    long long g = (n + per - 1) / per;
    return dim3((unsigned)std::min<long long>(std::max<long long>(g, 1), 65535));
}

View V(bf16_t *p, int Cs, int Co = 0) { return View{p, Cs, Co}; }

const float *bias_of(const ac_sur *s, int l) { return s->w32 + s->boff[l]; }
const bf16_t *wk_of(const ac_sur *s, int l) { return s->wb + s->kwoff[l]; }
const bf16_t *wt_of(const ac_sur *s, int l) { return s->wt + s->kwoff[l]; }

// Y = act(conv(X)); H, W: the resolution of X (and Y unless up)
// ul: the decoder 1x1 layer fused into the epilogue (UPC > 0), writing `up`
template <int CIN, int CN, int RW, int LOWC, bool POOL, bool HEAD, bool FIRST = false, int UPC = 0>
void launch_c3p(ac_sur *s, int l, View X, View Xlo, int B, int H, int W, View Y, View P,
                const float *phi = nullptr, float *out = nullptr, bf16_t *e1a_out = nullptr,
                int ul = -1, View up = View{nullptr, 0, 0}) {
    const LayerDef &L = kLayers[l];
    constexpr int lds = conv3p_lds_bytes<RW, CN, FIRST>();
    const void *kern =
        reinterpret_cast<const void *>(&conv3_patch_kernel<CIN, CN, RW, LOWC, POOL, HEAD, FIRST, UPC>);
    set_lds_limit(kern, lds);
    const int ntiles = B * ((H + 4 * RW - 1) / (4 * RW)) * ((W + 63) / 64);
    dim3 grid(xcd_grid(ntiles), L.cout / CN);
    const ConvAux aux{phi, out, s->w32 + s->woff[L_HEAD], s->w32 + s->boff[L_HEAD], s->w1f,
                      bias_of(s, L_E1A), e1a_out, ul >= 0 ? s->wf + s->kwoff[ul] : nullptr,
                      ul >= 0 ? bias_of(s, ul) : nullptr, up};
    hipLaunchKernelGGL((conv3_patch_kernel<CIN, CN, RW, LOWC, POOL, HEAD, FIRST, UPC>), grid, dim3(256), lds,
                       s->st, X, Xlo, B, H, W, s->wf + s->kwoff[l], bias_of(s, l), L.cout, Y, P, aux);
}


template <int KS, int WM, int WN>
void launch_wgrad(ac_sur *s, View dZ, int cout, View X, int lgcin, int B, int H, int W, float *dW) {
    const int M = B * H * W, Kw = KS * KS * (1 << lgcin);
    const int tiles = ((cout + 32 * WM - 1) / (32 * WM)) * ((Kw + 32 * WN - 1) / (32 * WN));
    int splits = std::max(1, std::min(2048 / tiles, (M + 255) / 256));
    int per = (M + splits - 1) / splits;
    per = (per + BK - 1) / BK * BK;
    splits = (M + per - 1) / per;
    dim3 gw((cout + 32 * WM - 1) / (32 * WM), (Kw + 32 * WN - 1) / (32 * WN), splits);
    hipLaunchKernelGGL((conv_wgrad_kernel<KS, WM, WN>), gw, dim3(256), 0, s->st, dZ, cout, X, lgcin,
                       B, H, W, dW, per);
}

template <int KS, int WM, int WN>
void launch_dgrad(ac_sur *s, int l, View dZ, int lgcout, int B, int H, int W, int cin, View dX,
                  View mask, int mask_c0) {
    const int M = B * H * W;
    dim3 gd(xcd_grid((M + 32 * WM - 1) / (32 * WM)), (cin + 32 * WN - 1) / (32 * WN));
    hipLaunchKernelGGL((conv_dgrad_kernel<KS, WM, WN>), gd, dim3(256), 0, s->st, dZ, lgcout, B, H, W,
                       wt_of(s, l), cin, dX, mask, mask_c0, 0);
}

// gradients of layer l from dZ (grad at its pre-activation output) and its
// input X: weight grad into dWdst (FP32, kernel layout), bias grad into the
// canonical array, and (if dX.p) the input grad with mask / fold.
void conv_bwd(ac_sur *s, int l, View X, View dZ, int B, int H, int W, float *dWdst, View dX,
              View mask, int mask_c0) {
    const LayerDef &L = kLayers[l];
    const int cin = l == L_E1A ? 8 : L.cin;
    const int M = B * H * W;
    const int lgcin = lg2(cin), lgcout = lg2(L.cout);
    // weight gradient: rows = output channels
    if (L.k == 3) {
        if (L.cout <= 32) launch_wgrad<3, 1, 4>(s, dZ, L.cout, X, lgcin, B, H, W, dWdst);
        else if (L.cout <= 64) launch_wgrad<3, 2, 2>(s, dZ, L.cout, X, lgcin, B, H, W, dWdst);
        else launch_wgrad<3, 4, 1>(s, dZ, L.cout, X, lgcin, B, H, W, dWdst);
    } else {
        if (L.cout <= 32) launch_wgrad<1, 1, 4>(s, dZ, L.cout, X, lgcin, B, H, W, dWdst);
        else if (L.cout <= 64) launch_wgrad<1, 2, 2>(s, dZ, L.cout, X, lgcin, B, H, W, dWdst);
        else launch_wgrad<1, 4, 1>(s, dZ, L.cout, X, lgcin, B, H, W, dWdst);
    }
    hipLaunchKernelGGL(bias_grad_kernel, dim3(std::min(1024, (M + 7) / 8)), dim3(256 / L.cout * L.cout),
                       0, s->st, dZ, L.cout, M, s->g + s->boff[l]);
    if (!dX.p) return;
    const bool narrow = cin <= 32;
    if (L.k == 3) {
        if (narrow) launch_dgrad<3, 4, 1>(s, l, dZ, lgcout, B, H, W, cin, dX, mask, mask_c0);
        else launch_dgrad<3, 2, 2>(s, l, dZ, lgcout, B, H, W, cin, dX, mask, mask_c0);
        const int nb = (H == 1 || W == 1) ? H * W : 2 * W + 2 * (H - 2);
        hipLaunchKernelGGL(dgrad_fold_kernel, grid1((long long)B * nb * cin), dim3(256), 0, s->st,
                           dZ, L.cout, B, H, W, wk_of(s, l), cin, dX, mask, mask_c0);
    } else {
        if (narrow) launch_dgrad<1, 4, 1>(s, l, dZ, lgcout, B, H, W, cin, dX, mask, mask_c0);
        else launch_dgrad<1, 2, 2>(s, l, dZ, lgcout, B, H, W, cin, dX, mask, mask_c0);
    }
}

void refresh_weights(ac_sur *s) {
    hipLaunchKernelGGL(round_first_weights_kernel, dim3(1), dim3(320), 0, s->st, s->w32 + s->woff[L_E1A],
                       32 * 9, s->w1f);
    for (int l = 0; l < NL; ++l) {
        if (l == L_HEAD) continue;   // the head reads the FP32 master directly
        const LayerDef &L = kLayers[l];
        const int cin_pad = l == L_E1A ? 8 : L.cin, taps = L.k * L.k;
        const int n = L.cout * taps * cin_pad;
        hipLaunchKernelGGL(pack_weights_kernel, grid1(n), dim3(256), 0, s->st, s->w32 + s->woff[l],
                           L.cout, taps, L.cin, cin_pad, s->wb + s->kwoff[l]);
        hipLaunchKernelGGL(transpose_w_kernel, grid1(n), dim3(256), 0, s->st, s->wb + s->kwoff[l],
                           L.cout, taps, cin_pad, s->wt + s->kwoff[l]);
        if (L.cin >= 32 && L.cout >= 16)   // 3x3 layers but the first; the decoder's 1x1 layers
            hipLaunchKernelGGL(pack_frag_weights_kernel, grid1(n), dim3(256), 0, s->st,
                               s->w32 + s->woff[l], L.cout, taps, L.cin, s->wf + s->kwoff[l]);
    }
}

}  // namespace

extern "C" {

int64_t ac_sur_num_params(void) {
    int64_t n = 0;
    for (int l = 0; l < NL; ++l) n += (int64_t)kLayers[l].cout * kLayers[l].k * kLayers[l].k * kLayers[l].cin + kLayers[l].cout;
    return n;
}

void ac_sur_destroy(ac_sur *s) {
    if (!s) return;
    (void)hipDeviceSynchronize();
    for (void *p : s->allocs) (void)hipFree(p);
    delete s;
}

ac_status ac_sur_create(ac_sur **out, int32_t batch_max, int32_t hw, void *stream) {
    g_err.clear();
    if (!out) return fail(AC_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    if (batch_max < 1 || hw < 8 || hw % 4 || (int64_t)batch_max * hw * hw > (1ll << 30))
        return fail(AC_ERR_INVALID_ARG, "batch_max >= 1 and hw >= 8, a multiple of 4, required");
    ac_sur *s = new ac_sur();
    s->Bmax = batch_max;
    s->H = s->W = hw;
    s->st = reinterpret_cast<hipStream_t>(stream);
    int64_t o = 0, ko = 0;
    for (int l = 0; l < NL; ++l) {
        const LayerDef &L = kLayers[l];
        s->woff[l] = o;
        o += (int64_t)L.cout * L.k * L.k * L.cin;
        s->boff[l] = o;
        o += L.cout;
        s->kwoff[l] = ko;
        ko += (int64_t)L.cout * L.k * L.k * (l == L_E1A ? 8 : L.cin);
        ko = (ko + 7) / 8 * 8;
    }
    s->nparam = o;
    const size_t n1 = (size_t)batch_max * hw * hw, n2 = n1 / 4, n3 = n1 / 16, B2 = sizeof(bf16_t);
    ac_status st = AC_OK;
    auto A = [&](void **p, size_t bytes) { if (st == AC_OK) st = sur_alloc(s, p, bytes); };
    A((void **)&s->w32, o * 4); A((void **)&s->m, o * 4); A((void **)&s->v, o * 4);
    A((void **)&s->g, o * 4); A((void **)&s->g_first, 32 * 72 * 4);
    A((void **)&s->wb, ko * B2); A((void **)&s->wt, ko * B2); A((void **)&s->wf, ko * B2);
    A((void **)&s->u2lo, n3 * 64 * B2); A((void **)&s->u1lo, n2 * 32 * B2);
    A((void **)&s->w1f, 32 * 9 * 4);
    A((void **)&s->out, n1 * 4); A((void **)&s->dU, n1 * 4); A((void **)&s->loss, 16);
    A((void **)&s->x0, n1 * 8 * B2); A((void **)&s->e1a, n1 * 32 * B2); A((void **)&s->cat1, n1 * 64 * B2);
    A((void **)&s->p1, n2 * 32 * B2); A((void **)&s->e2a, n2 * 64 * B2); A((void **)&s->cat2, n2 * 128 * B2);
    A((void **)&s->p2, n3 * 64 * B2); A((void **)&s->bt, n3 * 128 * B2); A((void **)&s->d2, n2 * 64 * B2);
    A((void **)&s->d1, n1 * 32 * B2);
    A((void **)&s->dd1, n1 * 32 * B2); A((void **)&s->dcat1, n1 * 64 * B2); A((void **)&s->du1, n2 * 32 * B2);
    A((void **)&s->dd2, n2 * 64 * B2); A((void **)&s->dcat2, n2 * 128 * B2); A((void **)&s->du2, n3 * 64 * B2);
    A((void **)&s->dbt, n3 * 128 * B2); A((void **)&s->dp2, n3 * 64 * B2); A((void **)&s->de2a, n2 * 64 * B2);
    A((void **)&s->dp1, n2 * 32 * B2); A((void **)&s->de1a, n1 * 32 * B2);
    if (st != AC_OK) {
        ac_sur_destroy(s);
        return st;
    }
    hipError_t e = hipMemsetAsync(s->w32, 0, o * 4, s->st);
    if (e == hipSuccess) e = hipMemsetAsync(s->m, 0, o * 4, s->st);
    if (e == hipSuccess) e = hipMemsetAsync(s->v, 0, o * 4, s->st);
    if (e != hipSuccess) {
        ac_sur_destroy(s);
        return hip_fail(e, "surrogate init");
    }
    refresh_weights(s);
    *out = s;
    return AC_OK;
}

ac_status ac_sur_set_weights(ac_sur *s, const float *host, int64_t n) {
    g_err.clear();
    if (!s || !host || n != s->nparam) return fail(AC_ERR_INVALID_ARG, "expected %lld weights", (long long)(s ? s->nparam : 0));
    hipError_t e = hipMemcpyAsync(s->w32, host, n * 4, hipMemcpyHostToDevice, s->st);
    if (e == hipSuccess) e = hipMemsetAsync(s->m, 0, n * 4, s->st);
    if (e == hipSuccess) e = hipMemsetAsync(s->v, 0, n * 4, s->st);
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    if (e != hipSuccess) return hip_fail(e, "set weights");
    refresh_weights(s);
    s->have_fwd = s->have_loss = false;
    return AC_OK;
}

ac_status ac_sur_get_weights(ac_sur *s, float *host, int64_t n) {
    g_err.clear();
    if (!s || !host || n != s->nparam) return fail(AC_ERR_INVALID_ARG, "expected %lld weights", (long long)(s ? s->nparam : 0));
    hipError_t e = hipMemcpyAsync(host, s->w32, n * 4, hipMemcpyDeviceToHost, s->st);
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    return e == hipSuccess ? AC_OK : hip_fail(e, "get weights");
}

ac_status ac_sur_get_grads(ac_sur *s, float *host, int64_t n) {
    g_err.clear();
    if (!s || !host || n != s->nparam) return fail(AC_ERR_INVALID_ARG, "expected %lld grads", (long long)(s ? s->nparam : 0));
    hipError_t e = hipMemcpyAsync(host, s->g, n * 4, hipMemcpyDeviceToHost, s->st);
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    return e == hipSuccess ? AC_OK : hip_fail(e, "get grads");
}

ac_status ac_sur_set_stream(ac_sur *s, void *stream) {
    if (!s) return fail(AC_ERR_INVALID_ARG, "null handle");
    s->st = reinterpret_cast<hipStream_t>(stream);
    return AC_OK;
}

ac_status ac_sur_forward(ac_sur *s, const float *phi_in, float *phi_out, int32_t batch) {
    g_err.clear();
    if (!s || !phi_in) return fail(AC_ERR_INVALID_ARG, "null handle or input");
    if (batch < 1 || batch > s->Bmax) return fail(AC_ERR_INVALID_ARG, "batch %d outside 1..%d", batch, s->Bmax);
    const int B = batch, H = s->H, W = s->W, H2 = H / 2, W2 = W / 2, H4 = H / 4, W4 = W / 4;
    const int n1 = B * H * W;
    hipLaunchKernelGGL(pack_input_kernel, grid1(n1), dim3(256), 0, s->st, phi_in, s->x0, n1);
    const View none{nullptr, 0, 0};
    // first two layers in one kernel (e1a kept for the backward pass)
    launch_c3p<32, 32, 1, 0, true, false, true>(s, L_E1B, none, none, B, H, W, V(s->cat1, 64, 32),
                                                V(s->p1, 32), phi_in, nullptr, s->e1a);
    launch_c3p<32, 64, 1, 0, false, false>(s, L_E2A, V(s->p1, 32), none, B, H2, W2, V(s->e2a, 64), none);
    launch_c3p<64, 64, 1, 0, true, false>(s, L_E2B, V(s->e2a, 64), none, B, H2, W2, V(s->cat2, 128, 64),
                                          V(s->p2, 64));
    // BT (all 128 channels per workgroup) with U2 fused, U2 upsampled into the concatenation
    launch_c3p<64, 128, 1, 0, false, false, false, 64>(s, L_BT, V(s->p2, 64), none, B, H4, W4,
                                                       V(s->bt, 128), none, nullptr, nullptr, nullptr,
                                                       L_U2, V(s->u2lo, 64));
    hipLaunchKernelGGL(up_copy_kernel, grid1((long long)n1), dim3(256), 0, s->st, V(s->u2lo, 64), 64, B,
                       H4, W4, V(s->cat2, 128, 0));
    // D2 with U1 fused (U1 at low resolution, then upsampled into the concatenation)
    launch_c3p<128, 64, 2, 0, false, false, false, 32>(s, L_D2, V(s->cat2, 128), none, B, H2, W2,
                                                       V(s->d2, 64), none, nullptr, nullptr, nullptr,
                                                       L_U1, V(s->u1lo, 32));
    hipLaunchKernelGGL(up_copy_kernel, grid1((long long)n1 * 4), dim3(256), 0, s->st, V(s->u1lo, 32), 32, B,
                       H2, W2, V(s->cat1, 64, 0));
    launch_c3p<64, 32, 2, 0, false, false>(s, L_D1, V(s->cat1, 64), none, B, H, W, V(s->d1, 32), none);
    float *o = phi_out ? phi_out : s->out;
    hipLaunchKernelGGL(head_fwd_kernel, grid1(n1), dim3(256), 0, s->st, V(s->d1, 32),
                       s->w32 + s->woff[L_HEAD], s->w32 + s->boff[L_HEAD], phi_in, o, n1);
    if (o != s->out) {
        hipError_t e = hipMemcpyAsync(s->out, o, (size_t)n1 * 4, hipMemcpyDeviceToDevice, s->st);
        if (e != hipSuccess) return hip_fail(e, "forward copy");
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "surrogate forward");
    s->have_fwd = true;
    s->have_loss = false;
    s->last_batch = batch;
    s->last_phi = phi_in;
    return AC_OK;
}

ac_status ac_sur_infer(ac_sur *s, const float *phi_in, float *phi_out, int32_t batch) {
    g_err.clear();
    if (!s || !phi_in || !phi_out) return fail(AC_ERR_INVALID_ARG, "null handle, input or output");
    if (batch < 1 || batch > s->Bmax) return fail(AC_ERR_INVALID_ARG, "batch %d outside 1..%d", batch, s->Bmax);
    const int B = batch, H = s->H, W = s->W, H2 = H / 2, W2 = W / 2, H4 = H / 4, W4 = W / 4;
    const View none{nullptr, 0, 0};
    // first two layers in one kernel: the first layer's output is never stored.
    // The skip output goes to a dense 32-channel tensor (the e1a buffer, unused
    // here), not into the concatenation: the last layer then reads whole
    // 64-byte pixels instead of half of every 128-byte one
    launch_c3p<32, 32, 1, 0, true, false, true>(s, L_E1B, none, none, B, H, W, V(s->e1a, 32),
                                                V(s->p1, 32), phi_in);
    launch_c3p<32, 64, 1, 0, false, false>(s, L_E2A, V(s->p1, 32), none, B, H2, W2, V(s->e2a, 64), none);
    launch_c3p<64, 64, 1, 0, true, false>(s, L_E2B, V(s->e2a, 64), none, B, H2, W2, V(s->cat2, 128, 64),
                                          V(s->p2, 64));
    // BT with the decoder's 1x1 layer U2 fused (only U2's output is stored, at
    // low resolution; the next 3x3 layer reads it through the nearest upsampling)
    launch_c3p<64, 128, 1, 0, false, false, false, 64>(s, L_BT, V(s->p2, 64), none, B, H4, W4, none, none,
                                                       nullptr, nullptr, nullptr, L_U2, V(s->u2lo, 64));
    // D2 with U1 fused into its epilogue: only U1's output is stored
    launch_c3p<128, 64, 2, 64, false, false, false, 32>(s, L_D2, V(s->cat2, 128, 64), V(s->u2lo, 64), B,
                                                        H2, W2, none, none, nullptr, nullptr, nullptr,
                                                        L_U1, V(s->u1lo, 32));
    // last 3x3 layer with the head and the residual in its epilogue
    launch_c3p<64, 32, 2, 32, false, true>(s, L_D1, V(s->e1a, 32), V(s->u1lo, 32), B, H, W, none,
                                           none, phi_in, phi_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "surrogate inference");
    s->have_fwd = false;             // activations are not those of a forward for backward
    s->have_loss = false;
    return AC_OK;
}

ac_status ac_sur_loss(ac_sur *s, const float *target, int32_t batch, float *loss_dev) {
    g_err.clear();
    if (!s || !target) return fail(AC_ERR_INVALID_ARG, "null handle or target");
    if (!s->have_fwd || batch != s->last_batch)
        return fail(AC_ERR_INVALID_ARG, "ac_sur_loss needs the forward pass of the same batch first");
    const int n1 = batch * s->H * s->W;
    hipError_t e = hipMemsetAsync(s->loss, 0, 4, s->st);
    if (e != hipSuccess) return hip_fail(e, "loss reset");
    hipLaunchKernelGGL(mse_kernel, dim3(std::min(1024, (n1 + 255) / 256)), dim3(256), 0, s->st, s->out,
                       target, s->dU, n1, s->loss);
    if (loss_dev) {
        e = hipMemcpyAsync(loss_dev, s->loss, 4, hipMemcpyDeviceToDevice, s->st);
        if (e != hipSuccess) return hip_fail(e, "loss copy");
    }
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "surrogate loss");
    s->have_loss = true;
    return AC_OK;
}

ac_status ac_sur_backward(ac_sur *s, const float *dloss_dout, int32_t batch) {
    g_err.clear();
    if (!s) return fail(AC_ERR_INVALID_ARG, "null handle");
    if (dloss_dout) {
        if (!s->have_fwd || batch != s->last_batch)
            return fail(AC_ERR_INVALID_ARG, "ac_sur_backward needs the forward pass of the same batch first");
    } else if (!s->have_loss || batch != s->last_batch) {
        return fail(AC_ERR_INVALID_ARG, "ac_sur_backward needs forward and loss of the same batch first");
    }
    const int B = batch, H = s->H, W = s->W, H2 = H / 2, W2 = W / 2, H4 = H / 4, W4 = W / 4;
    const int n1 = B * H * W;
    hipError_t e = hipSuccess;
    if (dloss_dout) {
        e = hipMemcpyAsync(s->dU, dloss_dout, (size_t)n1 * 4, hipMemcpyDeviceToDevice, s->st);
        if (e != hipSuccess) return hip_fail(e, "dloss_dout copy");
        s->have_loss = false;   // dU no longer holds the stored loss gradient
    }
    e = hipMemsetAsync(s->g, 0, s->nparam * 4, s->st);
    if (e == hipSuccess) e = hipMemsetAsync(s->g_first, 0, 32 * 72 * 4, s->st);
    if (e != hipSuccess) return hip_fail(e, "grad reset");
    const View none{nullptr, 0, 0};
    // head
    hipLaunchKernelGGL(head_bwd_kernel, dim3(std::min(1024, (n1 + 255) / 256)), dim3(256), 0, s->st,
                       V(s->d1, 32), s->dU, s->w32 + s->woff[L_HEAD], n1, V(s->dd1, 32),
                       s->g + s->woff[L_HEAD], s->g + s->boff[L_HEAD]);
    // d1 = relu conv3(cat1): dZ = dd1 (masked in the head kernel)
    conv_bwd(s, L_D1, V(s->cat1, 64), V(s->dd1, 32), B, H, W, s->g + s->woff[L_D1], V(s->dcat1, 64),
             V(s->cat1, 64), 32);
    // u1 = conv1(up d2): low-resolution gradient, then the 1x1 layer
    hipLaunchKernelGGL(up_bwd_kernel, grid1((long long)n1 / 4 * 32), dim3(256), 0, s->st,
                       V(s->dcat1, 64, 0), 32, B, H2, W2, V(s->du1, 32));
    conv_bwd(s, L_U1, V(s->d2, 64), V(s->du1, 32), B, H2, W2, s->g + s->woff[L_U1], V(s->dd2, 64),
             V(s->d2, 64), 0);
    // d2 = relu conv3(cat2)
    conv_bwd(s, L_D2, V(s->cat2, 128), V(s->dd2, 64), B, H2, W2, s->g + s->woff[L_D2],
             V(s->dcat2, 128), V(s->cat2, 128), 64);
    // u2 = conv1(up bt)
    hipLaunchKernelGGL(up_bwd_kernel, grid1((long long)n1 / 16 * 64), dim3(256), 0, s->st,
                       V(s->dcat2, 128, 0), 64, B, H4, W4, V(s->du2, 64));
    conv_bwd(s, L_U2, V(s->bt, 128), V(s->du2, 64), B, H4, W4, s->g + s->woff[L_U2], V(s->dbt, 128),
             V(s->bt, 128), 0);
    // bt = relu conv3(pool e2)
    conv_bwd(s, L_BT, V(s->p2, 64), V(s->dbt, 128), B, H4, W4, s->g + s->woff[L_BT], V(s->dp2, 64),
             none, 0);
    hipLaunchKernelGGL(pool_bwd_kernel, grid1((long long)n1 / 4 * 64), dim3(256), 0, s->st,
                       V(s->dp2, 64), 64, B, H2, W2, V(s->dcat2, 128, 64), V(s->cat2, 128, 64));
    // e2 = relu conv3(e2a)
    conv_bwd(s, L_E2B, V(s->e2a, 64), V(s->dcat2, 128, 64), B, H2, W2, s->g + s->woff[L_E2B],
             V(s->de2a, 64), V(s->e2a, 64), 0);
    // e2a = relu conv3(pool e1)
    conv_bwd(s, L_E2A, V(s->p1, 32), V(s->de2a, 64), B, H2, W2, s->g + s->woff[L_E2A], V(s->dp1, 32),
             none, 0);
    hipLaunchKernelGGL(pool_bwd_kernel, grid1((long long)n1 * 32), dim3(256), 0, s->st, V(s->dp1, 32),
                       32, B, H, W, V(s->dcat1, 64, 32), V(s->cat1, 64, 32));
    // e1 = relu conv3(e1a)
    conv_bwd(s, L_E1B, V(s->e1a, 32), V(s->dcat1, 64, 32), B, H, W, s->g + s->woff[L_E1B],
             V(s->de1a, 32), V(s->e1a, 32), 0);
    // e1a = relu conv3(phi): weights only
    conv_bwd(s, L_E1A, V(s->x0, 8), V(s->de1a, 32), B, H, W, s->g_first, none, none, 0);
    hipLaunchKernelGGL(unpack_first_grad_kernel, grid1(32 * 9), dim3(256), 0, s->st, s->g_first, 32,
                       s->g + s->woff[L_E1A]);
    e = hipGetLastError();
    return e == hipSuccess ? AC_OK : hip_fail(e, "surrogate backward");
}

ac_status ac_sur_adam_step(ac_sur *s, float lr, float b1, float b2, float eps_adam, int64_t t) {
    g_err.clear();
    if (!s || t < 1 || !(lr > 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps_adam > 0))
        return fail(AC_ERR_INVALID_ARG, "bad Adam arguments");
    const float bc1 = 1.f - std::pow(b1, (float)t), bc2 = 1.f - std::pow(b2, (float)t);
    hipLaunchKernelGGL(adam_kernel, grid1(s->nparam), dim3(256), 0, s->st, s->w32, s->m, s->v, s->g,
                       (int)s->nparam, lr, b1, b2, eps_adam, bc1, bc2);
    refresh_weights(s);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? AC_OK : hip_fail(e, "adam");
}

}  // extern "C"
