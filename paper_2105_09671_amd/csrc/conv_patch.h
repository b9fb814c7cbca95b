// 3x3 convolution (replicate padding) of NHWC bf16 activations as an implicit
// GEMM whose A operand is read from an input patch staged in LDS.
//
// A workgroup of 4 waves computes an output tile of TY = 4 RW rows x 64
// columns of one image and CN output channels (blockIdx.y picks the channel
// slice; every layer here takes all its channels in one slice).  Wave w owns
// the 16-column strip 16 w .. 16 w + 15 of all TY rows: TY A fragments of 16
// pixels, times CN / 16 B fragments.
//
// K runs over 32-channel chunks of the input and, per chunk, over the 9 taps.
// For a chunk the workgroup copies the (TY + 2) x 66 pixel patch around its
// tile (rows and columns clamped to the image: the replicate padding) into
// LDS, 32 channels per pixel at a pitch of 40 bf16 (80 bytes: sixteen
// consecutive pixels of one 16-byte channel group then fall on sixteen
// disjoint 4-bank groups, so a fragment read has no bank conflict).  The
// fragment of patch row r, columns c + dx .. c + dx + 15, is at
// (r * 66 + c + dx) * 40 + 8 * (lane / 16) + ...: a per-lane base plus a
// compile-time offset, so the K loop does no address arithmetic.  Per column
// shift dx a wave reads the TY + 2 rows of its strip once and uses row i + dy
// for tile row i at each row shift dy: one read serves three taps.  B
// fragments (weights) are read from global memory in fragment order
// ([chunk][tap][16-channel tile][lane][8]; 1 KiB per wave and fragment,
// L2-resident), one or two K steps ahead of their use.
//
// Channels may come from two sources: the first LOWC channels from a tensor
// at half resolution, read at (y / 2, x / 2) (the nearest 2x upsampling of a
// decoder input, fused into the load), the rest from a full-resolution view.
//
// Epilogue: bias, relu, rounding to bf16, then the tile is staged in LDS
// (pitch CN + 8) and written with 16-byte stores; optionally also the 2 x 2
// average of the tile (the pooled input of the next level); or the decoder's
// 1x1 layer over the staged tile (UPC outputs, no activation), written at
// this resolution; or -- for the last layer, CN = 32 -- the 1x1 head and the
// residual, out = phi + hb + sum_c a_c wh_c in FP32, in channel order.
#pragma once

#include <hip/hip_runtime.h>

#include "sur_kernels.h"

namespace ac {
namespace sur {

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// float -> bf16, round to nearest even, by the hardware conversion
// (v_cvt_pk_bf16_f32): one instruction where f2bf's NaN test branches.  The
// two agree on every finite value.
__device__ __forceinline__ bf16_t f2bf_rn(float f) { return __builtin_bit_cast(bf16_t, (__bf16)f); }

constexpr int PC = 32;          // channels per patch chunk
constexpr int PP = PC + 8;      // LDS pitch of a patch pixel (bf16 units)
constexpr int PW = 66;          // patch width: 64 columns + the two pad columns

template <int RW>
constexpr int patch_lds_bytes() { return (4 * RW + 2) * PW * PP * 2; }
template <int RW, int CN>
constexpr int stage_lds_bytes() { return 4 * RW * 64 * (CN + 8) * 2; }
// Pointers of the optional prologue / epilogue stages.
struct ConvAux {
    const float *phi;      // FIRST: the FP32 state the first layer reads; HEAD: the residual
    float *out;            // HEAD: phi + U
    const float *wh, *hb;  // HEAD: 1x1 head weights [32] and bias
    const float *w1, *b1;  // FIRST: first-layer weights [32][9] (BF16 values held as FP32), bias [32]
    bf16_t *e1a;           // FIRST: if not null, the first layer's output at the tile's pixels
    const bf16_t *wu;      // UPC: the fused 1x1 layer's weights in fragment order [CN/32][1][UPC/16][64][8]
    const float *bu;       // UPC: its bias [UPC]
    View up;               // UPC: its output, [pixel][UPC] at this layer's resolution
};

// FIRST: the FP32 phi patch (TY + 4 rows x 68 columns) follows the e1a patch
template <int RW>
constexpr int phi_patch_bytes() { return (4 * RW + 4) * 68 * 4; }
template <int RW, int CN, bool FIRST = false>
constexpr int conv3p_lds_bytes() {
    return patch_lds_bytes<RW>() + (FIRST ? phi_patch_bytes<RW>() : 0) > stage_lds_bytes<RW, CN>()
               ? patch_lds_bytes<RW>() + (FIRST ? phi_patch_bytes<RW>() : 0)
               : stage_lds_bytes<RW, CN>();
}

// The FP32 phi values of a tile's (TY + 4) x 68 phi patch (rows and columns
// clamped to the image) that thread t < 204 stages: column t % 68 of rows
// t / 68 + 3 i.  Loaded one tile ahead of their use.
template <int TY>
constexpr int phi_rows() { return (TY + 4 + 2) / 3; }

template <int TY>
__device__ __forceinline__ void phi_issue(const ConvAux &aux, float (&pv)[phi_rows<TY>()], int n, int H,
                                          int W, int y0, int x0)
{
    const int t = threadIdx.x;
    if (t >= 204) return;
    const int c = t % 68, rg = t / 68;
    const float *col = aux.phi + (size_t)n * H * W + min(max(x0 - 2 + c, 0), W - 1);
#pragma unroll
    for (int i = 0; i < phi_rows<TY>(); ++i) {
        const int r = rg + 3 * i;
        if (r < TY + 4) pv[i] = col[(size_t)min(max(y0 - 2 + r, 0), H - 1) * W];
    }
}

// The patch of the first layer's output, e1a = relu(b1 + sum_tap w1[c][tap] *
// bf16(phi)[neighbour]) rounded to BF16, for (TY + 2) x 66 pixels (rows and
// columns clamped like any patch, so a pixel outside the image repeats the
// nearest one inside) and 32 channels, written at the patch pitch.  It is a
// GEMM of 32-pixel fragments on v_mfma_f32_32x32x16_bf16, computed
// transposed: A = the weights (32 channels x K), B = each pixel's 9 BF16
// neighbours of phi at K = 0..8, FP32 accumulation, then the bias.  K = 9..15
// carry zero weights (lanes 32..63 feed them taps 1..7 of the same
// neighbourhood, finite values, so no lane needs a select).  pv: the tile's
// phi values from phi_issue; the caller may reload pv once this returns.
template <int TY>
__device__ inline void first_layer_patch(const ConvAux &aux, const float (&pv)[phi_rows<TY>()],
                                         bf16_t *lds, int n, int H, int W, int y0, int x0)
{
    constexpr int PR = TY + 4, PCOL = 68, NPIX = (TY + 2) * PW, NF = (NPIX + 31) / 32;
    float *ph = reinterpret_cast<float *>(lds + (TY + 2) * PW * PP);
    const int t = threadIdx.x, lane = t & 63, w = t >> 6, l32 = lane & 31, hi = lane >> 5;
    if (t < 204) {
        const int c = t % 68, rg = t / 68;
#pragma unroll
        for (int i = 0; i < phi_rows<TY>(); ++i) {
            const int r = rg + 3 * i;
            if (r < PR) ph[r * PCOL + c] = bf2f(f2bf_rn(pv[i]));
        }
    }
    // A operand: lane supplies K = 8 hi .. 8 hi + 7 of output channel l32
    // (lanes 0..31: taps 0..7; lanes 32..63: tap 8, then zeros)
    bf16x8 wa;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int k = 8 * hi + e;
        wa[e] = k < 9 ? (__bf16)aux.w1[l32 * 9 + k] : (__bf16)0.f;
    }
    // the product's lane holds channels 8 g + 4 hi + r (g, r = 0..3) of one pixel
    float bias[4][4];
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int r = 0; r < 4; ++r) bias[g][r] = aux.b1[8 * g + 4 * hi + r];
    __syncthreads();
    for (int f = w; f < NF; f += 4) {
        const int pix = min(32 * f + l32, NPIX - 1);
        const int pr = pix / PW, pc = pix - pr * PW;
        // the pixel itself clamped to the image, in phi-patch coordinates;
        // the patch was loaded clamped, so its 3 x 3 neighbourhood there is
        // the replicate-padded one
        const int cy = min(max(y0 - 1 + pr, 0), H - 1) - (y0 - 2);
        const int cx = min(max(x0 - 1 + pc, 0), W - 1) - (x0 - 2);
        const float *nb = ph + (cy - 1) * PCOL + (cx - 1);
        bf16x8 b;
        b[0] = (__bf16)nb[hi ? 2 * PCOL + 2 : 0];
#pragma unroll
        for (int e = 1; e < 8; ++e) b[e] = (__bf16)nb[(e / 3) * PCOL + e % 3];
        floatx16 acc = {};
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa, b, acc, 0, 0, 0);
        if (32 * f + l32 < NPIX) {
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                bf16x4 o;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float v = acc[4 * g + r] + bias[g][r];
                    o[r] = (__bf16)(v > 0.f ? v : 0.f);
                }
                *reinterpret_cast<bf16x4 *>(lds + (32 * f + l32) * PP + 8 * g + 4 * hi) = o;
            }
        }
    }
    if (aux.e1a) {
        __syncthreads();
        // the tile's own pixels: patch rows 1..TY, columns 1..64
        for (int v = t; v < TY * 64 * 4; v += 256) {
            const int q = v & 3, p = v >> 2, ty = p >> 6, tx = p & 63;
            const int y = y0 + ty, x = x0 + tx;
            if (y >= H || x >= W) continue;
            *reinterpret_cast<uint4 *>(aux.e1a + ((size_t)(n * H + y) * W + x) * 32 + 8 * q) =
                *reinterpret_cast<const uint4 *>(lds + ((ty + 1) * PW + tx + 1) * PP + 8 * q);
        }
    }
}

// Row-major tile grid over B images of H x W: (image, tile row, tile column);
// consecutive workgroups take horizontally, then vertically adjacent tiles of
// one image, and with the XCD-aware numbering (xcd_tile) each XCD takes a
// contiguous band, so the halo rows two tiles share are read through one L2.
//
// FIRST: the layer's input is the first layer's output e1a = relu(conv3(phi;
// 1 -> 32)), computed into the patch from an FP32 phi patch (rounded to BF16,
// as the network's input) with FP32 sums in tap order; the first layer's
// output is then never stored unless aux.e1a asks for it (training keeps it
// for the backward pass).
// Three waves per SIMD asked of the register allocator where it fits without
// spills (not the 128-channel layer, not the training copy of the last
// layer): about 1 % faster over the forward pass than the default allocation.
// (Measured and left out: a persistent launch walking several tiles per
// workgroup, and loading the next chunk's patch into registers during the
// current chunk's taps.  The weight fragments are global loads issued a step
// ahead, and the vector-memory counter retires loads in order, so each
// step's wait for its weights also waits for the patch loads issued before
// them: neither hid the patch loads, and both cost registers.)
//
// Waves per SIMD asked of the register allocator: three for the 32- and
// 64-channel layers of 4-row tiles (the 128-channel slice and the 8-row tiles
// need more registers).
template <int CIN, int CN, int RW>
constexpr int conv3p_waves() { return CIN <= 64 && RW == 1 && CN <= 64 ? 3 : 2; }
// Slots of B fragments: step s loads step s + NSLOT - 1, so a fragment is
// requested NSLOT - 1 steps (each NI x NJ MFMAs) before its use.  One slot
// (loaded at its step) where the accumulators take 128 VGPRs, three for the
// layers with 32 input channels (registers to spare), else two
template <int CIN, int CN, int RW>
constexpr int conv3p_bslots() { return (4 * RW) * (CN / 16) >= 32 ? 1 : CIN == 32 ? 3 : 2; }

template <int CIN, int CN, int RW, int LOWC, bool POOL, bool HEAD, bool FIRST = false, int UPC = 0>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(conv3p_waves<CIN, CN, RW>())))
conv3_patch_kernel(View X, View Xlo, int B, int H, int W, const bf16_t *Wf,
                   const float *__restrict__ bias, int Cout, View Y, View P, ConvAux aux)
{
    static_assert(CIN % PC == 0 && LOWC % PC == 0 && LOWC <= CIN, "32-channel chunks");
    static_assert(!FIRST || (CIN == 32 && LOWC == 0), "the first layer has 32 outputs");
    static_assert(CN == 32 || CN == 64 || (CN == 128 && UPC > 0), "channel slice of 32 or 64 (128: with a fused 1x1)");
    static_assert(!HEAD || CN == 32, "the head needs all 32 channels of a pixel");
    static_assert(UPC == 0 || ((UPC == 32 || UPC == 64) && !HEAD && !POOL), "fused 1x1 of 32 or 64 outputs");
    constexpr int TY = 4 * RW, NI = 4 * RW, NJ = CN / 16, NCH = CIN / PC, PR = TY + 2;
    constexpr bool kTapBarrier = !FIRST && NJ < 8;
    extern __shared__ __align__(16) bf16_t lds[];
    const int tiles_x = (W + 63) >> 6, tiles_y = (H + TY - 1) / TY;
    const int tpi = tiles_y * tiles_x;
    const int ntiles = B * tpi;
    const int tile = xcd_tile(ntiles);
    if (tile >= ntiles) return;                      // padding workgroup (whole group)
    const int n = tile / tpi, rem = tile - n * tpi;
    const int y0 = (rem / tiles_x) * TY, x0 = (rem % tiles_x) * 64;
    const int n0 = blockIdx.y * CN;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int lr = lane & 15, lq = lane >> 4;

    // wave w owns the 16-column strip 16 w .. 16 w + 15 of all TY tile rows:
    // fragment i = tile row i.  Per-lane A base of patch row 0, bf16 units; the
    // fragment of patch row r shifted by dx columns is at fbase + (r PW + dx) PP
    const int fbase = (16 * w + lr) * PP + 8 * lq;
    // B fragment (chunk, tap, j) of this workgroup's channel slice: lane's 16
    // bytes at Wf + (((chunk * 9 + tap) * (Cout / 16) + n0 / 16 + j) * 64 + lane) * 8;
    // the step part is uniform (scalar arithmetic), the lane part a fixed
    // 32-bit offset
    const int ntile16 = Cout >> 4;
    const bf16_t *wslice = Wf + (size_t)(n0 >> 4) * 512;
    const int wl = lane * 8;
    // K steps run chunk by chunk, per chunk column shift dx by dx and per dx
    // row shift dy by dy: step q is tap 3 dy + dx of chunk q / 9
    auto loadB = [&](int q, bf16x8 (&dst)[NJ]) __attribute__((always_inline)) {
        const int ch = q / 9, dx = (q % 9) / 3, dy = q % 3;
        const bf16_t *wb = wslice + (size_t)(ch * 9 + 3 * dy + dx) * ntile16 * 512;
#pragma unroll
        for (int j = 0; j < NJ; ++j) dst[j] = *reinterpret_cast<const bf16x8 *>(wb + j * 512 + wl);
    };

    // patch copy: in every patch row, lanes 16 k .. 16 k + 15 of wave w move
    // 16-byte group k of patch columns 16 w .. 16 w + 15 (sixteen consecutive
    // pixels of one group per quarter-wave, as the fragment reads: no bank
    // conflict at the 80-byte pitch); threads 0 .. 8 (TY + 2) - 1 also move
    // the two columns beyond.  issue() loads a chunk's rows into registers,
    // commit() writes them to LDS.
    const int pq = (t >> 4) & 3, pcol = (t & 15) + 16 * w;
    const int ex_q = t & 3, ex_r = t >> 3, ex_c = 64 + ((t >> 2) & 1);
    const bool ex = ex_r < PR;
    u32x4 val[FIRST ? 1 : PR], vex = {};
    float pv[phi_rows<TY>()];
    auto issue = [&](int ch) __attribute__((always_inline)) {
        if constexpr (FIRST) {
            phi_issue<TY>(aux, pv, n, H, W, y0, x0);
        } else {
            const bool low = ch * PC < LOWC;
            const View S = low ? Xlo : X;
            const int cofs = low ? ch * PC : ch * PC - LOWC;
            const int Hs = low ? (H >> 1) : H, Ws = low ? (W >> 1) : W;
            const bf16_t *img = S.p + (size_t)n * Hs * Ws * S.Cs + S.Co + cofs + 8 * pq;
            int gx = min(max(x0 - 1 + pcol, 0), W - 1);
            if (low) gx >>= 1;
#pragma unroll
            for (int pr = 0; pr < PR; ++pr) {
                int gy = min(max(y0 - 1 + pr, 0), H - 1);
                if (low) gy >>= 1;
                val[pr] = *reinterpret_cast<const u32x4 *>(img + ((size_t)gy * Ws + gx) * S.Cs);
            }
            if (ex) {
                int gy = min(max(y0 - 1 + ex_r, 0), H - 1), gxe = min(max(x0 - 1 + ex_c, 0), W - 1);
                if (low) { gy >>= 1; gxe >>= 1; }
                vex = *reinterpret_cast<const u32x4 *>(img + 8 * (ex_q - pq) + ((size_t)gy * Ws + gxe) * S.Cs);
            }
        }
    };
    auto commit = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int pr = 0; pr < PR; ++pr)
            *reinterpret_cast<u32x4 *>(lds + (pr * PW + pcol) * PP + 8 * pq) = val[pr];
        if (ex) *reinterpret_cast<u32x4 *>(lds + (ex_r * PW + ex_c) * PP + 8 * ex_q) = vex;
    };

    floatx4 acc[NI][NJ] = {};
    // NSLOT slots of B fragments: K step s (over all chunks) uses slot s %
    // NSLOT and loads step s + NSLOT - 1 into a free one; the chunk loop is
    // unrolled (at most 4 chunks), so every slot index is static and
    // nothing is copied
    constexpr int NSLOT = conv3p_bslots<CIN, CN, RW>();
    bf16x8 bq[NSLOT][NJ];
#pragma unroll
    for (int q = 0; q + 1 < NSLOT; ++q) loadB(q, bq[q]);
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
        // ---- stage the patch of this 32-channel chunk (clamped = replicate
        // pad) once every wave is done with the LDS
        if (ch > 0) __syncthreads();
        issue(ch);
        if constexpr (FIRST) first_layer_patch<TY>(aux, pv, lds, n, H, W, y0, x0);
        else commit();
        __syncthreads();
        // ---- 9 taps of this chunk.  Per column shift dx the wave reads the
        // TY + 2 patch rows of its strip once; tile row i takes tap (dy, dx)
        // from patch row i + dy, so each fragment read serves three taps
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
            bf16x8 a[TY + 2];
#pragma unroll
            for (int r = 0; r < TY + 2; ++r)
                a[r] = *reinterpret_cast<const bf16x8 *>(lds + fbase + (r * PW + dx) * PP);
#pragma unroll
            for (int dy = 0; dy < 3; ++dy) {
                const int step = ch * 9 + 3 * dx + dy;
                if (step + NSLOT - 1 < NCH * 9) loadB(step + NSLOT - 1, bq[(step + NSLOT - 1) % NSLOT]);
#pragma unroll
                for (int i = 0; i < NI; ++i)
#pragma unroll
                    for (int j = 0; j < NJ; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bq[step % NSLOT][j], a[i + dy],
                                                                             acc[i][j], 0, 0, 0);
                // the 128-channel layers: keep each tap's loads within the
                // tap, or the scheduler's early loads spill
                if constexpr (kTapBarrier) __builtin_amdgcn_sched_barrier(0);
            }
        }
    }

    // ---- epilogue: bias + relu -> bf16, staged in LDS as [pixel][CN].  The
    // products are computed transposed (weights as the MFMA's A operand), so
    // a lane holds 4 consecutive channels 16 j + 4 (lane / 16) + r of one
    // pixel: one 8-byte LDS write per fragment
    __syncthreads();                             // the patch is dead
    constexpr int SP = CN + 8;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int c0 = 16 * j + 4 * lq;
        float bv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) bv[r] = bias[n0 + c0 + r];
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int pix = i * 64 + 16 * w + lr;
            bf16x4 o;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float v = acc[i][j][r] + bv[r];
                o[r] = (__bf16)(v > 0.f ? v : 0.f);
            }
            *reinterpret_cast<bf16x4 *>(lds + pix * SP + c0) = o;
        }
    }
    __syncthreads();
    if constexpr (HEAD) {
        // one thread per pixel: out = phi + (hb + sum_c a_c wh_c), c in order
        for (int pix = t; pix < TY * 64; pix += 256) {
            const int y = y0 + (pix >> 6), x = x0 + (pix & 63);
            if (y >= H || x >= W) continue;
            const bf16_t *a = lds + pix * SP;
            float s = aux.hb[0];
#pragma unroll
            for (int c = 0; c < 32; ++c) s += bf2f(a[c]) * aux.wh[c];
            const size_t g = (size_t)(n * H + y) * W + x;
            aux.out[g] = aux.phi[g] + s;
        }
    } else {
        if constexpr (UPC > 0) {
            // the decoder's 1x1 layer fused: out[pix][co] = bu[co] + sum_c
            // a[pix][c] wu[co][c] over this layer's CN outputs (the whole
            // layer: one channel slice), FP32 sums, no activation.  Wave w
            // takes the pixels it produced; transposed products again, so a
            // lane ends with 4 consecutive outputs of one pixel
            constexpr int UJ = UPC / 16, UK = CN / 32;
            floatx4 u[NI][UJ] = {};
#pragma unroll
            for (int ks = 0; ks < UK; ++ks) {
                bf16x8 wq[UJ];
#pragma unroll
                for (int j = 0; j < UJ; ++j)
                    wq[j] = *reinterpret_cast<const bf16x8 *>(aux.wu + ((ks * UJ + j) * 64 + lane) * 8);
#pragma unroll
                for (int i = 0; i < NI; ++i) {
                    const int pix = i * 64 + 16 * w + lr;
                    const bf16x8 a = *reinterpret_cast<const bf16x8 *>(lds + pix * SP + 32 * ks + 8 * lq);
#pragma unroll
                    for (int j = 0; j < UJ; ++j)
                        u[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wq[j], a, u[i][j], 0, 0, 0);
                }
            }
#pragma unroll
            for (int j = 0; j < UJ; ++j) {
                const int c0 = 16 * j + 4 * lq;
                float bv[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) bv[r] = aux.bu[c0 + r];
#pragma unroll
                for (int i = 0; i < NI; ++i) {
                    const int y = y0 + i, x = x0 + 16 * w + lr;
                    if (y >= H || x >= W) continue;
                    bf16x4 o;
#pragma unroll
                    for (int r = 0; r < 4; ++r) o[r] = (__bf16)(u[i][j][r] + bv[r]);
                    *reinterpret_cast<bf16x4 *>(aux.up.p + ((size_t)(n * H + y) * W + x) * aux.up.Cs +
                                                aux.up.Co + c0) = o;
                }
            }
        }
        constexpr int CQ = CN / 8;               // 16-byte groups per pixel
        // consecutive lanes write consecutive 16-byte groups of a pixel
        // (whole 64- or 128-byte pixel rows per lane group: measured faster
        // than the LDS-conflict-free order of sixteen pixels per quarter-wave).
        // With a fused 1x1 layer the 3x3 output itself is optional (Y.p null)
        for (int v = t; (UPC == 0 || Y.p) && v < TY * 64 * CQ; v += 256) {
            const int q = v % CQ, pix = v / CQ;
            const int y = y0 + pix / 64, x = x0 + (pix & 63);
            if (y >= H || x >= W) continue;
            *reinterpret_cast<uint4 *>(Y.p + ((size_t)(n * H + y) * W + x) * Y.Cs + Y.Co + n0 + 8 * q) =
                *reinterpret_cast<const uint4 *>(lds + pix * SP + 8 * q);
        }
        if constexpr (POOL) {
            // 2 x 2 averages of the tile (TY and the tile origin are even),
            // summed in the order (y, x), (y, x+1), (y+1, x), (y+1, x+1) like
            // pool_kernel
            const int Ho = H >> 1, Wo = W >> 1;
            for (int v = t; v < (TY / 2) * 32 * CQ; v += 256) {
                const int q = v % CQ, pp = v / CQ, py = pp / 32, px = pp % 32;
                const int oy = (y0 >> 1) + py, ox = (x0 >> 1) + px;
                if (oy >= Ho || ox >= Wo) continue;
                float s[8] = {};
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    const int pix = (2 * py + (d >> 1)) * 64 + 2 * px + (d & 1);
                    const uint4 u = *reinterpret_cast<const uint4 *>(lds + pix * SP + 8 * q);
                    const bf16_t *e = reinterpret_cast<const bf16_t *>(&u);
#pragma unroll
                    for (int k = 0; k < 8; ++k) s[k] += bf2f(e[k]);
                }
                uint4 o;
                bf16_t *oe = reinterpret_cast<bf16_t *>(&o);
#pragma unroll
                for (int k = 0; k < 8; ++k) oe[k] = f2bf_rn(0.25f * s[k]);
                *reinterpret_cast<uint4 *>(P.p + ((size_t)(n * Ho + oy) * Wo + ox) * P.Cs + P.Co + n0 + 8 * q) = o;
            }
        }
    }
}

// FP32 canonical weights [Cout][k][k][Cin] (taps = k * k = 9 or 1) -> bf16
// fragment order [Cin/32][taps][Cout/16][64 lanes][8]: lane l of tile (chunk,
// tap, jt) holds output channel 16 jt + l % 16, input channels 32 chunk +
// 8 (l / 16) .. + 7.
__global__ void pack_frag_weights_kernel(const float *w, int Cout, int taps, int Cin, bf16_t *out)
{
    const int total = Cout * taps * Cin;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const int e = i & 7, lane = (i >> 3) & 63, rest = i >> 9;
        const int jt = rest % (Cout >> 4), r2 = rest / (Cout >> 4), tap = r2 % taps, chunk = r2 / taps;
        const int co = 16 * jt + (lane & 15), ci = 32 * chunk + 8 * (lane >> 4) + e;
        out[i] = f2bf(w[((size_t)co * taps + tap) * Cin + ci]);
    }
}

}  // namespace sur
}  // namespace ac
