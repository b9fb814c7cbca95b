/*
 * FP64 CPU oracle of the learned K-step surrogate network.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite (and the smoke check),
 * never by the product library; it shares no code with the GPU kernels.
 *
 * The surrogate is not in the paper; its definition here is the specification
 * the GPU kernels are checked against:
 *
 *   input  phi  [B][H][W]            (one channel)
 *   e1a = relu(conv3(phi;  1 -> c1))         H x W
 *   e1  = relu(conv3(e1a;  c1 -> c1))        H x W
 *   e2a = relu(conv3(pool(e1); c1 -> c2))    H/2
 *   e2  = relu(conv3(e2a;  c2 -> c2))        H/2
 *   bt  = relu(conv3(pool(e2); c2 -> c3))    H/4
 *   u2  = conv1(up(bt); c3 -> c2)            H/2
 *   d2  = relu(conv3(cat(u2, e2); 2c2 -> c2))
 *   u1  = conv1(up(d2); c2 -> c1)            H
 *   d1  = relu(conv3(cat(u1, e1); 2c1 -> c1))
 *   U   = conv1(d1; c1 -> 1)
 *   out = phi + U
 *
 * conv3: 3x3 cross-correlation with bias and replicate padding (an index
 * outside the image is clamped to the nearest row/column, the discrete
 * counterpart of the zero-Neumann boundary); conv1: 1x1 with bias; pool: 2x2
 * average; up: 2x nearest-neighbour; cat: channel concatenation, first operand
 * first.  Loss = mean over B*H*W of (out - target)^2.
 *
 * Parameters, flat, layer by layer in the order above: weights [Cout][3][3][Cin]
 * (conv3) or [Cout][Cin] (conv1), then bias [Cout].
 *
 * Layout here: [B][C][H][W] doubles.  Backward propagation is the plain
 * adjoint of each loop: a clamped read x[clamp(i)] in the forward pass becomes
 * an accumulation into dx[clamp(i)].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int cin, cout, k; /* k = 3 or 1 */
} layer_t;

enum { L_E1A, L_E1B, L_E2A, L_E2B, L_BT, L_U2, L_D2, L_U1, L_D1, L_HEAD, NL };

static void layers(int c1, int c2, int c3, layer_t *L) {
    L[L_E1A] = (layer_t){1, c1, 3};
    L[L_E1B] = (layer_t){c1, c1, 3};
    L[L_E2A] = (layer_t){c1, c2, 3};
    L[L_E2B] = (layer_t){c2, c2, 3};
    L[L_BT] = (layer_t){c2, c3, 3};
    L[L_U2] = (layer_t){c3, c2, 1};
    L[L_D2] = (layer_t){2 * c2, c2, 3};
    L[L_U1] = (layer_t){c2, c1, 1};
    L[L_D1] = (layer_t){2 * c1, c1, 3};
    L[L_HEAD] = (layer_t){c1, 1, 1};
}

static int64_t layer_size(layer_t l) { return (int64_t)l.cout * l.k * l.k * l.cin + l.cout; }

int64_t sur_num_params(int c1, int c2, int c3) {
    layer_t L[NL];
    layers(c1, c2, c3, L);
    int64_t n = 0;
    for (int i = 0; i < NL; ++i) n += layer_size(L[i]);
    return n;
}

static inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

#define AT(a, C, H, W, b, c, y, x) (a)[(((size_t)(b) * (C) + (c)) * (H) + (y)) * (W) + (x)]

/* y = conv(x) + bias; 3x3 with replicate padding, or 1x1 */
static void conv_fwd(const double *x, int B, int Cin, int H, int W, const double *w,
                     const double *bias, int Cout, int k, double *y) {
    for (int b = 0; b < B; ++b)
        for (int co = 0; co < Cout; ++co)
            for (int i = 0; i < H; ++i)
                for (int j = 0; j < W; ++j) {
                    double s = bias[co];
                    for (int ky = 0; ky < k; ++ky)
                        for (int kx = 0; kx < k; ++kx)
                            for (int ci = 0; ci < Cin; ++ci) {
                                const int yi = k == 3 ? clampi(i + ky - 1, 0, H - 1) : i;
                                const int xj = k == 3 ? clampi(j + kx - 1, 0, W - 1) : j;
                                s += w[((co * k + ky) * k + kx) * Cin + ci] *
                                     AT(x, Cin, H, W, b, ci, yi, xj);
                            }
                    AT(y, Cout, H, W, b, co, i, j) = s;
                }
}

/* adjoint of conv_fwd: dx += ..., dw += ..., db += ... */
static void conv_bwd(const double *x, int B, int Cin, int H, int W, const double *w, int Cout,
                     int k, const double *dy, double *dx, double *dw, double *db) {
    for (int b = 0; b < B; ++b)
        for (int co = 0; co < Cout; ++co)
            for (int i = 0; i < H; ++i)
                for (int j = 0; j < W; ++j) {
                    const double g = AT(dy, Cout, H, W, b, co, i, j);
                    db[co] += g;
                    for (int ky = 0; ky < k; ++ky)
                        for (int kx = 0; kx < k; ++kx)
                            for (int ci = 0; ci < Cin; ++ci) {
                                const int yi = k == 3 ? clampi(i + ky - 1, 0, H - 1) : i;
                                const int xj = k == 3 ? clampi(j + kx - 1, 0, W - 1) : j;
                                const size_t wi = ((size_t)(co * k + ky) * k + kx) * Cin + ci;
                                dw[wi] += g * AT(x, Cin, H, W, b, ci, yi, xj);
                                if (dx) AT(dx, Cin, H, W, b, ci, yi, xj) += g * w[wi];
                            }
                }
}

static void relu(double *a, size_t n) {
    for (size_t i = 0; i < n; ++i) a[i] = a[i] > 0 ? a[i] : 0;
}
/* dz = dy * [y > 0], y the relu output */
static void relu_bwd(const double *y, double *d, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!(y[i] > 0)) d[i] = 0;
}

static void pool_fwd(const double *x, int B, int C, int H, int W, double *y) {
    for (int b = 0; b < B; ++b)
        for (int c = 0; c < C; ++c)
            for (int i = 0; i < H / 2; ++i)
                for (int j = 0; j < W / 2; ++j)
                    AT(y, C, H / 2, W / 2, b, c, i, j) =
                        0.25 * (AT(x, C, H, W, b, c, 2 * i, 2 * j) + AT(x, C, H, W, b, c, 2 * i, 2 * j + 1) +
                                AT(x, C, H, W, b, c, 2 * i + 1, 2 * j) +
                                AT(x, C, H, W, b, c, 2 * i + 1, 2 * j + 1));
}
static void pool_bwd(const double *dy, int B, int C, int H, int W, double *dx) {
    for (int b = 0; b < B; ++b)
        for (int c = 0; c < C; ++c)
            for (int i = 0; i < H; ++i)
                for (int j = 0; j < W; ++j)
                    AT(dx, C, H, W, b, c, i, j) += 0.25 * AT(dy, C, H / 2, W / 2, b, c, i / 2, j / 2);
}
/* nearest 2x: y[i][j] = x[i/2][j/2]; H, W are the low-resolution sizes */
static void up_fwd(const double *x, int B, int C, int H, int W, double *y) {
    for (int b = 0; b < B; ++b)
        for (int c = 0; c < C; ++c)
            for (int i = 0; i < 2 * H; ++i)
                for (int j = 0; j < 2 * W; ++j)
                    AT(y, C, 2 * H, 2 * W, b, c, i, j) = AT(x, C, H, W, b, c, i / 2, j / 2);
}
static void up_bwd(const double *dy, int B, int C, int H, int W, double *dx) {
    for (int b = 0; b < B; ++b)
        for (int c = 0; c < C; ++c)
            for (int i = 0; i < 2 * H; ++i)
                for (int j = 0; j < 2 * W; ++j)
                    AT(dx, C, H, W, b, c, i / 2, j / 2) += AT(dy, C, 2 * H, 2 * W, b, c, i, j);
}
/* z = cat(a, b) along channels */
static void cat_fwd(const double *a, int Ca, const double *bb, int Cb, int B, int HW, double *z) {
    for (int b = 0; b < B; ++b) {
        memcpy(z + (size_t)b * (Ca + Cb) * HW, a + (size_t)b * Ca * HW, sizeof(double) * Ca * HW);
        memcpy(z + ((size_t)b * (Ca + Cb) + Ca) * HW, bb + (size_t)b * Cb * HW, sizeof(double) * Cb * HW);
    }
}
static void cat_bwd(const double *dz, int Ca, int Cb, int B, int HW, double *da, double *db) {
    for (int b = 0; b < B; ++b)
        for (size_t i = 0; i < (size_t)Ca * HW; ++i) da[(size_t)b * Ca * HW + i] += dz[(size_t)b * (Ca + Cb) * HW + i];
    for (int b = 0; b < B; ++b)
        for (size_t i = 0; i < (size_t)Cb * HW; ++i)
            db[(size_t)b * Cb * HW + i] += dz[((size_t)b * (Ca + Cb) + Ca) * HW + i];
}

typedef struct {
    int B, H, W, c1, c2, c3;
    double *e1a, *e1, *p1, *e2a, *e2, *p2, *bt, *ub, *u2, *cat2, *d2, *ud, *u1, *cat1, *d1, *U;
} acts_t;

static double *zalloc(size_t n) { return (double *)calloc(n ? n : 1, sizeof(double)); }

static int acts_alloc(acts_t *a, int B, int H, int W, int c1, int c2, int c3) {
    const size_t n1 = (size_t)B * H * W, n2 = n1 / 4, n3 = n1 / 16;
    a->B = B; a->H = H; a->W = W; a->c1 = c1; a->c2 = c2; a->c3 = c3;
    a->e1a = zalloc(n1 * c1); a->e1 = zalloc(n1 * c1); a->p1 = zalloc(n2 * c1);
    a->e2a = zalloc(n2 * c2); a->e2 = zalloc(n2 * c2); a->p2 = zalloc(n3 * c2);
    a->bt = zalloc(n3 * c3); a->ub = zalloc(n2 * c3); a->u2 = zalloc(n2 * c2);
    a->cat2 = zalloc(n2 * 2 * c2); a->d2 = zalloc(n2 * c2); a->ud = zalloc(n1 * c2);
    a->u1 = zalloc(n1 * c1); a->cat1 = zalloc(n1 * 2 * c1); a->d1 = zalloc(n1 * c1);
    a->U = zalloc(n1);
    return a->e1a && a->e1 && a->p1 && a->e2a && a->e2 && a->p2 && a->bt && a->ub && a->u2 &&
           a->cat2 && a->d2 && a->ud && a->u1 && a->cat1 && a->d1 && a->U;
}

static void acts_free(acts_t *a) {
    double *p[] = {a->e1a, a->e1, a->p1, a->e2a, a->e2, a->p2, a->bt, a->ub, a->u2,
                   a->cat2, a->d2, a->ud, a->u1, a->cat1, a->d1, a->U};
    for (unsigned i = 0; i < sizeof p / sizeof p[0]; ++i) free(p[i]);
}

static void offsets(const layer_t *L, int64_t *wo, int64_t *bo) {
    int64_t o = 0;
    for (int i = 0; i < NL; ++i) {
        wo[i] = o;
        o += (int64_t)L[i].cout * L[i].k * L[i].k * L[i].cin;
        bo[i] = o;
        o += L[i].cout;
    }
}

static void forward(const double *w, const layer_t *L, const double *phi, acts_t *a) {
    int64_t wo[NL], bo[NL];
    offsets(L, wo, bo);
    const int B = a->B, H = a->H, W = a->W, c1 = a->c1, c2 = a->c2, c3 = a->c3;
    const int H2 = H / 2, W2 = W / 2, H4 = H / 4, W4 = W / 4;
    conv_fwd(phi, B, 1, H, W, w + wo[L_E1A], w + bo[L_E1A], c1, 3, a->e1a);
    relu(a->e1a, (size_t)B * c1 * H * W);
    conv_fwd(a->e1a, B, c1, H, W, w + wo[L_E1B], w + bo[L_E1B], c1, 3, a->e1);
    relu(a->e1, (size_t)B * c1 * H * W);
    pool_fwd(a->e1, B, c1, H, W, a->p1);
    conv_fwd(a->p1, B, c1, H2, W2, w + wo[L_E2A], w + bo[L_E2A], c2, 3, a->e2a);
    relu(a->e2a, (size_t)B * c2 * H2 * W2);
    conv_fwd(a->e2a, B, c2, H2, W2, w + wo[L_E2B], w + bo[L_E2B], c2, 3, a->e2);
    relu(a->e2, (size_t)B * c2 * H2 * W2);
    pool_fwd(a->e2, B, c2, H2, W2, a->p2);
    conv_fwd(a->p2, B, c2, H4, W4, w + wo[L_BT], w + bo[L_BT], c3, 3, a->bt);
    relu(a->bt, (size_t)B * c3 * H4 * W4);
    up_fwd(a->bt, B, c3, H4, W4, a->ub);
    conv_fwd(a->ub, B, c3, H2, W2, w + wo[L_U2], w + bo[L_U2], c2, 1, a->u2);
    cat_fwd(a->u2, c2, a->e2, c2, B, H2 * W2, a->cat2);
    conv_fwd(a->cat2, B, 2 * c2, H2, W2, w + wo[L_D2], w + bo[L_D2], c2, 3, a->d2);
    relu(a->d2, (size_t)B * c2 * H2 * W2);
    up_fwd(a->d2, B, c2, H2, W2, a->ud);
    conv_fwd(a->ud, B, c2, H, W, w + wo[L_U1], w + bo[L_U1], c1, 1, a->u1);
    cat_fwd(a->u1, c1, a->e1, c1, B, H * W, a->cat1);
    conv_fwd(a->cat1, B, 2 * c1, H, W, w + wo[L_D1], w + bo[L_D1], c1, 3, a->d1);
    relu(a->d1, (size_t)B * c1 * H * W);
    conv_fwd(a->d1, B, c1, H, W, w + wo[L_HEAD], w + bo[L_HEAD], 1, 1, a->U);
}

/* out = phi + U.  Returns 0, or -1 on bad sizes / allocation failure. */
int sur_forward(const double *w, int c1, int c2, int c3, const double *phi, int B, int H, int W,
                double *out) {
    if (B < 1 || H < 4 || W < 4 || H % 4 || W % 4) return -1;
    layer_t L[NL];
    layers(c1, c2, c3, L);
    acts_t a;
    if (!acts_alloc(&a, B, H, W, c1, c2, c3)) { acts_free(&a); return -1; }
    forward(w, L, phi, &a);
    for (size_t i = 0; i < (size_t)B * H * W; ++i) out[i] = phi[i] + a.U[i];
    acts_free(&a);
    return 0;
}

/* loss = mean (phi + U - target)^2; grad (size sur_num_params) = d loss / d w. */
int sur_loss_grad(const double *w, int c1, int c2, int c3, const double *phi,
                  const double *target, int B, int H, int W, double *loss, double *grad) {
    if (B < 1 || H < 4 || W < 4 || H % 4 || W % 4) return -1;
    layer_t L[NL];
    layers(c1, c2, c3, L);
    int64_t wo[NL], bo[NL];
    offsets(L, wo, bo);
    acts_t a, g;
    if (!acts_alloc(&a, B, H, W, c1, c2, c3) || !acts_alloc(&g, B, H, W, c1, c2, c3)) {
        acts_free(&a);
        acts_free(&g);
        return -1;
    }
    forward(w, L, phi, &a);
    const size_t n1 = (size_t)B * H * W;
    const int H2 = H / 2, W2 = W / 2, H4 = H / 4, W4 = W / 4;
    double l = 0;
    for (size_t i = 0; i < n1; ++i) {
        const double r = phi[i] + a.U[i] - target[i];
        l += r * r;
        g.U[i] = 2.0 * r / (double)n1;
    }
    *loss = l / (double)n1;
    memset(grad, 0, sizeof(double) * (size_t)sur_num_params(c1, c2, c3));
    /* head */
    conv_bwd(a.d1, B, c1, H, W, w + wo[L_HEAD], 1, 1, g.U, g.d1, grad + wo[L_HEAD], grad + bo[L_HEAD]);
    relu_bwd(a.d1, g.d1, n1 * c1);
    conv_bwd(a.cat1, B, 2 * c1, H, W, w + wo[L_D1], c1, 3, g.d1, g.cat1, grad + wo[L_D1], grad + bo[L_D1]);
    cat_bwd(g.cat1, c1, c1, B, H * W, g.u1, g.e1);
    conv_bwd(a.ud, B, c2, H, W, w + wo[L_U1], c1, 1, g.u1, g.ud, grad + wo[L_U1], grad + bo[L_U1]);
    up_bwd(g.ud, B, c2, H2, W2, g.d2);
    relu_bwd(a.d2, g.d2, n1 / 4 * c2);
    conv_bwd(a.cat2, B, 2 * c2, H2, W2, w + wo[L_D2], c2, 3, g.d2, g.cat2, grad + wo[L_D2], grad + bo[L_D2]);
    cat_bwd(g.cat2, c2, c2, B, H2 * W2, g.u2, g.e2);
    conv_bwd(a.ub, B, c3, H2, W2, w + wo[L_U2], c2, 1, g.u2, g.ub, grad + wo[L_U2], grad + bo[L_U2]);
    up_bwd(g.ub, B, c3, H4, W4, g.bt);
    relu_bwd(a.bt, g.bt, n1 / 16 * c3);
    conv_bwd(a.p2, B, c2, H4, W4, w + wo[L_BT], c3, 3, g.bt, g.p2, grad + wo[L_BT], grad + bo[L_BT]);
    pool_bwd(g.p2, B, c2, H2, W2, g.e2);
    relu_bwd(a.e2, g.e2, n1 / 4 * c2);
    conv_bwd(a.e2a, B, c2, H2, W2, w + wo[L_E2B], c2, 3, g.e2, g.e2a, grad + wo[L_E2B], grad + bo[L_E2B]);
    relu_bwd(a.e2a, g.e2a, n1 / 4 * c2);
    conv_bwd(a.p1, B, c1, H2, W2, w + wo[L_E2A], c2, 3, g.e2a, g.p1, grad + wo[L_E2A], grad + bo[L_E2A]);
    pool_bwd(g.p1, B, c1, H, W, g.e1);
    relu_bwd(a.e1, g.e1, n1 * c1);
    conv_bwd(a.e1a, B, c1, H, W, w + wo[L_E1B], c1, 3, g.e1, g.e1a, grad + wo[L_E1B], grad + bo[L_E1B]);
    relu_bwd(a.e1a, g.e1a, n1 * c1);
    conv_bwd(phi, B, 1, H, W, w + wo[L_E1A], c1, 3, g.e1a, NULL, grad + wo[L_E1A], grad + bo[L_E1A]);
    acts_free(&a);
    acts_free(&g);
    return 0;
}

/* single-layer entry points, for checks of the building blocks */
void sur_conv_fwd(const double *x, int B, int Cin, int H, int W, const double *w,
                  const double *bias, int Cout, int k, double *y) {
    conv_fwd(x, B, Cin, H, W, w, bias, Cout, k, y);
}
void sur_pool_fwd(const double *x, int B, int C, int H, int W, double *y) { pool_fwd(x, B, C, H, W, y); }
void sur_up_fwd(const double *x, int B, int C, int H, int W, double *y) { up_fwd(x, B, C, H, W, y); }
