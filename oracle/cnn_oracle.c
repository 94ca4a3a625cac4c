/*
 * Reference oracle for the learned scorer: a 1-D convolutional network over
 * noise-normalised folded light curves (Sec. 2.5 describes the paper's CNN:
 * circular convolutions, max-pooling, fully connected layers with ReLU, a
 * sigmoid output, cross-entropy trained with Adam). The layer sizes are the
 * configured ones: four blocks of [circular conv1d, kernel 5 -> ReLU ->
 * max-pool 2] with 1->16->32->64->64 channels over 256 -> 16 positions, then
 * fully connected 1024 -> 256 -> 64 -> 1 with ReLU between, sigmoid output.
 *
 * TEST INFRASTRUCTURE ONLY: plain FP64 forward, backward and Adam, shared
 * with nothing in the GPU library. Compiled with -ffp-contract=off.
 *
 * Parameter vector (canonical layout, 312,449 values):
 *   conv l weight [Cout][Cin][5] then bias [Cout], l = 1..4;
 *   fc1 weight [256][1024], bias [256]; fc2 [64][256], [64]; fc3 [1][64], [1].
 * The flatten after block 4 is channel-major: index = channel * 16 + position.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NP 312449

static const int CH[5] = {1, 16, 32, 64, 64};
static const int LEN[5] = {256, 128, 64, 32, 16};   /* input length of block l is LEN[l-1] */

static int64_t conv_w_off(int l) {
    static const int64_t off[5] = {0, 0, 96, 2688, 12992};
    return off[l];
}
static int64_t conv_b_off(int l) { return conv_w_off(l) + (int64_t)CH[l] * CH[l - 1] * 5; }
#define F1W 33536
#define F1B 295680
#define F2W 295936
#define F2B 312320
#define F3W 312384
#define F3B 312448

int64_t oracle_cnn_nparams(void) { return NP; }

/*
 * Circular 1-D convolution (cross-correlation, padding 2 each side by
 * wrap-around because phase is periodic):
 *   y[b][co][x] = bias[co] + sum_ci sum_dx w[co][ci][dx] * in[b][ci][(x+dx-2) mod L]
 */
void oracle_conv1d_circ(const double *in, const double *w, const double *bias, int B, int Cin,
                        int Cout, int L, double *y) {
    for (int b = 0; b < B; ++b)
        for (int co = 0; co < Cout; ++co)
            for (int x = 0; x < L; ++x) {
                double s = bias ? bias[co] : 0.0;
                for (int ci = 0; ci < Cin; ++ci)
                    for (int dx = 0; dx < 5; ++dx) {
                        int p = ((x + dx - 2) % L + L) % L;
                        s += w[((int64_t)co * Cin + ci) * 5 + dx] * in[((int64_t)b * Cin + ci) * L + p];
                    }
                y[((int64_t)b * Cout + co) * L + x] = s;
            }
}

/* Max-pool by 2: out[x] = max(r[2x], r[2x+1]); idx[x] = the winner, the first on a tie. */
void oracle_maxpool2(const double *r, int n_out, double *out, int32_t *idx) {
    for (int x = 0; x < n_out; ++x) {
        int w = r[2 * x] >= r[2 * x + 1] ? 2 * x : 2 * x + 1;
        out[x] = r[w];
        idx[x] = w;
    }
}

static double relu(double v) { return v > 0.0 ? v : 0.0; }

/* Per-sample forward storage. */
typedef struct {
    double pre[5][64 * 256];   /* conv pre-activations, block l: [C_l][LEN[l-1]] */
    double act[5][64 * 256];   /* act[0] = input; act[l] = pooled output [C_l][LEN[l]] */
    int32_t arg[5][64 * 128];  /* pooling winner positions */
    double h1pre[256], h1[256], h2pre[64], h2[64];
    double z;
} Fwd;

static void forward_one(const double *p, const double *x, Fwd *f) {
    memcpy(f->act[0], x, sizeof(double) * 256);
    for (int l = 1; l <= 4; ++l) {
        const int Cin = CH[l - 1], Cout = CH[l], L = LEN[l - 1];
        oracle_conv1d_circ(f->act[l - 1], p + conv_w_off(l), p + conv_b_off(l), 1, Cin, Cout, L,
                           f->pre[l]);
        double r[256];
        for (int c = 0; c < Cout; ++c) {
            for (int xx = 0; xx < L; ++xx) r[xx] = relu(f->pre[l][c * L + xx]);
            oracle_maxpool2(r, L / 2, f->act[l] + c * (L / 2), f->arg[l] + c * (L / 2));
        }
    }
    const double *flat = f->act[4];   /* [64][16], channel-major */
    for (int o = 0; o < 256; ++o) {
        double s = p[F1B + o];
        for (int i = 0; i < 1024; ++i) s += p[F1W + (int64_t)o * 1024 + i] * flat[i];
        f->h1pre[o] = s;
        f->h1[o] = relu(s);
    }
    for (int o = 0; o < 64; ++o) {
        double s = p[F2B + o];
        for (int i = 0; i < 256; ++i) s += p[F2W + o * 256 + i] * f->h1[i];
        f->h2pre[o] = s;
        f->h2[o] = relu(s);
    }
    double s = p[F3B];
    for (int i = 0; i < 64; ++i) s += p[F3W + i] * f->h2[i];
    f->z = s;
}

/* Logits of B inputs x[B][256]. */
void oracle_cnn_forward(const double *params, const double *x, int B, double *logits) {
    Fwd *f = (Fwd *)malloc(sizeof(Fwd));
    for (int b = 0; b < B; ++b) {
        forward_one(params, x + (int64_t)b * 256, f);
        logits[b] = f->z;
    }
    free(f);
}

/*
 * Mean binary cross-entropy with logits over the batch, in the stable form
 * max(z, 0) - z y + log(1 + exp(-|z|)), and its gradient with respect to
 * every parameter (canonical layout). ReLU passes gradient only where its
 * input is > 0; max-pool routes it to the recorded winner.
 */
double oracle_cnn_loss_grad(const double *p, const double *x, const double *y, int B,
                            double *grad) {
    memset(grad, 0, sizeof(double) * NP);
    Fwd *f = (Fwd *)malloc(sizeof(Fwd));
    double loss = 0.0;
    for (int b = 0; b < B; ++b) {
        forward_one(p, x + (int64_t)b * 256, f);
        const double z = f->z, yy = y[b];
        loss += (z > 0.0 ? z : 0.0) - z * yy + log1p(exp(-fabs(z)));
        const double dz = (1.0 / (1.0 + exp(-z)) - yy) / (double)B;
        double dh2[64], dh1[256], dflat[1024];
        grad[F3B] += dz;
        for (int i = 0; i < 64; ++i) {
            grad[F3W + i] += dz * f->h2[i];
            dh2[i] = f->h2pre[i] > 0.0 ? dz * p[F3W + i] : 0.0;
        }
        for (int i = 0; i < 256; ++i) dh1[i] = 0.0;
        for (int o = 0; o < 64; ++o) {
            grad[F2B + o] += dh2[o];
            for (int i = 0; i < 256; ++i) {
                grad[F2W + o * 256 + i] += dh2[o] * f->h1[i];
                dh1[i] += p[F2W + o * 256 + i] * dh2[o];
            }
        }
        for (int i = 0; i < 256; ++i) dh1[i] = f->h1pre[i] > 0.0 ? dh1[i] : 0.0;
        for (int i = 0; i < 1024; ++i) dflat[i] = 0.0;
        for (int o = 0; o < 256; ++o) {
            grad[F1B + o] += dh1[o];
            for (int i = 0; i < 1024; ++i) {
                grad[F1W + (int64_t)o * 1024 + i] += dh1[o] * f->act[4][i];
                dflat[i] += p[F1W + (int64_t)o * 1024 + i] * dh1[o];
            }
        }
        double dact[64 * 128];
        memcpy(dact, dflat, sizeof(double) * 1024);
        for (int l = 4; l >= 1; --l) {
            const int Cin = CH[l - 1], Cout = CH[l], L = LEN[l - 1];
            static double dpre[64 * 256];
            memset(dpre, 0, sizeof(double) * Cout * L);
            for (int c = 0; c < Cout; ++c)
                for (int xx = 0; xx < L / 2; ++xx) {
                    int w = f->arg[l][c * (L / 2) + xx];
                    if (f->pre[l][c * L + w] > 0.0) dpre[c * L + w] = dact[c * (L / 2) + xx];
                }
            double *gw = grad + conv_w_off(l), *gb = grad + conv_b_off(l);
            const double *w = p + conv_w_off(l);
            const double *in = f->act[l - 1];
            for (int co = 0; co < Cout; ++co)
                for (int xx = 0; xx < L; ++xx) {
                    const double d = dpre[co * L + xx];
                    if (d == 0.0) continue;
                    gb[co] += d;
                    for (int ci = 0; ci < Cin; ++ci)
                        for (int dx = 0; dx < 5; ++dx) {
                            int q = ((xx + dx - 2) % L + L) % L;
                            gw[((int64_t)co * Cin + ci) * 5 + dx] += d * in[ci * L + q];
                        }
                }
            if (l > 1) {
                static double din[64 * 256];
                memset(din, 0, sizeof(double) * Cin * L);
                for (int co = 0; co < Cout; ++co)
                    for (int xx = 0; xx < L; ++xx) {
                        const double d = dpre[co * L + xx];
                        if (d == 0.0) continue;
                        for (int ci = 0; ci < Cin; ++ci)
                            for (int dx = 0; dx < 5; ++dx) {
                                int q = ((xx + dx - 2) % L + L) % L;
                                din[ci * L + q] += w[((int64_t)co * Cin + ci) * 5 + dx] * d;
                            }
                    }
                memcpy(dact, din, sizeof(double) * Cin * L);
            }
        }
    }
    free(f);
    return loss / (double)B;
}

/*
 * One Adam step (the optimiser the paper trains with, Sec. 2.5), with bias
 * correction: m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), t = step >= 1.
 */
void oracle_adam(double *p, const double *g, double *m, double *v, int64_t n, int64_t step,
                 double lr, double b1, double b2, double eps) {
    const double c1 = 1.0 - pow(b1, (double)step), c2 = 1.0 - pow(b2, (double)step);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        p[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}
