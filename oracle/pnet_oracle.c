/*
 * CPU oracle of the paper's own scoring network (Sec. 2.5, Fig. 5 of
 * arXiv:2312.02063): forward pass, binary cross-entropy and its gradient
 * in plain FP64 C.
 *
 * TEST INFRASTRUCTURE ONLY: the slow, obviously correct statement the GPU
 * kernels are checked against. It shares no code with the GPU library.
 *
 * The network as the paper describes it, with the readings its text leaves
 * open (the figure's layer sizes are not in the text):
 *   - the 1-D input (a normalised fold of S*S bins, S = 16) is reshaped,
 *     row-major, into an S x S image;
 *   - a circular convolution (periodic wrap-around padding in both image
 *     axes, output the same size) with F1 = 128 filters, then one with
 *     F2 = 256 filters, kernel K1 x K1 (K1 = 3), each followed by ReLU;
 *   - the image is read back as S*S positions of F2 channels and a global
 *     max-pool over the positions keeps F2 values;
 *   - the same sequence again, with larger kernels (K2 = 5): the F2 = S*S
 *     pooled values reshaped row-major into an S x S one-channel image,
 *     circular convolutions of F3 = 128 and F4 = 256 filters with ReLU, a
 *     global max-pool over positions (F4 values);
 *   - a fully connected layer of H = 128 units with ReLU, dropout (rate
 *     0.5 in training; the keep mask, already scaled by 1 / (1 - rate), is
 *     an input: NULL means inference) and a dense output unit whose sigmoid
 *     is the transit probability.
 * Counting input, reshapes, padding, convolution, pooling, flatten, dense
 * and dropout layers this gives the paper's 19 layers.
 * Convolution convention (cross-correlation): for a kernel of side K and
 * p = (K - 1) / 2,
 *   y[f][r][c] = b[f] + sum_{i, u, v} w[f][i][u][v] x[i][(r + u - p) mod S][(c + v - p) mod S].
 * Global max-pool ties route the gradient to the first position in
 * row-major order. Loss: BCE with logits, max(z, 0) - z y + log(1 + e^-|z|).
 *
 * Parameter layout (flat, FP64): w1 [F1][1][K1][K1], b1 [F1], w2
 * [F2][F1][K1][K1], b2 [F2], w3 [F3][1][K2][K2], b3 [F3], w4 [F4][F3][K2][K2],
 * b4 [F4], w5 [H][F4], b5 [H], w6 [H], b6 [1]. Sizes come in a config so
 * the tests can run a reduced network (F2 must equal S * S).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t S, F1, F2, F3, F4, K1, K2, H;
} pnet_cfg;

static int64_t off_w1(const pnet_cfg* c) { (void)c; return 0; }
static int64_t off_b1(const pnet_cfg* c) { return off_w1(c) + (int64_t)c->F1 * c->K1 * c->K1; }
static int64_t off_w2(const pnet_cfg* c) { return off_b1(c) + c->F1; }
static int64_t off_b2(const pnet_cfg* c) { return off_w2(c) + (int64_t)c->F2 * c->F1 * c->K1 * c->K1; }
static int64_t off_w3(const pnet_cfg* c) { return off_b2(c) + c->F2; }
static int64_t off_b3(const pnet_cfg* c) { return off_w3(c) + (int64_t)c->F3 * c->K2 * c->K2; }
static int64_t off_w4(const pnet_cfg* c) { return off_b3(c) + c->F3; }
static int64_t off_b4(const pnet_cfg* c) { return off_w4(c) + (int64_t)c->F4 * c->F3 * c->K2 * c->K2; }
static int64_t off_w5(const pnet_cfg* c) { return off_b4(c) + c->F4; }
static int64_t off_b5(const pnet_cfg* c) { return off_w5(c) + (int64_t)c->H * c->F4; }
static int64_t off_w6(const pnet_cfg* c) { return off_b5(c) + c->H; }
static int64_t off_b6(const pnet_cfg* c) { return off_w6(c) + c->H; }

int64_t oracle_pnet_nparams(const pnet_cfg* c) { return off_b6(c) + 1; }

static int wrap(int v, int S) { return ((v % S) + S) % S; }

/* Circular convolution of x [ci][S][S] by w [co][ci][K][K] + b, output
 * y [co][S][S] (pre-activation). */
void oracle_pnet_conv2d_circ(const double* x, const double* w, const double* b, int ci, int co,
                             int K, int S, double* y) {
    const int p = (K - 1) / 2;
    for (int f = 0; f < co; ++f)
        for (int r = 0; r < S; ++r)
            for (int c = 0; c < S; ++c) {
                double acc = b[f];
                for (int i = 0; i < ci; ++i)
                    for (int u = 0; u < K; ++u)
                        for (int v = 0; v < K; ++v)
                            acc += w[(((int64_t)f * ci + i) * K + u) * K + v] *
                                   x[((int64_t)i * S + wrap(r + u - p, S)) * S + wrap(c + v - p, S)];
                y[((int64_t)f * S + r) * S + c] = acc;
            }
}

/* Global max over the S*S positions of each of C channels of
 * y [C][S*S], after ReLU: out[f] = max(0, max_p y[f][p]); arg[f] = the first
 * position of the maximum of y[f] (the gradient's route; -1 if the maximum
 * is not positive, when ReLU blocks every position). */
static void gmp_relu(const double* y, int C, int P, double* out, int32_t* arg) {
    for (int f = 0; f < C; ++f) {
        int best = 0;
        for (int p = 1; p < P; ++p)
            if (y[(int64_t)f * P + p] > y[(int64_t)f * P + best]) best = p;
        const double m = y[(int64_t)f * P + best];
        out[f] = m > 0.0 ? m : 0.0;
        arg[f] = m > 0.0 ? best : -1;
    }
}

typedef struct {
    double *z1, *a1, *z2, *g1, *z3, *a3, *z4, *g2, *h, *hd;
    int32_t *arg1, *arg2;
} pnet_act;

static void act_alloc(const pnet_cfg* c, pnet_act* a) {
    const int P = c->S * c->S;
    a->z1 = malloc(sizeof(double) * c->F1 * P);
    a->a1 = malloc(sizeof(double) * c->F1 * P);
    a->z2 = malloc(sizeof(double) * c->F2 * P);
    a->g1 = malloc(sizeof(double) * c->F2);
    a->z3 = malloc(sizeof(double) * c->F3 * P);
    a->a3 = malloc(sizeof(double) * c->F3 * P);
    a->z4 = malloc(sizeof(double) * c->F4 * P);
    a->g2 = malloc(sizeof(double) * c->F4);
    a->h = malloc(sizeof(double) * c->H);
    a->hd = malloc(sizeof(double) * c->H);
    a->arg1 = malloc(sizeof(int32_t) * c->F2);
    a->arg2 = malloc(sizeof(int32_t) * c->F4);
}

static void act_free(pnet_act* a) {
    free(a->z1); free(a->a1); free(a->z2); free(a->g1); free(a->z3); free(a->a3);
    free(a->z4); free(a->g2); free(a->h); free(a->hd); free(a->arg1); free(a->arg2);
}

/* One input x [S*S] -> logit; keeps the activations in a. */
static double forward_one(const pnet_cfg* c, const double* prm, const double* x, const double* mask,
                          pnet_act* a) {
    const int S = c->S, P = S * S;
    oracle_pnet_conv2d_circ(x, prm + off_w1(c), prm + off_b1(c), 1, c->F1, c->K1, S, a->z1);
    for (int i = 0; i < c->F1 * P; ++i) a->a1[i] = a->z1[i] > 0.0 ? a->z1[i] : 0.0;
    oracle_pnet_conv2d_circ(a->a1, prm + off_w2(c), prm + off_b2(c), c->F1, c->F2, c->K1, S, a->z2);
    gmp_relu(a->z2, c->F2, P, a->g1, a->arg1);
    /* the F2 = S*S pooled values as a one-channel S x S image */
    oracle_pnet_conv2d_circ(a->g1, prm + off_w3(c), prm + off_b3(c), 1, c->F3, c->K2, S, a->z3);
    for (int i = 0; i < c->F3 * P; ++i) a->a3[i] = a->z3[i] > 0.0 ? a->z3[i] : 0.0;
    oracle_pnet_conv2d_circ(a->a3, prm + off_w4(c), prm + off_b4(c), c->F3, c->F4, c->K2, S, a->z4);
    gmp_relu(a->z4, c->F4, P, a->g2, a->arg2);
    const double* w5 = prm + off_w5(c);
    const double* b5 = prm + off_b5(c);
    for (int j = 0; j < c->H; ++j) {
        double acc = b5[j];
        for (int f = 0; f < c->F4; ++f) acc += w5[(int64_t)j * c->F4 + f] * a->g2[f];
        a->h[j] = acc > 0.0 ? acc : 0.0;
        a->hd[j] = mask ? a->h[j] * mask[j] : a->h[j];
    }
    const double* w6 = prm + off_w6(c);
    double z = prm[off_b6(c)];
    for (int j = 0; j < c->H; ++j) z += w6[j] * a->hd[j];
    return z;
}

/* Logits of B inputs x [B][S*S]; mask [B][H] or NULL (inference). */
void oracle_pnet_forward(const pnet_cfg* c, const double* prm, const double* x, int64_t B,
                         const double* mask, double* logits) {
    const int P = c->S * c->S;
#pragma omp parallel
    {
        pnet_act a;
        act_alloc(c, &a);
#pragma omp for schedule(dynamic, 1)
        for (int64_t b = 0; b < B; ++b)
            logits[b] = forward_one(c, prm, x + b * P, mask ? mask + b * c->H : NULL, &a);
        act_free(&a);
    }
}

/* Intermediate results of one input, for tests: g1 [F2], g2 [F4], h [H]. */
void oracle_pnet_features(const pnet_cfg* c, const double* prm, const double* x, double* g1,
                          double* g2, double* h) {
    pnet_act a;
    act_alloc(c, &a);
    forward_one(c, prm, x, NULL, &a);
    memcpy(g1, a.g1, sizeof(double) * c->F2);
    memcpy(g2, a.g2, sizeof(double) * c->F4);
    memcpy(h, a.h, sizeof(double) * c->H);
    act_free(&a);
}

/* Gradient of a circular convolution: given dy [co][S][S] (w.r.t. the
 * pre-activation), add to dw, db and (if dx) to dx [ci][S][S]. */
static void conv_backward(const double* x, const double* w, const double* dy, int ci, int co, int K,
                          int S, double* dw, double* db, double* dx) {
    const int p = (K - 1) / 2;
    for (int f = 0; f < co; ++f)
        for (int r = 0; r < S; ++r)
            for (int cc = 0; cc < S; ++cc) {
                const double g = dy[((int64_t)f * S + r) * S + cc];
                if (g == 0.0) continue;
                db[f] += g;
                for (int i = 0; i < ci; ++i)
                    for (int u = 0; u < K; ++u)
                        for (int v = 0; v < K; ++v) {
                            const int64_t xi = ((int64_t)i * S + wrap(r + u - p, S)) * S + wrap(cc + v - p, S);
                            const int64_t wi = (((int64_t)f * ci + i) * K + u) * K + v;
                            dw[wi] += g * x[xi];
                            if (dx) dx[xi] += g * w[wi];
                        }
            }
}

/* Mean BCE-with-logits loss over B inputs with labels y [B], and its
 * gradient w.r.t. every parameter into grad (overwritten). */
double oracle_pnet_loss_grad(const pnet_cfg* c, const double* prm, const double* x, const double* y,
                             int64_t B, const double* mask, double* grad) {
    const int S = c->S, P = S * S;
    const int64_t np = oracle_pnet_nparams(c);
    memset(grad, 0, sizeof(double) * np);
    pnet_act a;
    act_alloc(c, &a);
    double* dz1 = malloc(sizeof(double) * c->F1 * P);
    double* dz2 = malloc(sizeof(double) * c->F2 * P);
    double* dg1 = malloc(sizeof(double) * c->F2);
    double* dz3 = malloc(sizeof(double) * c->F3 * P);
    double* dz4 = malloc(sizeof(double) * c->F4 * P);
    double* dh = malloc(sizeof(double) * c->H);
    double* da1 = malloc(sizeof(double) * c->F1 * P);
    double* da3 = malloc(sizeof(double) * c->F3 * P);
    double loss = 0.0;
    for (int64_t b = 0; b < B; ++b) {
        const double* mk = mask ? mask + b * c->H : NULL;
        const double z = forward_one(c, prm, x + b * P, mk, &a);
        loss += (z > 0.0 ? z : 0.0) - z * y[b] + log1p(exp(-fabs(z)));
        const double dz = (1.0 / (1.0 + exp(-z)) - y[b]) / (double)B;
        /* output unit */
        grad[off_b6(c)] += dz;
        for (int j = 0; j < c->H; ++j) {
            grad[off_w6(c) + j] += dz * a.hd[j];
            const double dhd = dz * prm[off_w6(c) + j];
            const double dhj = mk ? dhd * mk[j] : dhd;
            dh[j] = a.h[j] > 0.0 ? dhj : 0.0;
        }
        /* hidden layer */
        memset(dg1, 0, sizeof(double) * c->F2);
        double* dg2 = malloc(sizeof(double) * c->F4);
        memset(dg2, 0, sizeof(double) * c->F4);
        for (int j = 0; j < c->H; ++j) {
            grad[off_b5(c) + j] += dh[j];
            for (int f = 0; f < c->F4; ++f) {
                grad[off_w5(c) + (int64_t)j * c->F4 + f] += dh[j] * a.g2[f];
                dg2[f] += dh[j] * prm[off_w5(c) + (int64_t)j * c->F4 + f];
            }
        }
        /* second global max-pool: the gradient goes to the routed position */
        memset(dz4, 0, sizeof(double) * c->F4 * P);
        for (int f = 0; f < c->F4; ++f)
            if (a.arg2[f] >= 0) dz4[(int64_t)f * P + a.arg2[f]] = dg2[f];
        free(dg2);
        memset(da3, 0, sizeof(double) * c->F3 * P);
        conv_backward(a.a3, prm + off_w4(c), dz4, c->F3, c->F4, c->K2, S, grad + off_w4(c),
                      grad + off_b4(c), da3);
        for (int i = 0; i < c->F3 * P; ++i) dz3[i] = a.z3[i] > 0.0 ? da3[i] : 0.0;
        conv_backward(a.g1, prm + off_w3(c), dz3, 1, c->F3, c->K2, S, grad + off_w3(c),
                      grad + off_b3(c), dg1);
        /* first global max-pool */
        memset(dz2, 0, sizeof(double) * c->F2 * P);
        for (int f = 0; f < c->F2; ++f)
            if (a.arg1[f] >= 0) dz2[(int64_t)f * P + a.arg1[f]] = dg1[f];
        memset(da1, 0, sizeof(double) * c->F1 * P);
        conv_backward(a.a1, prm + off_w2(c), dz2, c->F1, c->F2, c->K1, S, grad + off_w2(c),
                      grad + off_b2(c), da1);
        for (int i = 0; i < c->F1 * P; ++i) dz1[i] = a.z1[i] > 0.0 ? da1[i] : 0.0;
        conv_backward(x + b * P, prm + off_w1(c), dz1, 1, c->F1, c->K1, S, grad + off_w1(c),
                      grad + off_b1(c), NULL);
    }
    free(dz1); free(dz2); free(dg1); free(dz3); free(dz4); free(dh); free(da1); free(da3);
    act_free(&a);
    return loss / (double)B;
}
