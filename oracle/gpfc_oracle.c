/*
 * Reference oracle for the GPFC phase-fold + box-SNR hot path.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow, obviously correct
 * CPU statement of what the GPU library computes. Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does. It shares no code, header, table or constant
 * with the HIP library.
 *
 * Arithmetic: IEEE-754 binary64, round-to-nearest-even, compiled with
 * -O2 -ffp-contract=off -fno-fast-math so that every operation below is one
 * correctly rounded step in the order written.
 *
 * Paper: Wang, Ge, Willis, Wang, Zhao, "The GPU Phase Folding and Deep
 * Learning Method for Detecting Exoplanet Transits" (MNRAS 2024,
 * arXiv:2312.02063).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/*
 * Curve statistics used by the normalisation and the SNR.
 * mean  = (sum of flux in sample order) / n                    (sequential)
 * sigma = sqrt(sum (flux - mean)^2 / (n - 1))                   (two-pass)
 * sigma is the per-point photometric scatter that Eq. 2 (Sec. 2.6) divides
 * the depth by. n < 2 gives sigma = 0.
 */
void oracle_curve_stats(const double *t, const float *flux, int64_t n,
                        double *mean_out, double *sigma_out, double *tmax_out) {
    double s = 0.0, tmax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        s += (double)flux[i];
        double a = fabs(t[i]);
        if (a > tmax) tmax = a;
    }
    double mean = n > 0 ? s / (double)n : 0.0;
    double ss = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double d = (double)flux[i] - mean;
        ss += d * d;
    }
    *mean_out = mean;
    *sigma_out = n > 1 ? sqrt(ss / (double)(n - 1)) : 0.0;
    if (tmax_out) *tmax_out = tmax;
}

/*
 * Phase bin of one sample at one trial period (Sec. 2.3, first two steps of
 * the five-step fold; Fig. 4 panels a-b): the timestamp is reduced modulo the
 * trial period and the residual is mapped to one of nbins equal-width bins.
 *
 *   x = t / P              one correctly rounded binary64 division
 *   f = x - floor(x)       phase in cycles, in [0, 1]
 *   u = f * nbins          exact for a power-of-two nbins
 *   b = floor(u), clamped to nbins - 1 (f can round up to 1 for x < 0)
 *
 * Phase zero is t = 0 of the caller's time scale.
 */
int32_t oracle_bin(double t, double period, int32_t nbins) {
    double x = t / period;
    double f = x - floor(x);
    double u = f * (double)nbins;
    double fb = floor(u);
    int32_t b;
    if (!(fb >= 0.0)) b = 0;              /* NaN input: defined as bin 0 */
    else if (fb >= (double)nbins) b = nbins - 1;
    else b = (int32_t)fb;
    return b;
}

/*
 * Fold at every trial period (Sec. 2.3 steps one to three and five): for
 * each period k and each sample i, add one to counts[k][b] and the flux to
 * sums[k][b]; dsums[k][b] accumulates flux - ref instead (the deviation
 * sums the box statistic uses). Samples are taken in index order. Output
 * layout is row-major [k][nbins].
 *
 * A period that is not a finite positive number gives an all-zero row.
 * nthreads > 1 splits the periods over OpenMP threads; every period is
 * computed by exactly the same sequential loop, so the result does not
 * depend on nthreads.
 */
void oracle_fold(const double *t, const float *flux, int64_t n,
                 const double *periods, int64_t k, int32_t nbins, double ref,
                 double *sums, double *dsums, int32_t *counts, int nthreads) {
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
#endif
    for (int64_t kk = 0; kk < k; ++kk) {
        double *srow = sums ? sums + kk * nbins : NULL;
        double *drow = dsums ? dsums + kk * nbins : NULL;
        int32_t *crow = counts + kk * nbins;
        for (int32_t b = 0; b < nbins; ++b) {
            crow[b] = 0;
            if (srow) srow[b] = 0.0;
            if (drow) drow[b] = 0.0;
        }
        double P = periods[kk];
        if (!(P > 0.0) || !isfinite(P)) continue;   /* invalid period: empty row */
        for (int64_t i = 0; i < n; ++i) {
            int32_t b = oracle_bin(t[i], P, nbins);
            crow[b] += 1;
            if (srow) srow[b] += (double)flux[i];
            if (drow) drow[b] += (double)flux[i] - ref;
        }
    }
    (void)nthreads;
}

/*
 * Bin means (Sec. 2.3 step five, Fig. 4 panels d-e): sum / count, NaN for
 * an empty bin.
 */
void oracle_means(const double *sums, const int32_t *counts, int64_t m,
                  double *means) {
    for (int64_t j = 0; j < m; ++j)
        means[j] = counts[j] > 0 ? sums[j] / (double)counts[j] : NAN;
}

/*
 * Default box-width set: the distinct integers nearest to sqrt(2)^j that lie
 * in [1, nbins / 2] (nbins = 1 gives {1}). Ascending. Returns the count.
 */
int32_t oracle_default_widths(int32_t nbins, int32_t *out, int32_t cap) {
    int32_t m = 0, last = 0;
    int32_t wmax = nbins / 2 > 0 ? nbins / 2 : 1;
    for (int j = 0; j < 64; ++j) {
        double v = pow(sqrt(2.0), (double)j);
        int32_t w = (int32_t)floor(v + 0.5);
        if (w > wmax) break;
        if (w != last) {
            if (m < cap) out[m] = w;
            ++m;
            last = w;
        }
    }
    return m;
}

/*
 * Box-transit SNR of each folded curve. The paper gives the SNR of a transit
 * only in closed form (Eq. 2, Sec. 2.6: depth over per-point noise times the
 * square root of the in-transit sample count) and the box model of BLS
 * (Sec. 3.1); this is the statistic built from the two, for a box of w
 * consecutive bins starting at bin s, taken circularly because phase wraps:
 *
 *   n_in  = sum_{j<w} c[(s+j) mod B],  D_in = sum_{j<w} D[(s+j) mod B]
 *   n_out = n - n_in,                  D_out = S - D_in
 *   depth = D_out / n_out - D_in / n_in          (mean out minus mean in)
 *   snr   = depth * sqrt(n_in * n_out / n) / sigma
 *
 * where c are counts, D deviation sums, n = sum c and S = sum D. Boxes with
 * n_in = 0 or n_out = 0 are skipped, and so are widths w >= B (a box that
 * wide leaves no bin outside it). The result is the largest snr over
 * widths in ascending order and starts in ascending order, a later box
 * replacing the best only if strictly larger, starting from 0: only dips
 * score. With no positive box, or sigma not > 0, snr = 0, depth = 0 and
 * start = width = -1.
 */
void oracle_score(const int32_t *counts, const double *dsums, int64_t k,
                  int32_t nbins, double sigma, const int32_t *widths,
                  int32_t nw, double *snr, int32_t *start, int32_t *width,
                  double *depth) {
    for (int64_t kk = 0; kk < k; ++kk) {
        const int32_t *c = counts + kk * nbins;
        const double *D = dsums + kk * nbins;
        double best = 0.0, best_depth = 0.0;
        int32_t bs = -1, bw = -1;
        int64_t n = 0;
        double S = 0.0;
        for (int32_t b = 0; b < nbins; ++b) {
            n += c[b];
            S += D[b];
        }
        if (sigma > 0.0 && isfinite(sigma)) {
            for (int32_t wi = 0; wi < nw; ++wi) {
                int32_t w = widths[wi];
                if (w >= nbins) continue;   /* no out-of-box bins, or bins counted twice */
                for (int32_t s = 0; s < nbins; ++s) {
                    int64_t n_in = 0;
                    double D_in = 0.0;
                    for (int32_t j = 0; j < w; ++j) {
                        int32_t b = (s + j) % nbins;
                        n_in += c[b];
                        D_in += D[b];
                    }
                    int64_t n_out = n - n_in;
                    if (n_in == 0 || n_out == 0) continue;
                    double dep = (S - D_in) / (double)n_out - D_in / (double)n_in;
                    double v = dep * sqrt((double)n_in * (double)n_out / (double)n) / sigma;
                    if (v > best) {
                        best = v;
                        best_depth = dep;
                        bs = s;
                        bw = w;
                    }
                }
            }
        }
        snr[kk] = best;
        depth[kk] = best_depth;
        start[kk] = bs;
        width[kk] = bw;
    }
}

/*
 * Box statistic of one given box (same formula as above); used to judge a
 * near-tie: the value of the oracle's statistic at another implementation's
 * chosen (start, width). Returns 0 when the box is empty or full.
 */
double oracle_box_snr(const int32_t *c, const double *D, int32_t nbins,
                      double sigma, int32_t s, int32_t w) {
    int64_t n = 0, n_in = 0;
    double S = 0.0, D_in = 0.0;
    for (int32_t b = 0; b < nbins; ++b) {
        n += c[b];
        S += D[b];
    }
    for (int32_t j = 0; j < w; ++j) {
        int32_t b = (s + j) % nbins;
        n_in += c[b];
        D_in += D[b];
    }
    int64_t n_out = n - n_in;
    if (n_in == 0 || n_out == 0) return 0.0;
    double dep = (S - D_in) / (double)n_out - D_in / (double)n_in;
    return dep * sqrt((double)n_in * (double)n_out / (double)n) / sigma;
}

/*
 * Noise normalisation of a folded curve before the learned scorer (Sec. 2.1:
 * each folded curve is scaled to unit noise): over the non-empty bins of a
 * row, z = (mean_b - mu) / sd with mu and sd the mean and standard deviation
 * (ddof 0) of those bin means; empty bins, and every bin of a row whose sd
 * is 0, get 0. The paper also keeps the row's mean; adding a constant to every
 * input of the first convolution is absorbed by its bias, so it is dropped.
 */
void oracle_normalize(const double *sums, const int32_t *counts, int64_t k, int32_t nbins,
                      double *z) {
    for (int64_t kk = 0; kk < k; ++kk) {
        const double *s = sums + kk * nbins;
        const int32_t *c = counts + kk * nbins;
        double *zr = z + kk * nbins;
        int32_t m = 0;
        double mu = 0.0;
        for (int32_t b = 0; b < nbins; ++b)
            if (c[b] > 0) { mu += s[b] / (double)c[b]; ++m; }
        mu = m > 0 ? mu / (double)m : 0.0;
        double var = 0.0;
        for (int32_t b = 0; b < nbins; ++b)
            if (c[b] > 0) { double d = s[b] / (double)c[b] - mu; var += d * d; }
        double sd = m > 0 ? sqrt(var / (double)m) : 0.0;
        for (int32_t b = 0; b < nbins; ++b)
            zr[b] = (c[b] > 0 && sd > 0.0) ? (s[b] / (double)c[b] - mu) / sd : 0.0;
    }
}

/*
 * Trial-grid size of Eq. 1 (Sec. 2.1): N_sample = N_o * T / L.
 */
double oracle_grid_size(double n_o, double span, double width) {
    return n_o * span / width;
}

/*
 * Per-curve reduction of a periodogram (Sec. 2.1: the best of the scores over
 * all trial periods is the curve's detection; Sec. 3.2: the maximum score over
 * periods is the statistic a threshold is applied to). For each row of `rows`
 * rows of `len` scores: the `top` best entries, best first, where an entry is
 * a candidate when its value is not NaN and, if `gate` is given, gate >=
 * gate_min (a NaN gate never passes); order is by value descending, then by
 * index ascending. Missing places get value -inf and index -1.
 *
 * Plain selection: pick j is the best candidate strictly after pick j-1 in
 * that order (keys are unique because indices are).
 */
void oracle_topk(const float *values, const float *gate, float gate_min, int64_t rows, int64_t len,
                 int32_t top, float *out_val, int64_t *out_idx) {
    for (int64_t r = 0; r < rows; ++r) {
        const float *v = values + r * len;
        const float *g = gate ? gate + r * len : 0;
        float pv = 0.0f;
        int64_t pi = -1;             /* previous pick; -1: none yet */
        for (int32_t j = 0; j < top; ++j) {
            int64_t bi = -1;
            float bv = 0.0f;
            for (int64_t i = 0; i < len; ++i) {
                if (isnan(v[i])) continue;
                if (g && !(g[i] >= gate_min)) continue;
                /* must come strictly after the previous pick in the order */
                if (pi >= 0 && !(v[i] < pv || (v[i] == pv && i > pi))) continue;
                if (bi < 0 || v[i] > bv || (v[i] == bv && i < bi)) { bi = i; bv = v[i]; }
            }
            out_val[r * top + j] = bi >= 0 ? bv : -INFINITY;
            out_idx[r * top + j] = bi;
            if (bi < 0) {
                for (int32_t q = j + 1; q < top; ++q) { out_val[r * top + q] = -INFINITY; out_idx[r * top + q] = -1; }
                break;
            }
            pv = bv;
            pi = bi;
        }
    }
}

/*
 * The paper's two-tier equal-count fold (Sec. 2.3, steps 1-5 and Fig. 4):
 * per period, (1) the modular residual of each timestamp, (2) its bin among
 * n_mid equal-width intermediate bins (4096 in the paper), (3) counts and
 * flux sums per intermediate bin, (4) a left-to-right scan that merges the
 * intermediate bins into nbins final bins holding the same number of points
 * each, splitting a bin on a boundary in proportion (each split part carries
 * the bin's mean flux times the points it takes), (5) the mean flux of each
 * final bin.
 *
 * Reading: with N points each final bin holds N / nbins points, generally
 * fractional; the scan counts in units of 1/nbins point (a sample is nbins
 * units, a final bin N units), so the partition is exact integer arithmetic.
 * means f64[k][nbins]; N = 0 or an invalid period gives NaN means.
 */
void oracle_fold_eqcount(const double *t, const float *flux, int64_t n, const double *periods,
                         int64_t k, int32_t n_mid, int32_t nbins, double *means) {
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_mid);
    double *sum = (double *)malloc(sizeof(double) * (size_t)n_mid);
    for (int64_t kk = 0; kk < k; ++kk) {
        double *out = means + kk * nbins;
        const double P = periods[kk];
        if (n == 0 || !(P > 0.0) || !isfinite(P)) {
            for (int32_t j = 0; j < nbins; ++j) out[j] = NAN;
            continue;
        }
        for (int32_t b = 0; b < n_mid; ++b) { cnt[b] = 0; sum[b] = 0.0; }
        for (int64_t i = 0; i < n; ++i) {
            const int32_t b = oracle_bin(t[i], P, n_mid);
            cnt[b] += 1;
            sum[b] += (double)flux[i];
        }
        int32_t j = 0;
        int64_t room = n;          /* units left in final bin j */
        double acc = 0.0;
        for (int32_t b = 0; b < n_mid && j < nbins; ++b) {
            if (cnt[b] == 0) continue;
            const double mean = sum[b] / (double)cnt[b];
            int64_t left = cnt[b] * nbins;
            while (left > 0 && j < nbins) {
                const int64_t take = left < room ? left : room;
                acc += mean * (double)take;
                left -= take;
                room -= take;
                if (room == 0) {
                    out[j] = acc / (double)n;
                    ++j;
                    acc = 0.0;
                    room = n;
                }
            }
        }
    }
    free(cnt);
    free(sum);
}

/*
 * Periodogram post-processing, per row of `len` scores (one curve's
 * periodogram over its trial periods):
 *  - SDE (Eq. 3): (max - mean) / sd over the non-NaN scores, sd with ddof 0
 *    (0 when sd = 0 or no score);
 *  - peaks (Sec. 4.2: the best peak among those higher than 3 sigma and wider
 *    than 3 points): maximal runs of consecutive scores > mean + nsigma * sd
 *    (a NaN ends a run) longer than min_width points; a peak's value is the
 *    run's maximum, its index the first position of that maximum, its width
 *    the run length; peaks ordered by value descending, then index ascending;
 *  - harmonics: with periods given, code h (2, 3) for a peak at h times the
 *    best peak's period and -h at 1/h of it, within a relative 1e-3; 1 for the
 *    best peak itself; 0 otherwise.
 * Outputs per row: sde, mean, sd, n_peaks (all qualifying runs) and the first
 * max_peaks peaks (value -inf, index -1, width 0, code 0 where missing).
 */
void oracle_periodogram(const float *values, const double *periods, int64_t rows, int64_t len,
                        float nsigma, int32_t min_width, int32_t max_peaks, float *sde,
                        float *mean_out, float *sd_out, int32_t *n_peaks, float *pval,
                        int64_t *pidx, int32_t *pwidth, int32_t *pharm) {
    for (int64_t r = 0; r < rows; ++r) {
        const float *v = values + r * len;
        double s = 0.0, mx = -INFINITY;
        int64_t m = 0;
        for (int64_t i = 0; i < len; ++i)
            if (!isnan(v[i])) { s += v[i]; ++m; if (v[i] > mx) mx = v[i]; }
        const double mean = m ? s / (double)m : 0.0;
        double q = 0.0;
        for (int64_t i = 0; i < len; ++i)
            if (!isnan(v[i])) { const double d = v[i] - mean; q += d * d; }
        const double sd = m ? sqrt(q / (double)m) : 0.0;
        sde[r] = (float)((m && sd > 0.0) ? (mx - mean) / sd : 0.0);
        mean_out[r] = (float)mean;
        sd_out[r] = (float)sd;
        const double thr = mean + (double)nsigma * sd;
        float *ov = pval + r * max_peaks;
        int64_t *oi = pidx + r * max_peaks;
        int32_t *ow = pwidth + r * max_peaks;
        int32_t *oh = pharm + r * max_peaks;
        for (int32_t j = 0; j < max_peaks; ++j) { ov[j] = -INFINITY; oi[j] = -1; ow[j] = 0; oh[j] = 0; }
        int32_t np = 0;
        int64_t i = 0;
        while (i < len) {
            if (isnan(v[i]) || !(v[i] > thr)) { ++i; continue; }
            int64_t j = i, best = i;
            while (j < len && !isnan(v[j]) && v[j] > thr) { if (v[j] > v[best]) best = j; ++j; }
            const int64_t w = j - i;
            if (w > min_width) {
                ++np;
                /* insert (v[best], best, w) into the sorted list */
                int32_t pos = max_peaks;
                for (int32_t a = 0; a < max_peaks; ++a)
                    if (v[best] > ov[a] || (v[best] == ov[a] && (oi[a] < 0 || best < oi[a]))) { pos = a; break; }
                if (pos < max_peaks) {
                    for (int32_t a = max_peaks - 1; a > pos; --a) { ov[a] = ov[a - 1]; oi[a] = oi[a - 1]; ow[a] = ow[a - 1]; }
                    ov[pos] = v[best]; oi[pos] = best; ow[pos] = (int32_t)w;
                }
            }
            i = j;
        }
        n_peaks[r] = np;
        if (periods && max_peaks > 0 && oi[0] >= 0) {
            const double p0 = periods[oi[0]];
            oh[0] = 1;
            for (int32_t a = 1; a < max_peaks; ++a) {
                if (oi[a] < 0) break;
                const double ratio = periods[oi[a]] / p0;
                for (int h = 2; h <= 3; ++h) {
                    if (fabs(ratio - h) <= 1e-3 * h) oh[a] = h;
                    if (fabs(1.0 / ratio - h) <= 1e-3 * h) oh[a] = -h;
                }
            }
        }
    }
}
