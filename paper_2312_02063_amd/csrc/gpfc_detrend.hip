// Light-curve pre-processing on gfx950 (Sec. 2.2, Fig. 3 of
// arXiv:2312.02063): the curve is cut into segments at long time gaps and
// large flux steps; each segment's continuum is a least-squares cubic
// B-spline fitted with the known transits masked and outliers clipped
// iteratively, its knot spacing chosen by BIC; the flux is divided by the
// continuum and a fixed number of points is dropped at each segment end.
//
// Readings of what the text leaves open (the same as the CPU statement the
// tests compare with): time-sorted input; a time gap is measured from the
// previous sample, masked or not; a flux step only between unmasked samples,
// from the previous unmasked one, against a multiple of the sample std
// (ddof 1) of the unmasked flux (so a masked transit's dip does not split its
// segment); the spline has uniform knots, L = max(1, ceil(span / h)) spans and
// L + 3 basis functions for a spacing h from a candidate list; each fit
// clips the unmasked points with |residual| > clip_sigma times the residual
// scatter (ddof 0) of the fitted points, and refits until the clipped set
// repeats (at most max_fits fits; the last fit and the set it used are
// kept); BIC = n ln(RSS / n) + m ln n over the n fitted points and m basis
// functions, the smallest winning (ties: the earlier spacing); a spacing
// with fewer than 2m fitted points is not tried, and a segment with no
// tried spacing, or with at most 2 edge points, is dropped.
//
// Kernels: k_dt_segments (one block: the std, the previous unmasked sample
// by a running max-scan, segment starts compacted by a sum-scan);
// k_dt_fit (a block per (segment, spacing): normal equations of the banded
// B-spline system accumulated by one thread per basis function over the
// samples of its four knot spans in time order, banded Cholesky in FP64,
// residuals, scatter and clip flags; every sum in a fixed order, so results
// are deterministic); k_dt_apply (a block per segment: the BIC choice, the
// division and the edge crop).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "gpfc_internal.h"

namespace gdt {

using gpfc::kDetrendMaxBasis;
constexpr int kFitThreads = 256;

// Block-wide reductions in a fixed order (wave shuffles, then waves in order).
template <int NT>
__device__ double block_sum(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < NT / 64; ++w) s += red[w];
    return s;
}

template <int NT>
__device__ int64_t block_sum_i(int64_t v, int64_t* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    int64_t s = 0;
    for (int w = 0; w < NT / 64; ++w) s += red[w];
    return s;
}

// Inclusive scan across a block of NT threads; ident is the identity of op;
// *total receives the whole block's result.
template <int NT, class T, class Op>
__device__ T block_scan(T v, T* tmp, Op op, T ident, T* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int d = 1; d < 64; d <<= 1) {
        const T o = __shfl_up(v, d, 64);
        if (lane >= d) v = op(v, o);
    }
    __syncthreads();
    if (lane == 63) tmp[wave] = v;
    __syncthreads();
    T pre = ident;
    for (int w = 0; w < wave; ++w) pre = op(pre, tmp[w]);
    T all = ident;
    for (int w = 0; w < NT / 64; ++w) all = op(all, tmp[w]);
    *total = all;
    return op(pre, v);
}

// Segment starts of a time-sorted curve: seg[0] = 0, seg[1..nseg-1] the
// samples that open a segment, seg[nseg] = n; *nseg_out = nseg (0 if n = 0).
__global__ __launch_bounds__(1024) void k_dt_segments(const double* __restrict__ t,
                                                      const float* __restrict__ flux,
                                                      const uint8_t* __restrict__ tr, int64_t n,
                                                      double gap, double jump,
                                                      int32_t* __restrict__ seg,
                                                      int32_t* __restrict__ nseg_out) {
    __shared__ double red[16];
    __shared__ int64_t redi[16];
    __shared__ int32_t tmp[16];
    const int tid = threadIdx.x;
    // sample std (ddof 1) of the unmasked flux
    double s = 0.0;
    int64_t c = 0;
    for (int64_t i = tid; i < n; i += 1024)
        if (!(tr && tr[i])) { s += (double)flux[i]; ++c; }
    const double S = block_sum<1024>(s, red);
    const int64_t C = block_sum_i<1024>(c, redi);
    const double mean = C > 0 ? S / (double)C : 0.0;
    double ss = 0.0;
    for (int64_t i = tid; i < n; i += 1024)
        if (!(tr && tr[i])) { const double d = (double)flux[i] - mean; ss += d * d; }
    const double SS = block_sum<1024>(ss, red);
    const double sd = C > 1 ? sqrt(SS / (double)(C - 1)) : 0.0;
    const double thr = jump * sd;
    // tiles of 1024 samples: previous unmasked index by a max-scan, then the
    // segment openers compacted in order by a sum-scan
    __shared__ int32_t sc[1024];
    auto mx = [](int32_t a, int32_t b) { return a > b ? a : b; };
    auto add = [](int32_t a, int32_t b) { return a + b; };
    int32_t carry_prev = -1, carry_cnt = 0;
    for (int64_t base = 0; base < n; base += 1024) {
        const int64_t i = base + tid;
        const bool un = i < n && !(tr && tr[i]);
        int32_t tot, cnt;
        sc[tid] = block_scan<1024, int32_t>(un ? (int32_t)i : -1, tmp, mx, -1, &tot);
        __syncthreads();
        int32_t prev = tid > 0 ? sc[tid - 1] : -1;   // the last unmasked sample before i
        if (prev < 0) prev = carry_prev;
        // a time gap from the previous sample (any), or a flux step from the
        // previous unmasked sample (unmasked samples only)
        bool open = i < n && i > 0 && t[i] - t[i - 1] > gap;
        if (un && prev >= 0) open = open || fabs((double)flux[i] - (double)flux[prev]) > thr;
        const int32_t pos = block_scan<1024, int32_t>(open ? 1 : 0, tmp, add, 0, &cnt);
        if (open) seg[carry_cnt + pos] = (int32_t)i;   // seg[1 + carry_cnt + pos - 1]
        carry_cnt += cnt;
        carry_prev = tot > carry_prev ? tot : carry_prev;
        __syncthreads();
    }
    if (tid == 0) {
        if (n > 0) {
            seg[0] = 0;
            seg[1 + carry_cnt] = (int32_t)n;
            *nseg_out = 1 + carry_cnt;
        } else {
            *nseg_out = 0;
        }
    }
}

// Uniform cubic B-spline: span j = clamp(floor((t - a) / he), 0, L - 1) and
// the weights of basis functions j .. j+3 at u = (t - a) / he - j.
__device__ __forceinline__ int span_of(double tk, double a, double he, int L, double& u) {
    const double x = (tk - a) / he;
    double fj = floor(x);
    if (fj < 0.0) fj = 0.0;
    if (fj > (double)(L - 1)) fj = (double)(L - 1);
    u = x - fj;
    return (int)fj;
}
__device__ __forceinline__ void bweights(double u, double w[4]) {
    const double v = 1.0 - u;
    w[0] = v * v * v / 6.0;
    w[1] = (3.0 * u * u * u - 6.0 * u * u + 4.0) / 6.0;
    w[2] = (-3.0 * u * u * u + 3.0 * u * u + 3.0 * u + 1.0) / 6.0;
    w[3] = u * u * u / 6.0;
}

// Per (spacing, segment) results, stored at the segment's first sample index
// in arrays of n entries per spacing.
struct FitOut {
    double* bic;        // [ns][n]
    double* coef;       // [ns][n]: the m coefficients at [s0, s0 + m) (m <= len / 2)
    uint8_t* clip;      // [ns][2][n]: two clip-flag buffers per spacing
    int8_t* state;      // [ns][n]: 0 not tried, 1 tried with clip buffer 0, 2 with buffer 1
};

__global__ __launch_bounds__(kFitThreads) void k_dt_fit(
    const double* __restrict__ t, const float* __restrict__ flux, const uint8_t* __restrict__ tr,
    int64_t n, const int32_t* __restrict__ seg, const int32_t* __restrict__ nseg_p,
    gpfc::DetrendParams prm, FitOut out, int32_t* __restrict__ status) {
    __shared__ double Ab[kDetrendMaxBasis * 4];   // band: A[i][i + d], d = 0..3
    __shared__ double rhs[kDetrendMaxBasis];
    __shared__ double cf[kDetrendMaxBasis];
    __shared__ int32_t sstart[kDetrendMaxBasis];  // first sample of each knot span (L + 1 used)
    __shared__ double red[kFitThreads / 64];
    __shared__ int64_t redi[kFitThreads / 64];
    __shared__ int32_t flag;
    const int tid = threadIdx.x;
    const int si = blockIdx.y;
    const double h = prm.spacings[si];
    const int32_t edge = prm.edge, max_fits = prm.max_fits;
    const double clip_sigma = prm.clip_sigma;
    const int32_t nseg = *nseg_p;
    for (int32_t sg = blockIdx.x; sg < nseg; sg += gridDim.x) {
        const int64_t s0 = seg[sg], s1 = seg[sg + 1], len = s1 - s0;
        int8_t* st = out.state + (int64_t)si * n;
        if (len <= 2 * (int64_t)edge) {
            if (tid == 0) st[s0] = 0;
            continue;
        }
        const double a = t[s0], span = t[s1 - 1] - a;
        const int L = span > 0.0 ? (int)fmax(1.0, ceil(span / h)) : 1;
        const double he = span > 0.0 ? span / (double)L : 1.0;
        const int m = L + 3;
        if (m > kDetrendMaxBasis) {
            if (tid == 0) { st[s0] = 0; atomicOr(status, 1); }
            continue;
        }
        // first sample of each span: binary search on the (monotone) span index
        for (int j = tid; j <= L; j += kFitThreads) {
            int64_t lo = s0, hi = s1;   // first k with span(k) >= j
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                double u;
                if (span_of(t[mid], a, he, L, u) >= j) hi = mid; else lo = mid + 1;
            }
            sstart[j] = (int32_t)(j == L ? s1 : lo);
        }
        uint8_t* cb[2] = {out.clip + ((int64_t)si * 2 + 0) * n, out.clip + ((int64_t)si * 2 + 1) * n};
        for (int64_t k = s0 + tid; k < s1; k += kFitThreads) cb[0][k] = 0;
        __syncthreads();
        int cur = 0;          // buffer of the clip set the next fit uses
        bool tried = false;
        double rss = 0.0;
        int64_t nuse = 0;
        for (int it = 0; it < max_fits; ++it) {
            const uint8_t* clip = cb[cur];
            // normal equations: thread per basis i over the samples of spans i-3 .. i
            int64_t cnt = 0;
            for (int i = tid; i < m; i += kFitThreads) {
                double acc[4] = {0.0, 0.0, 0.0, 0.0}, r = 0.0;
                const int j0 = i - 3 > 0 ? i - 3 : 0, j1 = i < L - 1 ? i : L - 1;
                for (int64_t k = sstart[j0]; k < sstart[j1 + 1]; ++k) {
                    if ((tr && tr[k]) || clip[k]) continue;
                    double u;
                    const int j = span_of(t[k], a, he, L, u);
                    const int o = i - j;
                    if (o < 0 || o > 3) continue;
                    double w[4];
                    bweights(u, w);
                    const double bi = w[o];
                    for (int d = 0; o + d <= 3; ++d) acc[d] += bi * w[o + d];
                    r += bi * (double)flux[k];
                }
                for (int d = 0; d < 4; ++d) Ab[i * 4 + d] = acc[d];
                rhs[i] = r;
            }
            for (int64_t k = s0 + tid; k < s1; k += kFitThreads) cnt += !((tr && tr[k]) || clip[k]);
            nuse = block_sum_i<kFitThreads>(cnt, redi);
            if (nuse < 2 * (int64_t)m) { tried = false; break; }
            // banded Cholesky (A = C C^T, bandwidth 3) and the two triangular solves
            if (tid == 0) {
                int ok = 1;
                for (int i = 0; i < m && ok; ++i) {
                    for (int d = 3; d >= 1; --d) {          // C[i][i-d]
                        const int jj = i - d;
                        if (jj < 0) continue;
                        double v = Ab[jj * 4 + d];
                        for (int e = d + 1; e <= 3; ++e) {
                            const int kk = i - e;          // columns kk < jj shared by rows i and jj
                            if (kk < 0) continue;
                            v -= Ab[kk * 4 + e] * Ab[kk * 4 + (e - d)];
                        }
                        Ab[jj * 4 + d] = v / Ab[jj * 4 + 0];
                    }
                    double dgn = Ab[i * 4 + 0];
                    for (int d = 1; d <= 3; ++d) {
                        const int jj = i - d;
                        if (jj >= 0) dgn -= Ab[jj * 4 + d] * Ab[jj * 4 + d];
                    }
                    if (!(dgn > 0.0) || !isfinite(dgn)) { ok = 0; break; }
                    Ab[i * 4 + 0] = sqrt(dgn);
                }
                if (ok) {
                    for (int i = 0; i < m; ++i) {           // C y = rhs
                        double v = rhs[i];
                        for (int d = 1; d <= 3; ++d)
                            if (i - d >= 0) v -= Ab[(i - d) * 4 + d] * cf[i - d];
                        cf[i] = v / Ab[i * 4 + 0];
                    }
                    for (int i = m - 1; i >= 0; --i) {      // C^T x = y
                        double v = cf[i];
                        for (int d = 1; d <= 3; ++d)
                            if (i + d < m) v -= Ab[i * 4 + d] * cf[i + d];
                        cf[i] = v / Ab[i * 4 + 0];
                    }
                }
                flag = ok;
            }
            __syncthreads();
            if (!flag) {
                if (tid == 0) atomicOr(status, 2);
                tried = false;
                break;
            }
            // residual scatter over the fitted points (ddof 0), two passes
            double sr = 0.0;
            for (int64_t k = s0 + tid; k < s1; k += kFitThreads) {
                if ((tr && tr[k]) || clip[k]) continue;
                double u, w[4];
                const int j = span_of(t[k], a, he, L, u);
                bweights(u, w);
                const double sk = w[0] * cf[j] + w[1] * cf[j + 1] + w[2] * cf[j + 2] + w[3] * cf[j + 3];
                sr += (double)flux[k] - sk;
            }
            const double rmean = block_sum<kFitThreads>(sr, red) / (double)nuse;
            double s2 = 0.0, q2 = 0.0;
            for (int64_t k = s0 + tid; k < s1; k += kFitThreads) {
                if ((tr && tr[k]) || clip[k]) continue;
                double u, w[4];
                const int j = span_of(t[k], a, he, L, u);
                bweights(u, w);
                const double sk = w[0] * cf[j] + w[1] * cf[j + 1] + w[2] * cf[j + 2] + w[3] * cf[j + 3];
                const double r = (double)flux[k] - sk;
                s2 += (r - rmean) * (r - rmean);
                q2 += r * r;
            }
            const double sig = sqrt(block_sum<kFitThreads>(s2, red) / (double)nuse);
            rss = block_sum<kFitThreads>(q2, red);
            // the next clip set, and whether it differs from this fit's
            uint8_t* nxt = cb[cur ^ 1];
            int64_t diff = 0;
            for (int64_t k = s0 + tid; k < s1; k += kFitThreads) {
                uint8_t c = 0;
                if (!(tr && tr[k])) {
                    double u, w[4];
                    const int j = span_of(t[k], a, he, L, u);
                    bweights(u, w);
                    const double sk = w[0] * cf[j] + w[1] * cf[j + 1] + w[2] * cf[j + 2] + w[3] * cf[j + 3];
                    c = fabs((double)flux[k] - sk) > clip_sigma * sig ? 1 : 0;
                }
                nxt[k] = c;
                diff += c != clip[k];
            }
            tried = true;
            if (block_sum_i<kFitThreads>(diff, redi) == 0) break;   // the set repeats
            if (it + 1 < max_fits) cur ^= 1;   // refit with the new set; else keep this fit's
            __syncthreads();
        }
        // publish: BIC, coefficients, the clip buffer of the kept fit
        if (tid == 0) {
            st[s0] = tried ? (int8_t)(1 + cur) : 0;
            if (tried)
                out.bic[(int64_t)si * n + s0] = rss > 0.0 ? (double)nuse * log(rss / (double)nuse) +
                                                                (double)m * log((double)nuse)
                                                          : -INFINITY;
        }
        if (tried)
            for (int i = tid; i < m; i += kFitThreads) out.coef[(int64_t)si * n + s0 + i] = cf[i];
        __syncthreads();
    }
}

// Per segment: the spacing of smallest BIC (ties: the earlier), the flux
// divided by its continuum, and the kept points (not clipped by that fit,
// at least `edge` points from both segment ends). Dropped segments give 0.
__global__ __launch_bounds__(256) void k_dt_apply(
    const double* __restrict__ t, const float* __restrict__ flux, int64_t n,
    const int32_t* __restrict__ seg, const int32_t* __restrict__ nseg_p, gpfc::DetrendParams prm,
    FitOut fo, double* __restrict__ out, uint8_t* __restrict__ keep, int32_t* __restrict__ chosen) {
    const int32_t nseg = *nseg_p;
    const int32_t ns = prm.n_spacings, edge = prm.edge;
    for (int32_t sg = blockIdx.x; sg < nseg; sg += gridDim.x) {
        const int64_t s0 = seg[sg], s1 = seg[sg + 1], len = s1 - s0;
        int best = -1;
        double bb = 0.0;
        if (len > 2 * (int64_t)edge)
            for (int si = 0; si < ns; ++si) {
                if (!fo.state[(int64_t)si * n + s0]) continue;
                const double b = fo.bic[(int64_t)si * n + s0];
                if (best < 0 || b < bb) { best = si; bb = b; }
            }
        if (threadIdx.x == 0 && chosen) chosen[sg] = best;
        if (best < 0) {
            for (int64_t k = s0 + threadIdx.x; k < s1; k += 256) { out[k] = 0.0; keep[k] = 0; }
            continue;
        }
        const double h = prm.spacings[best];
        const double a = t[s0], span = t[s1 - 1] - a;
        const int L = span > 0.0 ? (int)fmax(1.0, ceil(span / h)) : 1;
        const double he = span > 0.0 ? span / (double)L : 1.0;
        const double* cf = fo.coef + (int64_t)best * n + s0;
        const uint8_t* clip = fo.clip + ((int64_t)best * 2 + (fo.state[(int64_t)best * n + s0] - 1)) * n;
        for (int64_t k = s0 + threadIdx.x; k < s1; k += 256) {
            double u, w[4];
            const int j = span_of(t[k], a, he, L, u);
            bweights(u, w);
            const double sk = w[0] * cf[j] + w[1] * cf[j + 1] + w[2] * cf[j + 2] + w[3] * cf[j + 3];
            out[k] = (double)flux[k] / sk;
            keep[k] = (!clip[k] && k - s0 >= edge && s1 - 1 - k >= edge) ? 1 : 0;
        }
    }
}

}  // namespace gdt

namespace gpfc {
namespace {
// Clears the status word and the segment count.
__global__ void k_set2(int32_t* p) {
    if (threadIdx.x < 2) p[threadIdx.x] = 0;
}
}  // namespace
}  // namespace gpfc

namespace gpfc {

namespace {
size_t al256(size_t x) { return (x + 255) & ~size_t(255); }
}

// Workspace: segment starts (n + 2), status and segment count (256 bytes),
// the chosen spacing per segment (n), then per spacing: BIC (n), coefficients
// (n), two clip-flag buffers (2n) and the fit state (n).
size_t detrend_workspace_bytes(int64_t n, int32_t ns) {
    const size_t nn = (size_t)(n > 0 ? n : 1);
    return al256((nn + 2) * 4) + 256 + al256(nn * 4) + 2 * al256(ns * nn * 8) + al256(ns * nn * 2) +
           al256(ns * nn);
}

DetrendWs detrend_carve(void* ws, int64_t n, int32_t ns) {
    const size_t nn = (size_t)(n > 0 ? n : 1);
    char* p = (char*)ws;
    DetrendWs w;
    w.seg = (int32_t*)p; p += al256((nn + 2) * 4);
    w.status = (int32_t*)p;
    w.nseg = w.status + 1;
    p += 256;
    w.chosen = (int32_t*)p; p += al256(nn * 4);
    w.bic = (double*)p; p += al256(ns * nn * 8);
    w.coef = (double*)p; p += al256(ns * nn * 8);
    w.clip = (uint8_t*)p; p += al256(ns * nn * 2);
    w.state = (int8_t*)p;
    return w;
}

hipError_t launch_detrend(const double* t, const float* flux, const uint8_t* tr, int64_t n,
                          const DetrendParams& prm, const DetrendWs& w, double* out, uint8_t* keep,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_set2, dim3(1), dim3(64), 0, s, w.status);
    hipLaunchKernelGGL(gdt::k_dt_segments, dim3(1), dim3(1024), 0, s, t, flux, tr, n,
                       prm.gap_cadences * prm.cadence, prm.jump_sigma, w.seg, w.nseg);
    gdt::FitOut fo{w.bic, w.coef, w.clip, w.state};
    const unsigned g = (unsigned)std::min<int64_t>(std::max<int64_t>(n / 64, 1), 512);
    hipLaunchKernelGGL(gdt::k_dt_fit, dim3(g, (unsigned)prm.n_spacings), dim3(gdt::kFitThreads), 0, s,
                       t, flux, tr, n, w.seg, w.nseg, prm, fo, w.status);
    hipLaunchKernelGGL(gdt::k_dt_apply, dim3(g), dim3(256), 0, s, t, flux, n, w.seg, w.nseg, prm, fo,
                       out, keep, w.chosen);
    return hipGetLastError();
}

}  // namespace gpfc
