// HIP kernels for gfx950 (MI355X): curve statistics, fixed-point packing,
// the LDS phase fold, the fused fold + box-SNR, box-SNR of materialised
// folds, and the plain global-atomic fold used as the baseline.
//
// Method: GPU phase folding (Sec. 2.3 of arXiv:2312.02063) with equal-width
// phase bins, scored by the box statistic built from Eq. 2 (Sec. 2.6) and
// the BLS box (Sec. 3.1).
#include <math.h>

#include <algorithm>
#include <type_traits>

#include "gpfc_internal.h"

namespace gpfc {

// Set to 1 by k_curve_stats when a curve holds a non-finite time or flux;
// read and cleared by take_input_fault (the next synchronisation).
__device__ int32_t g_input_fault = 0;

namespace {

constexpr int kWaves = 16;                 // waves per fold block: 4 per SIMD
constexpr int kThreads = kWaves * 64;
constexpr int kRowsPerWave = kFineBins / kWaves;
constexpr int kHalfBytes = kFineBins * 32 * 8;   // one half of the histogram: 32 lanes

// ------------------------------------------------------------------ reductions

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_or_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
    return v;
}

// ------------------------------------------------------------------ curve statistics

// One block of 1024 threads. Pass 1: sum of flux, max |t|, finiteness and the
// finest binary exponent of the fluxes; pass 2: sum of squared deviations and
// the largest deviation from the grid-rounded reference. The fixed-point unit
// 2^e0 is the ulp of the smallest-magnitude flux, so flux - ref is an exact
// integer multiple of it (ref a multiple of 2^e0). One packed word per sample
// holds deviations below 2^27 units; two words (high and low, 27 bits apart)
// hold them below 2^53 units, still exactly. Past that the low word's unit is
// coarsened to leave 53 bits for the largest deviation, and each sample's
// deviation is rounded to it (exact = 0): an error of at most one unit, about
// maxdev 2^-52, per sample.
//
// Block c handles curve c: samples [soff[c], soff[c+1]) (or [0, n1) when soff
// is null), result in info[c].
__global__ __launch_bounds__(1024) void k_curve_stats(const double* __restrict__ t,
                                                      const float* __restrict__ flux,
                                                      const int64_t* __restrict__ soff, int64_t n1,
                                                      CurveInfo* __restrict__ info) {
    const int64_t i0 = soff ? soff[blockIdx.x] : 0;
    const int64_t n = soff ? soff[blockIdx.x + 1] - i0 : n1;
    t += i0;
    flux += i0;
    info += blockIdx.x;
    __shared__ double sd[16];
    __shared__ double sd2[16];
    __shared__ int si[16];
    __shared__ int si2[16];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    double s = 0.0, tm = 0.0;
    int emin = 1 << 20, bad = 0;
    for (int64_t i = tid; i < n; i += 1024) {
        const float fv = flux[i];
        const double a = fabs(t[i]);
        s += (double)fv;
        if (!(a <= 1.7976931348623157e308)) bad = 1;
        else tm = fmax(tm, a);
        if (!isfinite(fv)) bad = 1;
        else if (fv != 0.0f) emin = min(emin, ilogbf(fv));
    }
    s = wave_sum(s);
    tm = wave_max(tm);
    emin = wave_min_i(emin);
    bad = wave_or_i(bad);
    if (lane == 0) { sd[wv] = s; sd2[wv] = tm; si[wv] = emin; si2[wv] = bad; }
    __syncthreads();
    double S = 0.0, TM = 0.0;
    int EMIN = 1 << 20, BAD = 0;
    for (int j = 0; j < 16; ++j) { S += sd[j]; TM = fmax(TM, sd2[j]); EMIN = min(EMIN, si[j]); BAD |= si2[j]; }
    __syncthreads();
    const double mean = n > 0 ? S / (double)n : 0.0;
    const int e0 = EMIN == (1 << 20) ? -24 : max(EMIN - 23, -149);
    double ref = ldexp(rint(ldexp(mean, -e0)), e0);
    double ss = 0.0, md = 0.0;
    for (int64_t i = tid; i < n; i += 1024) {
        const double f = (double)flux[i];
        const double d = f - mean;
        ss += d * d;
        md = fmax(md, fabs(f - ref));
    }
    ss = wave_sum(ss);
    md = wave_max(md);
    if (lane == 0) { sd[wv] = ss; sd2[wv] = md; }
    __syncthreads();
    if (tid == 0) {
        double SS = 0.0, MD = 0.0;
        for (int j = 0; j < 16; ++j) { SS += sd[j]; MD = fmax(MD, sd2[j]); }
        int words = 1, exact = 1, e = e0, e_lo = e0;
        if (BAD) {
            exact = 0;
            g_input_fault = 1;
        } else if (!(MD < ldexp(1.0, e0 + 27))) {
            words = 2;
            if (!(MD < ldexp(1.0, e0 + 53))) {
                exact = 0;
                e_lo = ilogb(MD) - 52;
                ref = ldexp(rint(ldexp(mean, -e_lo)), e_lo);
            }
            e = e_lo + kLoBits;
        }
        CurveInfo ci;
        ci.mean = mean;
        ci.sigma = n > 1 ? sqrt(SS / (double)(n - 1)) : 0.0;
        ci.ref = ref;
        ci.qscale = ldexp(1.0, e);
        ci.tmax = BAD ? __builtin_inf() : TM;
        ci.maxdev = MD;
        ci.n = n;
        ci.e = e;
        ci.exact = exact;
        ci.finite = BAD ? 0 : 1;
        ci.words = words;
        ci.e_lo = e_lo;
        ci.pad = 0;
        *info = ci;
    }
}

// Prepared curve: record i = {t_i, (1 << 46) + (q_i + 2^27)} with
// q_i = RN((flux_i - ref) / 2^e) for a one-word curve. For a two-word curve
// q_i = RN((flux_i - ref) / 2^e_lo) (exact unless the curve is flagged
// inexact) is split as q_hi 2^27 + q_lo, |q_lo| <= 2^26: the record holds
// q_hi's packed word and lo[i] = (1 << 46) + (q_lo + 2^27). Records from n up
// to `total` are {0, 0} (and lo 0): they add nothing to any bin, so folds can
// run over whole blocks of records without a tail. Block row y handles curve
// y: samples [soff[y], soff[y+1]) into records [roff[y], roff[y+1]) (one
// curve of n1 samples and total1 records when soff is null).
__global__ __launch_bounds__(256) void k_pack(const double* __restrict__ t,
                                              const float* __restrict__ flux,
                                              const int64_t* __restrict__ soff, int64_t n1,
                                              const int64_t* __restrict__ roff, int64_t total1,
                                              const CurveInfo* __restrict__ info,
                                              Rec* __restrict__ rec, uint64_t* __restrict__ lo) {
    const int c = blockIdx.y;
    const int64_t i0 = soff ? soff[c] : 0;
    const int64_t n = soff ? soff[c + 1] - i0 : n1;
    const int64_t r0 = soff ? roff[c] : 0;
    const int64_t total = soff ? roff[c + 1] - r0 : total1;
    t += i0;
    flux += i0;
    rec += r0;
    lo += r0;
    info += c;
    const double ref = info->ref;
    const bool two = info->words == 2;
    const int e = two ? info->e_lo : info->e;
    const double lim = two ? 0x1p53 : (double)kBias;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        Rec r{0.0, 0};
        uint64_t rl = 0;
        if (i < n) {
            double q = rint(ldexp((double)flux[i] - ref, -e));
            q = fmin(fmax(q, -lim), lim);
            r.t = t[i];
            if (two) {
                const double qh = rint(ldexp(q, -kLoBits));
                const double ql = q - ldexp(qh, kLoBits);   // exact, |ql| <= 2^26
                r.c = (uint64_t(1) << kCountShift) + (uint64_t)((int64_t)qh + kBias);
                rl = (uint64_t(1) << kCountShift) + (uint64_t)((int64_t)ql + kBias);
            } else {
                r.c = (uint64_t(1) << kCountShift) + (uint64_t)((int64_t)q + kBias);
            }
        }
        rec[i] = r;
        if (two) lo[i] = rl;
    }
}

// ------------------------------------------------------------------ phase bin

// The IEEE sequence of the fold's bin definition at 256 fine bins:
// x = RN(t / P); f = x - floor(x); b = floor(256 f) clamped to 255; NaN -> 0.
// Used for the rare updates the fast path cannot certify.
__device__ __forceinline__ uint32_t fine_bin_ieee(double t, double P) {
    const double x = t / P;
    const double f = x - floor(x);
    const double fb = floor(f * 256.0);
    if (!(fb >= 0.0)) return 0u;
    if (fb >= 256.0) return 255u;
    return (uint32_t)fb;
}

// Per-lane constants of the certified fast path (see fast_lo).
struct LaneSetup {
    double P;         // the lane's period (1.0 for an invalid lane)
    double rB;        // 256 * RN(1/P), an exact scaling of RN(1/P)
    uint32_t lim;     // 65536 - 2, or 0 when the fast path is off for the lane
    bool valid;
};

// Added inside the phase FMA: 1.5 * 2^36 - 2^-16, exactly representable (the
// binade [2^36, 2^37) has spacing 2^-16).
constexpr double kPhaseC = 0x1.8p36 - 0x1p-16;

__device__ __forceinline__ LaneSetup lane_setup(const double* __restrict__ periods, int64_t kk,
                                                int64_t k, double tmax) {
    LaneSetup L;
    double P = kk < k ? periods[kk] : 1.0;
    L.valid = kk < k && P > 0.0 && isfinite(P);
    if (!L.valid) P = 1.0;
    L.P = P;
    L.rB = (1.0 / P) * 256.0;
    // |t rB - 256 RN(t/P)| <= 2u zmax (1 + u), u = 2^-53: below 2^-18
    // whenever zmax = max|t| rB < 2^34, which also keeps t rB + kPhaseC in
    // the binade of kPhaseC.
    const double zmax = tmax * L.rB;
    const bool fast = zmax < 0x1p34;   // false for NaN / inf
    L.lim = fast ? 65536u - 2u : 0u;
    return L;
}

// ------------------------------------------------------------------ the LDS fold

// Accumulate one wave's slice of the curve into the block's histogram.
//
// Lane j of every wave owns trial period blockIdx*64 + j; the 16 waves split
// the samples. A sample's time and packed contribution are the same for the
// whole wave (scalar loads). The histogram bin of (sample, lane) lives at byte
// half*65536 + bin*256 + (j & 31)*8, half = j >> 5: the 16 lanes of a 64-bit
// LDS access hit 32 distinct banks, so every update is one conflict-free
// ds_add_u64.
//
// Fast path, certified: y = fma(t, 256 RN(1/P), kPhaseC) rounds t * rB once,
// to the 2^-16 grid of kPhaseC's binade, so the low 32 bits of y hold G - 1,
// G = round(2^16 t rB) (2^52 * 1.5 vanishes mod 2^32): bits [16, 24) are the
// bin and bits [0, 16) the fraction shifted down by one unit. With z = 256
// RN(t/P), the IEEE sequence's bin is floor(z) mod 256 and |G 2^-16 - z| <=
// 2^-17 + 2^-18 < 2^-16; a fraction field below 65534 means G mod 2^16 lies in
// [1, 65534], so z is strictly inside the unit interval of (G - 1) 2^-16 and
// the bin field is exact. Otherwise (about 2 updates in 65536) the lane
// recomputes the bin with the IEEE sequence.
__device__ __forceinline__ void lds_add(char* hist, uint32_t addr, uint64_t v) {
    __hip_atomic_fetch_add(reinterpret_cast<uint64_t*>(hist + addr), v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ uint32_t fast_lo(double ti, double rB) {
    return (uint32_t)__double_as_longlong(__builtin_fma(ti, rB, kPhaseC));
}

// byte0 <- laneoff.byte0, byte1 <- lo.byte2 (the bin), byte2 <- laneoff.byte2
__device__ __forceinline__ uint32_t fast_addr(uint32_t lo, uint32_t laneoff) {
    return __builtin_amdgcn_perm(lo, laneoff, 0x0C020600u);
}

// One update on the fast path; returns its low word, whose fraction field the
// caller checks against the certificate (the contribution goes to the fast
// bin either way).
__device__ __forceinline__ uint32_t fold_update(char* hist, double ti, uint64_t ci, double rB,
                                                uint32_t laneoff) {
    const uint32_t lo = fast_lo(ti, rB);
    lds_add(hist, fast_addr(lo, laneoff), ci);
    return lo;
}

// Largest fraction field (low 16 bits) of three words, in the low 16 bits of
// the result: one v_max3_u16, which the compiler does not form by itself.
__device__ __forceinline__ uint32_t max3_frac(uint32_t m, uint32_t a, uint32_t b) {
    uint32_t r;
    asm("v_max3_u16 %0, %1, %2, %3" : "=v"(r) : "v"(m), "v"(a), "v"(b));
    return r;
}

// Rare repair of a block in which some lane failed the certificate: for each
// such update, take the contribution back out of the fast bin and put it in
// the bin of the IEEE sequence (integer adds, so this is exact). A two-word
// fold (kTwo) gives lanes 32-63 the low words `blo`.
template <bool kTwo>
__device__ __forceinline__ void fold_repair(char* hist, const Rec* blk, const uint64_t* blo,
                                            int cnt, LaneSetup L, uint32_t laneoff, bool upper) {
    for (int j = 0; j < cnt; ++j) {
        const double ti = blk[j].t;
        const uint64_t ci = (kTwo && upper) ? blo[j] : blk[j].c;
        const uint32_t lo = fast_lo(ti, L.rB);
        if ((lo & 0xFFFFu) >= L.lim) {
            lds_add(hist, fast_addr(lo, laneoff), uint64_t(0) - ci);
            lds_add(hist, (fine_bin_ieee(ti, L.P) << 8) | laneoff, ci);
        }
    }
}

// Records come in through scalar loads, kBlk per request, two requests per
// chunk of 2 kBlk: the second half of a chunk is requested before the first
// is processed and the next chunk's first half before the second is
// processed, so each wait (which also covers the LDS atomics already issued)
// sits kBlk updates after its request.
constexpr int kBlk = 8;

// Wait for every outstanding scalar load and LDS operation, and keep the
// scheduler from moving work across the wait.
__device__ __forceinline__ void wait_lgkm() {
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0), vmcnt and expcnt untouched
    __builtin_amdgcn_sched_barrier(0);
}

// Fold a block's records with the chunks handed out dynamically: each wave
// takes the next chunk index from a counter in LDS (one lane's atomic, read
// after the next wait), so waves that the LDS arbiter serves less often
// take fewer chunks and all finish together; with fixed equal slices the
// last-served waves ran alone for a fifth of the fold. The sums are
// integers, so the order of the updates does not change them. Chunk c lies
// at offset (c / cps) * stride + (c % cps) * 2 kBlk from rec (cps chunks per
// segment, segments `stride` records apart), or at c * 2 kBlk when kContig.
// kTwo: lanes 32-63 add the low words lo[] of the same records (lanes j and
// j + 32 fold the same period into the two halves of the histogram).
template <bool kContig, bool kTwo>
__device__ __forceinline__ void fold_chunks(char* hist, uint32_t* ctr, const Rec* __restrict__ rec,
                                            const uint64_t* __restrict__ lo, int64_t nch,
                                            int64_t cps, int64_t stride, const LaneSetup& L,
                                            uint32_t laneoff, int lane) {
    auto at = [&](int64_t c) -> int64_t {
        if (kContig) return c * (2 * kBlk);
        const int64_t sg = c / cps;
        return sg * stride + (c - sg * cps) * (2 * kBlk);
    };
    const bool upper = lane >= 32;
    // ds_inc_rtn (an increment that wraps at 2^32 - 1): unlike an add, the
    // compiler does not rewrite it into a wave-level pattern that waits for
    // the returned value at once
    auto grab = [&]() -> uint32_t {
        uint32_t v = 0;
        if (lane == 0) v = atomicInc(ctr, 0xFFFFFFFFu);
        return v;
    };
    int64_t c = (int64_t)__builtin_amdgcn_readfirstlane(grab());
    if (c >= nch) return;
    int64_t o = at(c);
    const Rec* p = rec + o;
    Rec a[kBlk], b[kBlk];
    uint64_t la[kBlk], lb[kBlk];
#pragma unroll
    for (int j = 0; j < kBlk; ++j) a[j] = p[j];
    if (kTwo) {
#pragma unroll
        for (int j = 0; j < kBlk; ++j) la[j] = lo[o + j];
    }
    uint32_t vn = grab();
    for (;;) {
        wait_lgkm();
#pragma unroll
        for (int j = 0; j < kBlk; ++j) b[j] = p[kBlk + j];
        if (kTwo) {
#pragma unroll
            for (int j = 0; j < kBlk; ++j) lb[j] = lo[o + kBlk + j];
        }
        __builtin_amdgcn_sched_barrier(0);
        uint32_t m = 0;
#pragma unroll
        for (int j = 0; j < kBlk; j += 2) {
            const uint64_t c0 = (kTwo && upper) ? la[j] : a[j].c;
            const uint64_t c1 = (kTwo && upper) ? la[j + 1] : a[j + 1].c;
            m = max3_frac(m, fold_update(hist, a[j].t, c0, L.rB, laneoff),
                          fold_update(hist, a[j + 1].t, c1, L.rB, laneoff));
        }
        if (__builtin_amdgcn_uicmp(m & 0xFFFFu, L.lim, 35 /* unsigned >= */))
            fold_repair<kTwo>(hist, p, lo + o, kBlk, L, laneoff, upper);
        const int64_t cn = (int64_t)__builtin_amdgcn_readfirstlane(vn);
        const bool more = cn < nch;
        const int64_t on = more ? at(cn) : o;
        const Rec* pn = rec + on;
        wait_lgkm();
        if (more) {
#pragma unroll
            for (int j = 0; j < kBlk; ++j) a[j] = pn[j];
            if (kTwo) {
#pragma unroll
                for (int j = 0; j < kBlk; ++j) la[j] = lo[on + j];
            }
            vn = grab();
        }
        __builtin_amdgcn_sched_barrier(0);
        m = 0;
#pragma unroll
        for (int j = 0; j < kBlk; j += 2) {
            const uint64_t c0 = (kTwo && upper) ? lb[j] : b[j].c;
            const uint64_t c1 = (kTwo && upper) ? lb[j + 1] : b[j + 1].c;
            m = max3_frac(m, fold_update(hist, b[j].t, c0, L.rB, laneoff),
                          fold_update(hist, b[j + 1].t, c1, L.rB, laneoff));
        }
        if (__builtin_amdgcn_uicmp(m & 0xFFFFu, L.lim, 35 /* unsigned >= */))
            fold_repair<kTwo>(hist, p + kBlk, lo + o + kBlk, kBlk, L, laneoff, upper);
        if (!more) break;
        p = pn;
        o = on;
    }
}

__device__ __forceinline__ uint32_t hist_off(int row, int lane) {
    return (uint32_t)((lane >> 5) * kHalfBytes + row * 256 + (lane & 31) * 8);
}

__device__ __forceinline__ void decode(uint64_t v, double qscale, uint32_t& cnt, double& dev) {
    cnt = (uint32_t)(v >> kCountShift);
    const int64_t sq = (int64_t)(v & kSumMask) - (int64_t)cnt * kBias;
    dev = (double)sq * qscale;
}

// Two-word decode: the count from the high word, the deviation from both
// (the integer sums scaled by their units; one FP64 rounding each).
__device__ __forceinline__ void decode2(uint64_t vh, uint64_t vl, double qs_hi, double qs_lo,
                                        uint32_t& cnt, double& dev) {
    cnt = (uint32_t)(vh >> kCountShift);
    const int64_t sh = (int64_t)(vh & kSumMask) - (int64_t)cnt * kBias;
    const int64_t sl = (int64_t)(vl & kSumMask) - (int64_t)cnt * kBias;
    dev = (double)sh * qs_hi + (double)sl * qs_lo;
}

// The block's histogram of its periods over all kWaves * per records (one
// word: 64 periods; two words: 32 periods, high words in half 0 and low words
// in half 1).
template <bool kTwo>
__device__ __forceinline__ void fold_block(char* hist, const Rec* __restrict__ rec,
                                           const uint64_t* __restrict__ lo, int64_t per,
                                           const LaneSetup& L, int lane, int wave) {
    __shared__ uint32_t ctr;
    uint64_t* h64 = reinterpret_cast<uint64_t*>(hist);
    for (int i = threadIdx.x; i < kFineBins * 64; i += kThreads) h64[i] = 0;
    if (threadIdx.x == 0) ctr = 0u;
    __syncthreads();
    const uint32_t laneoff = (uint32_t)((lane & 31) * 8 + (lane >> 5) * kHalfBytes);
    const int64_t nch = per * kWaves / (2 * kBlk);
    fold_chunks<true, kTwo>(hist, &ctr, rec, lo, nch, nch, 0, L, laneoff, lane);
    __syncthreads();
}

// Period index of a lane: one word, kbase + lane; two words, pass `half`
// of the block's 64 periods, kbase + 32 half + (lane & 31).
__device__ __forceinline__ int64_t lane_period(int64_t kbase, int lane, bool two, int half) {
    return two ? kbase + 32 * half + (lane & 31) : kbase + lane;
}

// Bin sums, counts and means of a block's periods from its histogram. One
// word: every lane writes its period. Two words: lanes 0-31 combine their high
// words with their partner lanes' low words and write, lanes 32-63 idle.
template <bool kTwo>
__device__ __forceinline__ void fold_flush(const char* hist, const CurveInfo* __restrict__ info,
                                           const LaneSetup& L, int64_t kk, int64_t k, int log2g,
                                           int lane, int wave, double* __restrict__ sums,
                                           int32_t* __restrict__ counts,
                                           double* __restrict__ means) {
    if (kk >= k || (kTwo && lane >= 32)) return;
    const int g = 1 << log2g;
    const int nb = kFineBins >> log2g;
    const double ref = info->ref, qs = info->qscale, qlo = ldexp(1.0, info->e_lo);
    auto bin = [&](int b, double& s, int32_t& c, double& m) {
        uint64_t acc = 0, acl = 0;
        for (int j = 0; j < g; ++j) {
            acc += *reinterpret_cast<const uint64_t*>(hist + hist_off(b * g + j, lane));
            if (kTwo) acl += *reinterpret_cast<const uint64_t*>(hist + hist_off(b * g + j, lane + 32));
        }
        uint32_t cu;
        double d;
        if (kTwo) decode2(acc, acl, qs, qlo, cu, d);
        else decode(acc, qs, cu, d);
        s = L.valid ? (double)cu * ref + d : 0.0;
        if (!L.valid) cu = 0;
        c = (int32_t)cu;
        m = cu ? s / (double)cu : __builtin_nan("");
    };
    const bool aligned = ((((uintptr_t)sums | (uintptr_t)means) & 15) | ((uintptr_t)counts & 7)) == 0;
    if (nb >= 2 * kWaves && aligned) {
        // each wave a contiguous run of bins of every period, written as bin
        // pairs: 16-byte sums and means, 8-byte counts (the caller's buffers
        // aligned to those sizes; otherwise the loop below)
        const int per_wave = nb / kWaves;
        for (int b = wave * per_wave; b < (wave + 1) * per_wave; b += 2) {
            double s0, s1, m0, m1;
            int32_t c0, c1;
            bin(b, s0, c0, m0);
            bin(b + 1, s1, c1, m1);
            const int64_t o = kk * nb + b;
            *reinterpret_cast<double2*>(sums + o) = make_double2(s0, s1);
            *reinterpret_cast<int2*>(counts + o) = make_int2(c0, c1);
            if (means) *reinterpret_cast<double2*>(means + o) = make_double2(m0, m1);
        }
        return;
    }
    for (int b = wave; b < nb; b += kWaves) {
        double s, m;
        int32_t c;
        bin(b, s, c, m);
        const int64_t o = kk * nb + b;
        sums[o] = s;
        counts[o] = c;
        if (means) means[o] = m;
    }
}

__global__ __launch_bounds__(kThreads, 1) void k_fold(
    const Rec* __restrict__ rec, const uint64_t* __restrict__ lo, int64_t per,
    const double* __restrict__ periods, int64_t k, int32_t log2g,
    const CurveInfo* __restrict__ info, double* __restrict__ sums, int32_t* __restrict__ counts,
    double* __restrict__ means) {
    __shared__ __attribute__((aligned(16))) char hist[kFineBins * 64 * 8];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t kbase = (int64_t)blockIdx.x * 64;
    if (info->words == 2) {
        for (int half = 0; half < 2; ++half) {
            const int64_t kk = lane_period(kbase, lane, true, half);
            const LaneSetup L = lane_setup(periods, kk, k, info->tmax);
            fold_block<true>(hist, rec, lo, per, L, lane, wave);
            fold_flush<true>(hist, info, L, kk, k, log2g, lane, wave, sums, counts, means);
            __syncthreads();
        }
        return;
    }
    const int64_t kk = kbase + lane;
    const LaneSetup L = lane_setup(periods, kk, k, info->tmax);
    fold_block<false>(hist, rec, lo, per, L, lane, wave);
    fold_flush<false>(hist, info, L, kk, k, log2g, lane, wave, sums, counts, means);
}

// ------------------------------------------------------------------ FP32 fold sums (precision study)

// Fold with FP32 bin sums accumulated by float LDS atomics, plain or
// compensated: with kTwoSum the atomic returns the old sum, the lane
// recomputes the rounded new sum and its exact error (TwoSum, Knuth) and adds
// the error into a second float array. Deviations enter as flux - ref (from
// the packed words) rounded to FP32. 32 periods per block (lanes 32-63 idle):
// counts u32, sums f32 and errors f32 at [bin][32] fill 96 KB. Bins use the
// certified fast path with a per-update IEEE fallback.
template <bool kTwoSum>
__global__ __launch_bounds__(kThreads, 1) void k_fold_f32(
    const Rec* __restrict__ rec, const uint64_t* __restrict__ lo, int64_t per,
    const double* __restrict__ periods, int64_t k,
    int32_t log2g, const CurveInfo* __restrict__ info, double* __restrict__ sums,
    int32_t* __restrict__ counts, double* __restrict__ means) {
    __shared__ uint32_t hc[kFineBins * 32];
    __shared__ float hs[kFineBins * 32];
    __shared__ float he[kFineBins * 32];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t kk = (int64_t)blockIdx.x * 32 + (lane & 31);
    const LaneSetup L = lane_setup(periods, kk, k, info->tmax);
    for (int i = threadIdx.x; i < kFineBins * 32; i += kThreads) { hc[i] = 0; hs[i] = 0.0f; he[i] = 0.0f; }
    __syncthreads();
    const double qs = info->qscale, qlo = ldexp(1.0, info->e_lo);
    const bool two = info->words == 2;
    const Rec* p = rec + (int64_t)wave * per;
    const uint64_t* pl = lo + (int64_t)wave * per;
    if (lane < 32) {
        for (int64_t i = 0; i < per; ++i) {
            const double ti = p[i].t;
            const uint64_t ci = p[i].c;
            if (ci == 0) continue;   // padding record
            const uint32_t lw = fast_lo(ti, L.rB);
            uint32_t bin = (lw >> 16) & 255u;
            if ((lw & 0xFFFFu) >= L.lim) bin = fine_bin_ieee(ti, L.P);
            const int j = (int)bin * 32 + lane;
            // flux - ref rounded to FP32
            double xd = (double)((int64_t)(ci & kSumMask) - kBias) * qs;
            if (two) xd += (double)((int64_t)(pl[i] & kSumMask) - kBias) * qlo;
            const float x = (float)xd;
            atomicAdd(&hc[j], 1u);
            if (kTwoSum) {
                const float old = atomicAdd(&hs[j], x);
                const float s = old + x;
                const float bp = s - old;
                const float err = (old - (s - bp)) + (x - bp);
                atomicAdd(&he[j], err);
            } else {
                atomicAdd(&hs[j], x);
            }
        }
    }
    __syncthreads();
    if (lane >= 32 || kk >= k) return;
    const int g = 1 << log2g;
    const int nb = kFineBins >> log2g;
    const double ref = info->ref;
    for (int b = wave; b < nb; b += kWaves) {
        uint32_t c = 0;
        double d = 0.0;
        for (int jj = 0; jj < g; ++jj) {
            const int j = (b * g + jj) * 32 + lane;
            c += hc[j];
            d += (double)hs[j] + (double)he[j];
        }
        if (!L.valid) { c = 0; d = 0.0; }
        const double sm = c ? (double)c * ref + d : 0.0;
        const int64_t o = kk * nb + b;
        sums[o] = sm;
        counts[o] = (int32_t)c;
        if (means) means[o] = c ? sm / (double)c : __builtin_nan("");
    }
}

// ------------------------------------------------------------------ box scan

// Slot (row r, period lane j) of the prefix table that replaces the
// histogram in place: inclusive prefixes over rows of the count (float,
// exact below 2^24) and of n times the flux-deviation sum (float).
struct alignas(8) Slot {
    float c;
    float dn;
};

__device__ __forceinline__ Slot slot_at(const char* tab, int row, int lane) {
    return *reinterpret_cast<const Slot*>(tab + hist_off(row, lane));
}

// Box value proportional to the box SNR (the row's common factor
// 1/(sigma sqrt(n)) dropped): (S cin - n din) / sqrt(cin (n - cin)), from the
// box count cin and dn_in = n din. kChecked = false assumes 0 < cin < n or
// cin = 0 (then dn_in = 0 exactly and the value is NaN, which fmaxf skips);
// kChecked = true returns 0 for an empty or full box.
template <bool kChecked>
__device__ __forceinline__ float box_value(float cin, float dn_in, float nf, float Sf) {
    const float cout = nf - cin;
    const float num = __builtin_fmaf(Sf, cin, -dn_in);
    const float v = num * __builtin_amdgcn_rsqf(cin * cout);
    if (kChecked) return (cin > 0.5f && cout > 0.5f) ? v : 0.0f;
    return v;
}

// Prefix of coarse boundary b (0..nb) for a table with `g` rows per coarse bin.
__device__ __forceinline__ Slot coarse_prefix(const char* tab, int b, int g, int lane) {
    if (b == 0) return Slot{0.0f, 0.0f};
    return slot_at(tab, b * g - 1, lane);
}

// Largest box value of width w over the circular starts [s0, s1) of one row.
// Starts whose box wraps past the last bin add the row total to the end
// prefix; start 0 takes the end prefix alone. kG1: one fine row per coarse
// bin (g = 1), so consecutive starts are consecutive rows and the slot
// addresses of an unrolled step differ by constants.
template <bool kChecked, bool kG1>
__device__ float scan_range(const char* tab, int w, int s0, int s1, int nb, int g_rt, int lane,
                            float nf, float Sf, Slot tot) {
    const int g = kG1 ? 1 : g_rt;
    float best = 0.0f;
    int s = s0;
    if (s == 0) {
        const Slot e = coarse_prefix(tab, w, g, lane);
        best = fmaxf(best, box_value<kChecked>(e.c, e.dn, nf, Sf));
        s = 1;
    }
    const int m1 = min(s1, nb - w + 1);   // boxes that end inside the row: s + w <= nb
    if (kG1) {
        const char* pa = tab + hist_off(s - 1, lane);
        const char* pe = pa + w * 256;
#pragma unroll 4
        for (; s < m1; ++s, pa += 256, pe += 256) {
            const Slot a = *reinterpret_cast<const Slot*>(pa);
            const Slot e = *reinterpret_cast<const Slot*>(pe);
            best = fmaxf(best, box_value<kChecked>(e.c - a.c, e.dn - a.dn, nf, Sf));
        }
        pe -= nb * 256;
#pragma unroll 4
        for (; s < s1; ++s, pa += 256, pe += 256) {
            const Slot a = *reinterpret_cast<const Slot*>(pa);
            const Slot e = *reinterpret_cast<const Slot*>(pe);
            best = fmaxf(best, box_value<kChecked>((e.c + tot.c) - a.c, (e.dn + tot.dn) - a.dn, nf, Sf));
        }
        return best;
    }
#pragma unroll 4
    for (; s < m1; ++s) {
        const Slot a = slot_at(tab, s * g - 1, lane);
        const Slot e = slot_at(tab, (s + w) * g - 1, lane);
        best = fmaxf(best, box_value<kChecked>(e.c - a.c, e.dn - a.dn, nf, Sf));
    }
#pragma unroll 4
    for (; s < s1; ++s) {
        const Slot a = slot_at(tab, s * g - 1, lane);
        const Slot e = slot_at(tab, (s + w - nb) * g - 1, lane);
        best = fmaxf(best, box_value<kChecked>((e.c + tot.c) - a.c, (e.dn + tot.dn) - a.dn, nf, Sf));
    }
    return best;
}

// Per-block scratch of the scorer.
struct ScoreShared {
    float nrow[64];       // samples per period (float)
    double Srow[64];      // flux-deviation total per period
    int32_t nz[64];       // non-empty coarse bins per period
    float bestv[kFusedWidths * 64];
    int32_t first[kWaves * 64];
    int32_t nzc[kWaves * 64];
};

// Shared tail of the fused and the materialised scorer. The prefix table of
// the block's 64 periods is in `tab`, per-period totals in sh. The (width,
// start) boxes are cut into 16 equal runs of consecutive starts, one per
// wave, each covering at most two widths; a wave's run maximum of a width is
// merged into that width's maximum by an integer max of the bit patterns
// (exact: every value is >= +0). A period whose samples fill more coarse
// bins than the widest box can hold is scanned without per-box checks (no
// box can be full; an empty box gives NaN, which the max skips); the others
// use the checked form. Then every wave evaluates the winning width at its
// own range of starts and keeps the first start whose value equals the
// maximum, and wave 0 takes the smallest and evaluates the box in FP64.
//
// kTwo: the table holds 32 periods (lanes j and j + 32 both stand for period
// j, reading table lane j); only lanes 0-31 write results.
template <bool kTwo>
__device__ void score_table(const char* tab, int nb, int g, const Widths& W, ScoreShared& sh,
                            double sigma, bool valid, int64_t kk, int64_t k, int lane, int wave,
                            float* snr, int32_t* start, int32_t* width, float* depth) {
    const int tl = kTwo ? (lane & 31) : lane;   // the lane's column of the table
    const float nf = sh.nrow[tl];
    const float Sf = (float)sh.Srow[tl];
    const Slot tot = coarse_prefix(tab, nb, g, tl);
    const bool ok_sigma = sigma > 0.0 && isfinite(sigma);
    int wmax = 0, nact = 0;
    for (int wi = 0; wi < W.n; ++wi)
        if (W.w[wi] < nb) { wmax = max(wmax, W.w[wi]); ++nact; }
    const bool fast = g <= kRowsPerWave && sh.nz[tl] > wmax;
    uint32_t* bestu = reinterpret_cast<uint32_t*>(sh.bestv);
    for (int i = threadIdx.x; i < kFusedWidths * 64; i += kThreads) bestu[i] = 0u;
    __syncthreads();
    if (ok_sigma) {
        // runs of E consecutive boxes in width-major order over the widths < nb
        const int log2nb = 31 - __builtin_clz(nb);
        const int total = nact << log2nb;
        const int E = (total + kWaves - 1) / kWaves;
        int idx = wave * E;
        const int hi = min(total, idx + E);
        while (idx < hi) {
            const int ai = idx >> log2nb, s0 = idx & (nb - 1);
            const int s1 = min(nb, s0 + (hi - idx));
            int wi = -1;   // the ai-th width below nb
            for (int j = 0, c = 0; j < W.n; ++j)
                if (W.w[j] < nb) { if (c == ai) wi = j; ++c; }
            const int w = W.w[wi];
            float b;
            if (g == 1)
                b = fast ? scan_range<false, true>(tab, w, s0, s1, nb, g, tl, nf, Sf, tot)
                         : scan_range<true, true>(tab, w, s0, s1, nb, g, tl, nf, Sf, tot);
            else
                b = fast ? scan_range<false, false>(tab, w, s0, s1, nb, g, tl, nf, Sf, tot)
                         : scan_range<true, false>(tab, w, s0, s1, nb, g, tl, nf, Sf, tot);
            if (b > 0.0f) atomicMax(&bestu[wi * 64 + lane], __float_as_uint(b));
            idx += s1 - s0;
        }
    }
    __syncthreads();
    float best = 0.0f;
    int bwi = -1;
    for (int wi = 0; wi < W.n; ++wi) {
        const float v = sh.bestv[wi * 64 + lane];
        if (v > best) { best = v; bwi = wi; }
    }
    // first start of the winning width with the maximum value: the boxes of
    // this wave's starts are evaluated with the scan's expressions (same
    // bits), their slots loaded together
    int first = 0x7fffffff;
    if (bwi >= 0) {
        const int w = W.w[bwi];
        const int per = (nb + kWaves - 1) / kWaves;   // <= 16
        const int sb = wave * per;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int st = sb + j;
            if (j < per && st < nb) {
                const Slot a = st ? slot_at(tab, st * g - 1, tl) : Slot{0.0f, 0.0f};
                const bool wrap = st + w > nb;
                const Slot e = slot_at(tab, (wrap ? st + w - nb : st + w) * g - 1, tl);
                const float ec = wrap ? e.c + tot.c : e.c;
                const float ed = wrap ? e.dn + tot.dn : e.dn;
                const float v = fast ? box_value<false>(ec - a.c, ed - a.dn, nf, Sf)
                                     : box_value<true>(ec - a.c, ed - a.dn, nf, Sf);
                if (v == best) first = min(first, st);
            }
        }
    }
    sh.first[wave * 64 + lane] = first;
    __syncthreads();
    if (wave != 0 || kk >= k || (kTwo && lane >= 32)) return;
    int s = 0x7fffffff;
    for (int wv = 0; wv < kWaves; ++wv) s = min(s, sh.first[wv * 64 + lane]);
    float o_snr = 0.0f, o_depth = 0.0f;
    int32_t o_s = -1, o_w = -1;
    if (bwi >= 0 && valid && s < nb) {
        const int w = W.w[bwi];
        const Slot a = coarse_prefix(tab, s, g, tl);
        double ec, edn;
        if (s + w <= nb) {
            const Slot e = coarse_prefix(tab, s + w, g, tl);
            ec = e.c;
            edn = e.dn;
        } else {
            const Slot e = coarse_prefix(tab, s + w - nb, g, tl);
            ec = (double)e.c + (double)tot.c;
            edn = (double)e.dn + (double)tot.dn;
        }
        const double n = (double)nf;
        const double nin = ec - (double)a.c;
        const double din = (edn - (double)a.dn) / n;
        const double nout = n - nin;
        const double S = sh.Srow[tl];
        const double dep = (S - din) / nout - din / nin;
        o_snr = (float)(dep * sqrt(nin * nout / n) / sigma);
        o_depth = (float)dep;
        o_s = s;
        o_w = w;
    }
    snr[kk] = o_snr;
    depth[kk] = o_depth;
    start[kk] = o_s;
    width[kk] = o_w;
}

// Round to nearest even bfloat16 (v_cvt_pk_bf16_f32: the same bits as
// rounding the bit pattern, for every finite value).
__device__ __forceinline__ uint16_t bf16_rne(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

// Everything after the fold: the block's packed histogram (64 periods x 256
// fine bins; kTwo: 32 periods, high words in half 0 and low words in half 1)
// becomes the fused score, and optionally the normalised folds. Outputs are
// indexed by the curve's period index kk. zfold (optional, nb >= 16): the
// folded curve of each period as bfloat16 z-scores over its non-empty bins
// (bin means minus their mean, over their std with ddof 0; empty bins and zero
// spread give 0) - the input the learned scorer takes.
template <bool kTwo>
__device__ void score_body(char* hist, uint64_t* chunk, ScoreShared& sh,
                           const CurveInfo* __restrict__ info, const LaneSetup& L, int64_t kk,
                           int64_t k, int32_t log2g, const Widths& W, float* snr, int32_t* start,
                           int32_t* width, float* depth, uint16_t* zfold) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool act = !kTwo || lane < 32;   // the lane converts and writes its period

    // Inclusive prefix over the wave's 16 fine rows (packed values add exactly).
    const int r0 = wave * kRowsPerWave;
    uint64_t acc = 0;
    for (int r = r0; r < r0 + kRowsPerWave; ++r) {
        uint64_t* p = reinterpret_cast<uint64_t*>(hist + hist_off(r, lane));
        acc += *p;
        *p = acc;
    }
    chunk[wave * 64 + lane] = acc;
    __syncthreads();
    uint64_t off = 0, all = 0, offl = 0, alll = 0;
    for (int w = 0; w < kWaves; ++w) {
        const uint64_t v = chunk[w * 64 + lane];
        off += w < wave ? v : 0;
        all += v;
        if (kTwo) {   // the partner lane's low words
            const uint64_t vl = chunk[w * 64 + (lane ^ 32)];
            offl += w < wave ? vl : 0;
            alll += vl;
        }
    }
    __syncthreads();   // chunk is reused below
    const double qs = info->qscale;
    const double qlo = kTwo ? ldexp(1.0, info->e_lo) : 0.0;
    auto dec = [&](uint64_t vh, uint64_t vl, uint32_t& c, double& d) {
        if (kTwo) decode2(vh, vl, qs, qlo, c, d);
        else decode(vh, qs, c, d);
    };
    uint32_t call;
    double dall;
    dec(all, alll, call, dall);
    const float nf = (L.valid && act) ? (float)call : 0.0f;
    // Convert to the float prefix table, count non-empty coarse bins and (for
    // the normalised folds) sum the bin means (coarse bins of g <= 16 rows
    // never straddle two waves). kTwo: lanes 0-31 read their partner's low
    // words (half 1, which nothing writes here) and write half 0.
    const int g = 1 << log2g;
    uint32_t cprev;
    double dprev;
    dec(off, offl, cprev, dprev);
    int nzl = 0;
    float zs = 0.0f, zq = 0.0f;
    if (act) {
        for (int r = r0; r < r0 + kRowsPerWave; ++r) {
            char* p = hist + hist_off(r, lane);
            const uint64_t v = *reinterpret_cast<uint64_t*>(p) + off;
            const uint64_t vl =
                kTwo ? *reinterpret_cast<const uint64_t*>(hist + hist_off(r, lane + 32)) + offl : 0;
            uint32_t c;
            double d;
            dec(v, vl, c, d);
            if (((r + 1) & (g - 1)) == 0) {
                if (c > cprev) {
                    ++nzl;
                    if (zfold) {   // bin-mean moments, for the normalised folds only
                        const float m = (float)((d - dprev) / (double)(c - cprev));
                        zs += m;
                        zq += m * m;
                    }
                }
                cprev = c;
                dprev = d;
            }
            Slot sl{(float)c, (float)((double)nf * d)};
            if (!L.valid) sl = Slot{0.0f, 0.0f};
            *reinterpret_cast<Slot*>(p) = sl;
        }
    }
    sh.nzc[wave * 64 + lane] = nzl;
    float2* zpart = reinterpret_cast<float2*>(chunk);
    zpart[wave * 64 + lane] = make_float2(zs, zq);
    if (wave == 0) {
        sh.nrow[lane] = nf;
        sh.Srow[lane] = (L.valid && act) ? dall : 0.0;
    }
    __syncthreads();
    if (wave == 0) {
        int nz = 0;
        for (int w = 0; w < kWaves; ++w) nz += sh.nzc[w * 64 + lane];
        sh.nz[lane] = nz;
    }
    const int nb = kFineBins >> log2g;
    if (zfold && g <= kRowsPerWave && kk < k && act) {
        int nz = 0;
        float s1 = 0.0f, s2 = 0.0f;
        for (int w = 0; w < kWaves; ++w) {
            nz += sh.nzc[w * 64 + lane];
            const float2 zp = zpart[w * 64 + lane];
            s1 += zp.x;
            s2 += zp.y;
        }
        const float mu = nz ? s1 / (float)nz : 0.0f;
        const float var = nz ? fmaxf(s2 / (float)nz - mu * mu, 0.0f) : 0.0f;
        const float inv = var > 0.0f ? 1.0f / sqrtf(var) : 0.0f;
        uint16_t* zrow = zfold + kk * nb;
        const int b0 = r0 >> log2g, b1 = (r0 + kRowsPerWave) >> log2g;
        auto zval = [&](int b) {
            const Slot e = slot_at(hist, (b + 1) * g - 1, lane);
            const Slot a = b ? slot_at(hist, b * g - 1, lane) : Slot{0.0f, 0.0f};
            const float cb = e.c - a.c;
            float z = 0.0f;
            if (cb > 0.5f && L.valid) z = ((e.dn - a.dn) / (nf * cb) - mu) * inv;
            return (uint32_t)bf16_rne(z);
        };
        if (b1 - b0 == 16) {   // the wave's 16 bins of this period: two 16-byte stores
            uint32_t pk[8];
            for (int j = 0; j < 8; ++j) pk[j] = zval(b0 + 2 * j) | (zval(b0 + 2 * j + 1) << 16);
            uint4* dst = reinterpret_cast<uint4*>(zrow + b0);
            dst[0] = make_uint4(pk[0], pk[1], pk[2], pk[3]);
            dst[1] = make_uint4(pk[4], pk[5], pk[6], pk[7]);
        } else {
            for (int b = b0; b < b1; ++b) zrow[b] = (uint16_t)zval(b);
        }
    }
    __syncthreads();
    score_table<kTwo>(hist, nb, g, W, sh, info->sigma, L.valid, kk, k, lane, wave, snr, start,
                      width, depth);
}

// Fold + score of one block of 64 periods of one prepared curve (periods
// kbase .. kbase+63 of the curve's k): one pass for a one-word curve, two
// passes of 32 periods for a two-word curve.
__device__ void fold_score_body(char* hist, uint64_t* chunk, ScoreShared& sh,
                                const Rec* __restrict__ rec, const uint64_t* __restrict__ lo,
                                int64_t per, const CurveInfo* __restrict__ info,
                                const double* __restrict__ periods, int64_t k, int64_t kbase,
                                int32_t log2g, const Widths& W, float* snr, int32_t* start,
                                int32_t* width, float* depth, uint16_t* zfold) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (info->words == 2) {
        for (int half = 0; half < 2; ++half) {
            const int64_t kk = lane_period(kbase, lane, true, half);
            const LaneSetup L = lane_setup(periods, kk, k, info->tmax);
            fold_block<true>(hist, rec, lo, per, L, lane, wave);
            score_body<true>(hist, chunk, sh, info, L, kk, k, log2g, W, snr, start, width, depth,
                             zfold);
            __syncthreads();
        }
        return;
    }
    const int64_t kk = kbase + lane;
    const LaneSetup L = lane_setup(periods, kk, k, info->tmax);
    fold_block<false>(hist, rec, lo, per, L, lane, wave);
    score_body<false>(hist, chunk, sh, info, L, kk, k, log2g, W, snr, start, width, depth, zfold);
}

__global__ __launch_bounds__(kThreads, 1) void k_fold_score(
    const Rec* __restrict__ rec, const uint64_t* __restrict__ lo, int64_t per,
    const double* __restrict__ periods, int64_t k, int32_t log2g,
    const CurveInfo* __restrict__ info, Widths W, float* __restrict__ snr,
    int32_t* __restrict__ start, int32_t* __restrict__ width, float* __restrict__ depth,
    uint16_t* __restrict__ zfold) {
    __shared__ __attribute__((aligned(16))) char hist[kFineBins * 64 * 8];
    __shared__ uint64_t chunk[kWaves * 64];
    __shared__ ScoreShared sh;
    fold_score_body(hist, chunk, sh, rec, lo, per, info, periods, k, (int64_t)blockIdx.x * 64,
                    log2g, W, snr, start, width, depth, zfold);
}

// Fold + score with the samples split over gridDim.y blocks per 64-period
// tile, for grids too small to fill the chip: block (tile, s) folds part s of
// every wave slice into its LDS histogram and adds it into the tile's global
// histogram with 64-bit integer atomics (exact, any order). The block that
// arrives last (a device counter per tile, after a release fence) takes the
// merged histogram back into LDS, clearing the global copy and the counter
// for the next launch, and scores it like k_fold_score. No block waits on
// another. A two-word curve runs this twice per block, once per 32-period
// half of the tile, each half with its own global histogram and counter.
template <bool kTwo>
__device__ void split_pass(char* hist, uint64_t* chunk, ScoreShared& sh, int32_t* is_last,
                           uint32_t* ctr, const Rec* __restrict__ rec,
                           const uint64_t* __restrict__ lo, int64_t per, int64_t per_s,
                           const double* __restrict__ periods, int64_t k, int32_t log2g,
                           const CurveInfo* __restrict__ info, const Widths& W, float* snr,
                           int32_t* start, int32_t* width, float* depth, uint16_t* zfold,
                           unsigned long long* gh, int32_t* arrivals, int half) {
    const int lane = threadIdx.x & 63;
    const int tile = blockIdx.x;
    const int64_t kk = lane_period((int64_t)tile * 64, lane, kTwo, half);
    const LaneSetup L = lane_setup(periods, kk, k, info->tmax);
    uint64_t* h64 = reinterpret_cast<uint64_t*>(hist);
    for (int i = threadIdx.x; i < kFineBins * 64; i += kThreads) h64[i] = 0;
    if (threadIdx.x == 0) *ctr = 0u;
    __syncthreads();
    // part y of the records: [b0, b0 + len) of each of the kWaves segments
    const int64_t b0 = (int64_t)blockIdx.y * per_s;
    const int64_t len = b0 < per ? min(per_s, per - b0) : 0;   // a multiple of 2 kBlk
    const uint32_t laneoff = (uint32_t)((lane & 31) * 8 + (lane >> 5) * kHalfBytes);
    const int64_t cps = len / (2 * kBlk);
    if (cps > 0)
        fold_chunks<false, kTwo>(hist, ctr, rec + b0, lo + b0, cps * kWaves, cps, per, L, laneoff,
                                 lane);
    __syncthreads();
    const int slot = 2 * tile + half;
    unsigned long long* g = gh + (int64_t)slot * (kFineBins * 64);
    for (int i = threadIdx.x; i < kFineBins * 64; i += kThreads) {
        const uint64_t v = h64[i];
        if (v) atomicAdd(g + i, (unsigned long long)v);
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) *is_last = atomicAdd(arrivals + slot, 1) == (int)gridDim.y - 1;
    __syncthreads();
    if (!*is_last) return;
    __threadfence();
    for (int i = threadIdx.x; i < kFineBins * 64; i += kThreads) h64[i] = atomicExch(g + i, 0ull);
    if (threadIdx.x == 0) atomicExch(arrivals + slot, 0);
    __syncthreads();
    score_body<kTwo>(hist, chunk, sh, info, L, kk, k, log2g, W, snr, start, width, depth, zfold);
}

__global__ __launch_bounds__(kThreads, 1) void k_fold_score_split(
    const Rec* __restrict__ rec, const uint64_t* __restrict__ lo, int64_t per, int64_t per_s,
    const double* __restrict__ periods, int64_t k, int32_t log2g,
    const CurveInfo* __restrict__ info, Widths W, float* __restrict__ snr,
    int32_t* __restrict__ start, int32_t* __restrict__ width, float* __restrict__ depth,
    uint16_t* __restrict__ zfold, unsigned long long* __restrict__ gh, int32_t* __restrict__ arrivals) {
    __shared__ __attribute__((aligned(16))) char hist[kFineBins * 64 * 8];
    __shared__ uint64_t chunk[kWaves * 64];
    __shared__ ScoreShared sh;
    __shared__ int32_t is_last;
    __shared__ uint32_t ctr;
    if (info->words == 2) {
        for (int half = 0; half < 2; ++half) {
            split_pass<true>(hist, chunk, sh, &is_last, &ctr, rec, lo, per, per_s, periods, k, log2g,
                             info, W, snr, start, width, depth, zfold, gh, arrivals, half);
            __syncthreads();
        }
        return;
    }
    split_pass<false>(hist, chunk, sh, &is_last, &ctr, rec, lo, per, per_s, periods, k, log2g, info,
                      W, snr, start, width, depth, zfold, gh, arrivals, 0);
}

// Persistent multi-curve fold + score: one block per CU pulls work items
// (curve, block of 64 of its periods) from a device counter until none are
// left; items are ordered longest curve first. Every block reaches the exit
// test on each round, so the grid drains.
__global__ __launch_bounds__(kThreads, 1) void k_batch_fold_score(
    const Rec* __restrict__ rec, const uint64_t* __restrict__ lo,
    const BatchCurve* __restrict__ curves,
    const int2* __restrict__ items, int32_t n_items, int32_t* __restrict__ counter,
    const CurveInfo* __restrict__ infos, const double* __restrict__ periods, int32_t log2g,
    Widths W, float* __restrict__ snr, int32_t* __restrict__ start, int32_t* __restrict__ width,
    float* __restrict__ depth, uint16_t* __restrict__ zfold) {
    __shared__ __attribute__((aligned(16))) char hist[kFineBins * 64 * 8];
    __shared__ uint64_t chunk[kWaves * 64];
    __shared__ ScoreShared sh;
    __shared__ int32_t cur_item;
    const int nb = kFineBins >> log2g;
    for (;;) {
        if (threadIdx.x == 0) cur_item = atomicAdd(counter, 1);
        __syncthreads();
        const int32_t it = cur_item;
        __syncthreads();
        if (it >= n_items) break;
        const int2 item = items[it];
        const BatchCurve bc = curves[item.x];
        fold_score_body(hist, chunk, sh, rec + bc.rec_off, lo + bc.rec_off, bc.per, infos + item.x,
                        periods + bc.p_off, bc.k, (int64_t)item.y * 64, log2g, W, snr + bc.o_off,
                        start + bc.o_off, width + bc.o_off, depth + bc.o_off,
                        zfold ? zfold + bc.z_off * nb : nullptr);
        __syncthreads();
    }
}

__global__ void k_set_i32(int32_t* __restrict__ p, int32_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// Box-SNR of materialised folds: lane j owns row blockIdx*64 + j; the waves
// split the bins. Deviations are taken from each row's own mean (the SNR does
// not depend on the reference).
__global__ __launch_bounds__(kThreads, 1) void k_score(const double* __restrict__ sums,
                                                       const int32_t* __restrict__ counts,
                                                       int64_t k, int32_t nb, double sigma,
                                                       Widths W, float* __restrict__ snr,
                                                       int32_t* __restrict__ start,
                                                       int32_t* __restrict__ width,
                                                       float* __restrict__ depth) {
    __shared__ __attribute__((aligned(16))) char tab[kFineBins * 64 * 8];
    __shared__ double csum[kWaves * 64];
    __shared__ double ccnt[kWaves * 64];
    __shared__ ScoreShared sh;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t kk = (int64_t)blockIdx.x * 64 + lane;
    const bool valid = kk < k;
    const int per = (nb + kWaves - 1) / kWaves;
    const int b0 = min(nb, wave * per), b1 = min(nb, b0 + per);
    double s = 0.0, c = 0.0;
    if (valid)
        for (int b = b0; b < b1; ++b) { s += sums[kk * nb + b]; c += (double)counts[kk * nb + b]; }
    csum[wave * 64 + lane] = s;
    ccnt[wave * 64 + lane] = c;
    __syncthreads();
    double ts = 0.0, tc = 0.0;
    for (int w = 0; w < kWaves; ++w) { ts += csum[w * 64 + lane]; tc += ccnt[w * 64 + lane]; }
    const double ref = tc > 0.0 ? ts / tc : 0.0;
    double dacc = 0.0, cacc = 0.0;
    int nzl = 0;
    for (int b = b0; b < b1; ++b) {
        const double cb = valid ? (double)counts[kk * nb + b] : 0.0;
        const double sb = valid ? sums[kk * nb + b] : 0.0;
        dacc += sb - cb * ref;
        cacc += cb;
        nzl += cb > 0.0;
    }
    __syncthreads();
    csum[wave * 64 + lane] = dacc;
    ccnt[wave * 64 + lane] = cacc;
    sh.nzc[wave * 64 + lane] = nzl;
    __syncthreads();
    double doff = 0.0, coff = 0.0, dall = 0.0, call = 0.0;
    int nz = 0;
    for (int w = 0; w < kWaves; ++w) {
        const double dv = csum[w * 64 + lane], cv = ccnt[w * 64 + lane];
        if (w < wave) { doff += dv; coff += cv; }
        dall += dv;
        call += cv;
        nz += sh.nzc[w * 64 + lane];
    }
    for (int b = b0; b < b1; ++b) {
        const double cb = valid ? (double)counts[kk * nb + b] : 0.0;
        const double sb = valid ? sums[kk * nb + b] : 0.0;
        doff += sb - cb * ref;
        coff += cb;
        *reinterpret_cast<Slot*>(tab + hist_off(b, lane)) = Slot{(float)coff, (float)(call * doff)};
    }
    if (wave == 0) {
        sh.nrow[lane] = (float)call;
        sh.Srow[lane] = dall;
        sh.nz[lane] = nz;
    }
    __syncthreads();
    score_table<false>(tab, nb, 1, W, sh, sigma, valid, kk, k, lane, wave, snr, start, width, depth);
}

// ------------------------------------------------------------------ plain fold (baseline)

template <typename T>
__global__ __launch_bounds__(256) void k_zero(T* __restrict__ p, int64_t m) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256)
        p[i] = T(0);
}

// One block per period, one thread per sample: IEEE division, then one
// device-memory atomic for the count and one FP64 atomic for the sum.
__global__ __launch_bounds__(256) void k_fold_naive(const double* __restrict__ t,
                                                    const float* __restrict__ flux, int64_t n,
                                                    const double* __restrict__ periods,
                                                    int32_t nbins, double* __restrict__ sums,
                                                    int32_t* __restrict__ counts) {
    const int64_t kk = blockIdx.x;
    const double P = periods[kk];
    if (!(P > 0.0) || !isfinite(P)) return;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double x = t[i] / P;
        const double f = x - floor(x);
        const double fb = floor(f * (double)nbins);
        int b = !(fb >= 0.0) ? 0 : (fb >= (double)nbins ? nbins - 1 : (int)fb);
        atomicAdd(&counts[kk * nbins + b], 1);
        unsafeAtomicAdd(&sums[kk * nbins + b], (double)flux[i]);
    }
}

}  // namespace

// ------------------------------------------------------------------ equal-count fold
//
// The paper's two-tier fold (Sec. 2.3 steps 1-5, Fig. 4): 4096 equal-width
// intermediate bins, then final bins holding N / nbins points each, a bin on
// a boundary split in proportion. One block of 16 waves folds 4 periods: 4
// waves per period, lanes take consecutive records (coalesced 16-byte loads),
// each update one 64-bit integer LDS atomic into the period's 4096-bin packed
// histogram (count and fixed-point flux sum, exact). The bin comes from the
// certified fast path at 4096 bins (fraction field 16 bits below the bin);
// a lane whose fraction it cannot certify takes the IEEE sequence instead.
// Then one wave per period scans the histogram: in units of 1/nbins point
// (a sample is nbins units, a final bin N units) every boundary j*N falls in
// one intermediate bin, whose lane records the cumulative deviation sum there
// as an exact integer part (the bins before it) plus the interpolated share of
// that bin; a final bin's sum is the difference of its two boundaries.
constexpr int kMid = 4096;
typedef uint32_t u32x4b __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2b __attribute__((ext_vector_type(2)));
constexpr int kEqPeriods = 4;
constexpr int kEqMaxBins = 256;

struct EqBoundary {
    int64_t ipart;    // cumulative fixed-point deviation of the bins before (high words)
    int64_t ilo;      // the same for the low words of a two-word curve (0 otherwise)
    double frac;      // share of the boundary's own bin, in units of the high word
};

__device__ __forceinline__ uint32_t mid_bin_ieee(double t, double P) {
    const double x = t / P;
    const double f = x - floor(x);
    const double fb = floor(f * (double)kMid);
    if (!(fb >= 0.0)) return 0u;
    if (fb >= (double)kMid) return kMid - 1;
    return (uint32_t)fb;
}

// One pass of the equal-count fold over `np` of the block's periods
// (np = 4, one word; np = 2, two words: region 2 + p of the LDS histogram
// holds period p's low words). The four regions are interleaved by bin
// (slot 4 b + region) and each lane adds its record to the four regions in
// rotation, so one 16-lane pass of a 64-bit atomic carries 4 records x 4
// regions, and only records of one region whose bins agree mod 4 meet on a
// bank group (with one region per pass, 16 records would share 4 groups).
template <bool kTwo>
__device__ __forceinline__ void eqcount_pass(uint64_t* hist, EqBoundary (*bnd)[kEqMaxBins + 1], int64_t* eqn, int* dsel,
                             int64_t (*wtot)[3],
                             const Rec* __restrict__ rec, const uint64_t* __restrict__ lo,
                             int64_t nrec, const double* __restrict__ periods, int64_t k,
                             int64_t kbase, int32_t nbins, const CurveInfo* __restrict__ info,
                             double* __restrict__ means, uint16_t* __restrict__ zfold) {
    constexpr int np = kTwo ? kEqPeriods / 2 : kEqPeriods;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < kEqPeriods * kMid; i += kThreads) hist[i] = 0;
    // Each lane loads one record and adds it to all four regions, region
    // (lane + j) mod 4 at its j-th update, so a 16-lane pass always holds 4
    // records x the 4 regions and one record load serves 4 updates.
    double rBj[4];
    uint32_t limj[4], roffj[4];
    bool vj[4];
    bool allv = true;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int g = (lane + j) & 3;                  // the region
        const int64_t kk = kbase + (kTwo ? (g & 1) : g);
        double P = kk < k ? periods[kk] : 1.0;
        vj[j] = kk < k && P > 0.0 && isfinite(P);
        allv = allv && vj[j];
        if (!vj[j]) P = 1.0;
        rBj[j] = (1.0 / P) * (double)kMid;
        limj[j] = info->tmax * rBj[j] < 0x1p34 ? 65536u - 2u : 0u;
        roffj[j] = (uint32_t)g * (uint32_t)sizeof(uint64_t);
    }
    // Two lanes of a 16-lane pass of a 64-bit LDS atomic conflict when their
    // slots agree mod 16: with slot 4 b + region, when two records of one
    // region have bins that agree mod 4. A region's 4 records in a pass are a
    // comb spaced a apart (a = 2^e <= 16; a wave's 64 records split into
    // windows of 4a, each into a combs), with a chosen so that a times the bin
    // advance per record is near 1 or 3 mod 4 for the block's periods: the
    // comb's bins mod 4 are then x, x + D, x + 2 D, x + 3 D with D about 1 or 3,
    // all distinct. Any a gives the same sums. (worked out once per block by
    // its first thread)
    if (threadIdx.x == 0) {
        int e = 0;
        if (nrec > 1) {
            double dt = rec[1].t - rec[0].t;                 // the cadence: the least of a few spacings
            for (int64_t i = 2; i < 9 && i < nrec; ++i) dt = fmin(dt, rec[i].t - rec[i - 1].t);
            double best = 1e30;
            for (int ee = 0; ee <= 4; ++ee) {
                double miss = 0.0;
                for (int j = 0; j < 4; ++j) {
                    const double dl = (double)(1 << ee) * dt * rBj[j];   // bins per comb step
                    const double del = dl - 4.0 * floor(dl * 0.25);
                    miss += fmin(fabs(del - 1.0), fabs(del - 3.0));
                }
                if (miss < best) { best = miss; e = ee; }
            }
        }
        dsel[0] = e;
    }
    __syncthreads();
    const int e = dsel[0];
    const int cm = ((lane >> 4) << 2) | (lane & 3), kq = (lane >> 2) & 3;   // comb, place in it
    const int lrec = wave * 64 + ((cm >> e) << (e + 2)) + (cm & ((1 << e) - 1)) + (kq << e);
    // kEqU records per lane per step; the next step's records are requested
    // before this step's updates, so their latency overlaps them (more records
    // per step measured slower). Steps wholly inside the curve take no
    // bounds checks; the last partial step re-reads the curve's last record
    // for indices past it and adds 0 there. Every update goes to its fast-path
    // bin; when some lane's fraction falls outside the certificate (rare) the
    // step is repaired: each such update is taken back from the fast bin and
    // added to the IEEE bin. Regions of invalid periods (only in a block past
    // the grid's end or for a bad period) add 0.
    constexpr int kEqU = 1;
    auto repair = [&](int64_t i0) {
#pragma unroll 1
        for (int q = 0; q < kEqU * 4; ++q) {
            const int64_t i = i0 + 1024 * (q >> 2) + lrec;
            const int g = (lane + q) & 3;
            const int64_t kk = kbase + (kTwo ? (g & 1) : g);
            const double P = kk < k ? periods[kk] : 1.0;
            if (i >= nrec || !(kk < k && P > 0.0 && isfinite(P))) continue;
            const double rB = (1.0 / P) * (double)kMid;
            const uint32_t lim = info->tmax * rB < 0x1p34 ? 65536u - 2u : 0u;
            const double ti = rec[i].t;
            const uint32_t lw = fast_lo(ti, rB);
            if ((lw & 0xFFFFu) < lim) continue;
            const uint64_t v = (kTwo && g >= 2) ? lo[i] : rec[i].c;
            uint64_t* h = (uint64_t*)((char*)hist + (g * (int)sizeof(uint64_t)));
            __hip_atomic_fetch_add(h + ((lw >> 16) & (kMid - 1)) * kEqPeriods, uint64_t(0) - v,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_add(h + mid_bin_ieee(ti, P) * kEqPeriods, v, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    };
    auto updates = [&](auto kAll, int64_t i0, const double* tv, const uint64_t* cv, const uint64_t* lv) {
        uint64_t bad = 0;   // lanes (any update) outside the certificate
#pragma unroll
        for (int u = 0; u < kEqU; ++u)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t lw = fast_lo(tv[u], rBj[j]);   // the certified path, at 4096 bins
                bad |= __builtin_amdgcn_ballot_w64((lw & 0xFFFFu) >= limj[j]);
                uint64_t v = cv[u];
                if (kTwo && (((lane + j) & 3) >= 2)) v = lv[u];
                if (!decltype(kAll)::value && !vj[j]) v = 0;
                __hip_atomic_fetch_add((uint64_t*)((char*)hist + ((((lw >> 16) & (kMid - 1)) << 5) | roffj[j])), v,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        if (bad) repair(i0);
    };
    auto run = [&](auto kAll) {
        int64_t i0 = 0;
        if (nrec < (int64_t)1 << 27) {
            // buffer loads: the lane's byte offset in a VGPR, the step's in an
            // SGPR, so no vector address arithmetic per load (byte offsets stay
            // below 2^31 for fewer than 2^27 records)
            const __amdgpu_buffer_rsrc_t rr = __builtin_amdgcn_make_buffer_rsrc(
                (void*)rec, (short)0, (int)(nrec * (int64_t)sizeof(Rec)), 0x00020000);
            const __amdgpu_buffer_rsrc_t rl =
                __builtin_amdgcn_make_buffer_rsrc((void*)lo, (short)0, lo ? (int)(nrec * 8) : 0, 0x00020000);
            const int boff = lrec * (int)sizeof(Rec), loff = lrec * 8;
            // each step's records are requested before the previous step's updates
            const int64_t nfull = nrec / (1024 * kEqU);   // whole steps
            auto load = [&](int64_t s0, double* tv, uint64_t* cv, uint64_t* lv) {
#pragma unroll
                for (int u = 0; u < kEqU; ++u) {
                    const int so = (int)(s0 + 1024 * u);
                    const u32x4b r = __builtin_amdgcn_raw_buffer_load_b128(rr, boff, so * (int)sizeof(Rec), 0);
                    tv[u] = __builtin_bit_cast(double, (uint64_t)r[0] | (uint64_t)r[1] << 32);
                    cv[u] = (uint64_t)r[2] | (uint64_t)r[3] << 32;
                    lv[u] = 0;
                    if (kTwo) {
                        const u32x2b l = __builtin_amdgcn_raw_buffer_load_b64(rl, loff, so * 8, 0);
                        lv[u] = (uint64_t)l[0] | (uint64_t)l[1] << 32;
                    }
                }
            };
            if (nfull > 0) {
                double tv[kEqU], tn[kEqU];
                uint64_t cv[kEqU], lv[kEqU], cn[kEqU], ln[kEqU];
                load(0, tv, cv, lv);
                for (int64_t st = 0; st < nfull; ++st) {
                    const int64_t nx = st + 1 < nfull ? st + 1 : st;   // the last step re-reads itself
                    load(nx * 1024 * kEqU, tn, cn, ln);
                    __builtin_amdgcn_sched_barrier(0);
                    updates(kAll, st * 1024 * kEqU, tv, cv, lv);
#pragma unroll
                    for (int u = 0; u < kEqU; ++u) {
                        tv[u] = tn[u];
                        cv[u] = cn[u];
                        lv[u] = ln[u];
                    }
                }
                i0 = nfull * 1024 * kEqU;
            }
        } else {
            for (; i0 + 1024 * kEqU <= nrec; i0 += 1024 * kEqU) {
                double tv[kEqU];
                uint64_t cv[kEqU], lv[kEqU];
#pragma unroll
                for (int u = 0; u < kEqU; ++u) {
                    const Rec r = rec[i0 + 1024 * u + lrec];
                    tv[u] = r.t;
                    cv[u] = r.c;
                    lv[u] = kTwo ? lo[i0 + 1024 * u + lrec] : 0;
                }
                __builtin_amdgcn_sched_barrier(0);
                updates(kAll, i0, tv, cv, lv);
            }
        }
        if (i0 < nrec) {
            double tv[kEqU];
            uint64_t cv[kEqU], lv[kEqU];
#pragma unroll
            for (int u = 0; u < kEqU; ++u) {
                const int64_t i = i0 + 1024 * u + lrec;
                const int64_t ic = i < nrec ? i : nrec - 1;
                const Rec r = rec[ic];
                tv[u] = r.t;
                cv[u] = i < nrec ? r.c : 0;
                lv[u] = kTwo && i < nrec ? lo[ic] : 0;
            }
            updates(kAll, i0, tv, cv, lv);
        }
    };
    if (allv)
        run(std::integral_constant<bool, true>());
    else
        run(std::integral_constant<bool, false>());
    __syncthreads();
    // The boundary scan, on all 16 waves: wave w takes period w mod np and
    // part w / np of W = 16 / np equal parts of its bins, each lane a run of
    // about BL bins in bin order, read once into registers. Runs start at
    // BL lane + (lane mod 4) within the part, so a 16-lane pass reads bins of
    // 4 residues mod 4 (a region's slots fall in 4 of the 16 bank groups of a
    // 64-bit access: 4 lanes per group is the fewest possible, where runs
    // starting at BL lane would put all 16 in one).
    {
        constexpr int W = kThreads / 64 / np;        // waves per period
        constexpr int BW = kMid / W;                  // bins per wave
        constexpr int BL = BW / 64;                   // bins per lane, about
        const int p2 = wave % np, part = wave / np;
        const int64_t k2 = kbase + p2;
        const double P2 = k2 < k ? periods[k2] : 1.0;
        const bool v2 = k2 < k && P2 > 0.0 && isfinite(P2);
        const uint64_t* hh = hist + p2;
        const uint64_t* hl = hist + p2 + 2;           // low words (kTwo)
        const int blo = part * BW + lane * BL + (lane & 3);
        const int bhi = part * BW + (lane == 63 ? BW : (lane + 1) * BL + ((lane + 1) & 3));
        auto bin_at = [&](int b, int64_t& c, int64_t& d, int64_t& dl) {
            const uint64_t v = hh[b * kEqPeriods];
            c = (int64_t)(v >> kCountShift);
            d = (int64_t)(v & kSumMask) - c * kBias;
            dl = kTwo ? (int64_t)(hl[b * kEqPeriods] & kSumMask) - c * kBias : 0;
        };
        // the lane's totals: the run is BL - 3 to BL + 1 bins, all read at once
        // (slots past the run re-read its last bin and add nothing)
        int64_t lc = 0, ls = 0, ll = 0;
        {
            uint64_t hv[BL + 1], hlv[BL + 1];
#pragma unroll
            for (int i = 0; i < BL + 1; ++i) {
                const int b = blo + i < bhi ? blo + i : bhi - 1;
                hv[i] = hh[b * kEqPeriods];
                hlv[i] = kTwo ? hl[b * kEqPeriods] : 0;
            }
#pragma unroll
            for (int i = 0; i < BL + 1; ++i)
                if (blo + i < bhi) {
                    const int64_t c = (int64_t)(hv[i] >> kCountShift);
                    lc += c;
                    ls += (int64_t)(hv[i] & kSumMask) - c * kBias;
                    if (kTwo) ll += (int64_t)(hlv[i] & kSumMask) - c * kBias;
                }
        }
        int64_t pc = lc, ps = ls, pl = ll;   // inclusive prefix over lanes
        for (int d = 1; d < 64; d <<= 1) {
            const int64_t oc = __shfl_up(pc, d), os = __shfl_up(ps, d);
            const int64_t ol = kTwo ? __shfl_up(pl, d) : 0;
            if (lane >= d) { pc += oc; ps += os; pl += ol; }
        }
        if (lane == 63) {
            wtot[wave][0] = pc;
            wtot[wave][1] = ps;
            wtot[wave][2] = pl;
        }
        __syncthreads();
        // the period's totals and those of its parts before this one
        int64_t N = 0, Stot = 0, Ltot = 0, C = pc - lc, S = ps - ls, SL = pl - ll;
        for (int q = 0; q < W; ++q) {
            const int64_t* t3 = wtot[q * np + p2];
            if (q < part) { C += t3[0]; S += t3[1]; SL += t3[2]; }
            N += t3[0];
            Stot += t3[1];
            Ltot += t3[2];
        }
        if (v2 && N > 0) {
            // the next boundary j N at or after the lane's first unit (one division
            // per lane; later boundaries follow by steps of N)
            int64_t j = (C * nbins + N - 1) / N;
            int64_t jN = j * N;
            // bins in order, each read one bin ahead of its use
            int64_t c, d, dl;
            bin_at(blo, c, d, dl);
            for (int b = blo; b < bhi; ++b) {
                int64_t cn, dn, dln;
                bin_at(b + 1 < bhi ? b + 1 : b, cn, dn, dln);
                if (c != 0) {
                    const int64_t u0 = C * nbins, u1 = (C + c) * nbins;   // the bin's units
                    // interior boundaries j N (0 < j < nbins) inside [u0, u1)
                    if (jN < u1) {
                        // the bin's deviation in units of the high word
                        const double dd = kTwo ? (double)d + ldexp((double)dl, -kLoBits) : (double)d;
                        for (; jN < u1; ++j, jN += N) {
                            if (j == 0) continue;
                            bnd[p2][j].ipart = S;
                            bnd[p2][j].ilo = SL;
                            bnd[p2][j].frac = (double)(jN - u0) / (double)(c * nbins) * dd;
                        }
                    }
                    C += c;
                    S += d;
                    SL += dl;
                }
                c = cn;
                d = dn;
                dl = dln;
            }
            if (part == 0 && lane == 0) {
                bnd[p2][0] = EqBoundary{0, 0, 0.0};
                bnd[p2][nbins] = EqBoundary{Stot, Ltot, 0.0};
            }
        }
        if (part == 0 && lane == 0) eqn[p2] = (v2 && k2 < k) ? N : -1;
    }
    __syncthreads();
    if (wave < np) {
        const int p2 = wave;
        const int64_t k2 = kbase + p2;
        const int64_t N = eqn[p2];           // -1: invalid period
        if (k2 < k) {
            const double qs = info->qscale, ref = info->ref;
            const bool any = N > 0;
            float zs = 0.0f, zq = 0.0f;
            float mloc[kEqMaxBins / 64];
            int nl = 0;
            for (int j = lane; j < nbins; j += 64, ++nl) {
                double m = __builtin_nan("");
                mloc[nl] = 0.0f;
                if (any) {
                    const EqBoundary a = bnd[p2][j], e = bnd[p2][j + 1];
                    double dsum = (double)(e.ipart - a.ipart);
                    if (kTwo) dsum += ldexp((double)(e.ilo - a.ilo), -kLoBits);
                    dsum += e.frac - a.frac;
                    const double dm = qs * dsum * (double)nbins / (double)N;
                    m = ref + dm;
                    mloc[nl] = (float)dm;
                    zs += mloc[nl];
                    zq += mloc[nl] * mloc[nl];
                }
                if (means) means[k2 * nbins + j] = m;
            }
            if (zfold) {
                for (int d = 32; d > 0; d >>= 1) {
                    zs += __shfl_xor(zs, d);
                    zq += __shfl_xor(zq, d);
                }
                const float mu = any ? zs / (float)nbins : 0.0f;
                const float var = any ? fmaxf(zq / (float)nbins - mu * mu, 0.0f) : 0.0f;
                const float inv = var > 0.0f ? 1.0f / sqrtf(var) : 0.0f;
                nl = 0;
                for (int j = lane; j < nbins; j += 64, ++nl)
                    zfold[k2 * nbins + j] = bf16_rne(any ? (mloc[nl] - mu) * inv : 0.0f);
            }
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(kThreads, 1) void k_fold_eqcount(
    const Rec* __restrict__ rec, const uint64_t* __restrict__ lo, int64_t nrec,
    const double* __restrict__ periods, int64_t k, int32_t nbins,
    const CurveInfo* __restrict__ info, double* __restrict__ means, uint16_t* __restrict__ zfold) {
    __shared__ __attribute__((aligned(16))) uint64_t hist[kEqPeriods * kMid];
    __shared__ EqBoundary bnd[kEqPeriods][kEqMaxBins + 1];
    __shared__ int64_t eqn[kEqPeriods];
    __shared__ int dsel[kEqPeriods];
    __shared__ int64_t wtot[kThreads / 64][3];
    const int64_t kbase = (int64_t)blockIdx.x * kEqPeriods;
    if (info->words == 2) {
        for (int h = 0; h < 2; ++h)
            eqcount_pass<true>(hist, bnd, eqn, dsel, wtot, rec, lo, nrec, periods, k, kbase + 2 * h, nbins, info,
                               means, zfold);
        return;
    }
    eqcount_pass<false>(hist, bnd, eqn, dsel, wtot, rec, lo, nrec, periods, k, kbase, nbins, info, means, zfold);
}

// ------------------------------------------------------------------ general path
//
// Any n and nbins up to 4096: the fold of a part of the curve (fewer than
// 2^18 samples, so the packed words cannot overflow) into an LDS histogram of
// PB = 2^LOGP periods x FB = 16384 / PB fine bins (128 KB), added into global
// integer histograms that later parts add to. Lanes: period p = lane % PB,
// record stream lane / PB (64 / PB records per wave instruction); the slot of
// (bin, p) is bin * PB + p, so a pass of 16 lanes of one record touches 16
// consecutive 8-byte slots (conflict-free for PB >= 16; with PB = 8 or 4 the
// 2 or 4 records of a pass can meet on a bank). The bin is the certified fast
// path at FB bins with a per-update IEEE fallback; coarse bins (nbins < FB,
// only for FB = 256) are unions of FB / nbins fine bins.

__device__ __forceinline__ uint32_t bin_ieee_at(double t, double P, int fb) {
    const double x = t / P;
    const double f = x - floor(x);
    const double u = floor(f * (double)fb);
    if (!(u >= 0.0)) return 0u;
    if (u >= (double)fb) return (uint32_t)fb - 1u;
    return (uint32_t)u;
}

template <int LOGP>
__global__ __launch_bounds__(kThreads, 1) void k_fold_wide(
    const Rec* __restrict__ rec, const uint64_t* __restrict__ lo, int64_t r0, int64_t r1,
    const double* __restrict__ periods, int64_t k, int32_t log2g,
    const CurveInfo* __restrict__ info, int32_t use_lo, int32_t first,
    uint32_t* __restrict__ cnt, int64_t* __restrict__ shi, int64_t* __restrict__ slo) {
    constexpr int PB = 1 << LOGP;
    constexpr int S = 64 / PB;
    constexpr int FB = 16384 / PB;
    constexpr int kU = 8;                    // records per lane per step
    __shared__ __attribute__((aligned(16))) uint64_t hist[FB * PB];
    if (use_lo && info->words != 2) return;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int p = lane & (PB - 1);
    const int sidx = lane >> LOGP;
    const int64_t kk = (int64_t)blockIdx.x * PB + p;
    double P = kk < k ? periods[kk] : 1.0;
    if (!(kk < k && P > 0.0 && isfinite(P))) P = 1.0;
    const double rB = (1.0 / P) * (double)FB;
    const uint32_t lim = info->tmax * rB < 0x1p34 ? 65536u - 2u : 0u;
    for (int i = threadIdx.x; i < FB * PB; i += kThreads) hist[i] = 0;
    __syncthreads();
    constexpr int64_t G = (int64_t)S * kU;     // records per wave step
    const int64_t ng = (r1 - r0 + G - 1) / G;
    const int64_t gpw = (ng + kWaves - 1) / kWaves;
    const int64_t g0 = wave * gpw, g1 = min(ng, g0 + gpw);
    for (int64_t g = g0; g < g1; ++g) {
        const int64_t base = r0 + g * G + sidx;
        double tv[kU];
        uint64_t cv[kU];
#pragma unroll
        for (int j = 0; j < kU; ++j) {
            const int64_t i = base + (int64_t)j * S;
            tv[j] = 0.0;
            cv[j] = 0;
            if (i < r1) {
                tv[j] = rec[i].t;
                cv[j] = use_lo ? lo[i] : rec[i].c;
            }
        }
#pragma unroll
        for (int j = 0; j < kU; ++j) {
            const uint32_t lw = fast_lo(tv[j], rB);
            uint32_t b = (lw >> 16) & (uint32_t)(FB - 1);
            if ((lw & 0xFFFFu) >= lim) b = bin_ieee_at(tv[j], P, FB);
            if (cv[j])
                __hip_atomic_fetch_add(hist + b * PB + p, cv[j], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    __syncthreads();
    const int nb = FB >> log2g;
    const int gsz = 1 << log2g;
    for (int idx = threadIdx.x; idx < PB * nb; idx += kThreads) {
        const int pp = idx / nb, b = idx - pp * nb;
        const int64_t k2 = (int64_t)blockIdx.x * PB + pp;
        if (k2 >= k) continue;
        uint64_t acc = 0;
        for (int j = 0; j < gsz; ++j) acc += hist[(b * gsz + j) * PB + pp];
        const uint32_t c = (uint32_t)(acc >> kCountShift);
        const int64_t sm = (int64_t)(acc & kSumMask) - (int64_t)c * kBias;
        const int64_t o = k2 * nb + b;
        if (use_lo) {
            slo[o] = first ? sm : slo[o] + sm;
        } else {
            cnt[o] = first ? c : cnt[o] + c;
            shi[o] = first ? sm : shi[o] + sm;
        }
    }
}

// Sums, counts and means of the general path's integer histograms (the
// formula of the fused kernels' decode, so the results match theirs bit for
// bit where both apply).
__global__ __launch_bounds__(256) void k_wide_finish(
    const uint32_t* __restrict__ cnt, const int64_t* __restrict__ shi,
    const int64_t* __restrict__ slo, const double* __restrict__ periods, int64_t k, int32_t nbins,
    const CurveInfo* __restrict__ info, double* __restrict__ sums, int32_t* __restrict__ counts,
    double* __restrict__ means) {
    const double ref = info->ref, qs = info->qscale, qlo = ldexp(1.0, info->e_lo);
    const bool two = info->words == 2;
    const int64_t m = k * nbins;
    for (int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x; o < m; o += (int64_t)gridDim.x * 256) {
        const int64_t kk = o / nbins;
        const double P = periods[kk];
        const bool valid = P > 0.0 && isfinite(P);
        uint32_t c = cnt[o];
        double d = (double)shi[o] * qs;
        if (two) d += (double)slo[o] * qlo;
        const double sm = valid ? (double)c * ref + d : 0.0;
        if (!valid) c = 0;
        sums[o] = sm;
        counts[o] = (int32_t)c;
        if (means) means[o] = c ? sm / (double)c : __builtin_nan("");
    }
}

// Box-SNR of materialised folds at any nbins (power of two <= 4096): one
// block of 256 threads per row. Deviations from the row's own mean
// (D_b = sum_b - count_b ref; the SNR does not depend on the reference), FP64
// prefix sums {count, D} in LDS, every (width, start) box valued in FP32 by
// (S c_in - n D_in) / sqrt(c_in (n - c_in)) (proportional to its SNR) with
// c_in and D_in taken in FP64; the largest positive value wins (ties: smaller
// width, then smaller start), and is evaluated in FP64.
template <int NBMAX>
__global__ __launch_bounds__(256) void k_score_wide(
    const double* __restrict__ sums, const int32_t* __restrict__ counts, int64_t k, int32_t nb,
    double sigma_host, const double* __restrict__ sigma_dev, Widths W, float* __restrict__ snr,
    int32_t* __restrict__ start, int32_t* __restrict__ width, float* __restrict__ depth) {
    __shared__ double2 pre[NBMAX + 1];          // [nb + 1]: {count prefix, D prefix}
    __shared__ double red_d[8];
    __shared__ double red_c[8];
    __shared__ float red_v[4];
    __shared__ int32_t red_i[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t kk = blockIdx.x;
    const double* srow = sums + kk * nb;
    const int32_t* crow = counts + kk * nb;
    const double sigma = sigma_dev ? *sigma_dev : sigma_host;
    // totals (fixed order: contiguous chunks per thread, then waves in order)
    const int per = (nb + 255) / 256;
    const int b0 = min(nb, tid * per), b1 = min(nb, b0 + per);
    double ls = 0.0, lc = 0.0;
    for (int b = b0; b < b1; ++b) { ls += srow[b]; lc += (double)crow[b]; }
    double ws = ls, wc = lc;
    for (int d = 1; d < 64; d <<= 1) {   // inclusive wave prefix
        const double os = __shfl_up(ws, d), oc = __shfl_up(wc, d);
        if (lane >= d) { ws += os; wc += oc; }
    }
    if (lane == 63) { red_d[wave] = ws; red_c[wave] = wc; }
    __syncthreads();
    double Ssum = 0.0, n = 0.0;
    for (int w = 0; w < 4; ++w) { Ssum += red_d[w]; n += red_c[w]; }
    const double ref = n > 0.0 ? Ssum / n : 0.0;
    __syncthreads();
    // prefix of {count, D}: the thread's chunk, then an exclusive block offset
    double dl = 0.0;
    for (int b = b0; b < b1; ++b) dl += srow[b] - (double)crow[b] * ref;
    double wd = dl, wc2 = lc;
    for (int d = 1; d < 64; d <<= 1) {
        const double od = __shfl_up(wd, d), oc = __shfl_up(wc2, d);
        if (lane >= d) { wd += od; wc2 += oc; }
    }
    if (lane == 63) { red_d[wave] = wd; red_c[wave] = wc2; }
    __syncthreads();
    double od = __shfl_up(wd, 1), oc = __shfl_up(wc2, 1);   // exclusive within the wave
    if (lane == 0) { od = 0.0; oc = 0.0; }
    for (int w = 0; w < wave; ++w) { od += red_d[w]; oc += red_c[w]; }
    if (tid == 0) pre[0] = make_double2(0.0, 0.0);
    for (int b = b0; b < b1; ++b) {
        oc += (double)crow[b];
        od += srow[b] - (double)crow[b] * ref;
        pre[b + 1] = make_double2(oc, od);
    }
    __syncthreads();
    const double2 tot = pre[nb];
    const double S = tot.y;
    // active widths (w < nb), in order
    __shared__ int32_t wact[kMaxWidths];
    int nact = 0;
    for (int i = 0; i < W.n; ++i)
        if (W.w[i] < nb) {
            if (tid == 0) wact[nact] = W.w[i];
            ++nact;
        }
    __syncthreads();
    const bool ok = sigma > 0.0 && isfinite(sigma) && n > 0.0;
    float best = 0.0f;
    int bidx = 0x7fffffff;
    if (ok) {
        const int log2nb = 31 - __builtin_clz(nb);
        const int total = nact << log2nb;
        for (int idx = tid; idx < total; idx += 256) {
            const int wi = idx >> log2nb, s0 = idx & (nb - 1);
            const int w = wact[wi];
            const double2 a = pre[s0];
            double2 e;
            if (s0 + w <= nb) {
                e = pre[s0 + w];
            } else {
                const double2 e0 = pre[s0 + w - nb];
                e = make_double2(e0.x + tot.x, e0.y + tot.y);
            }
            const double cin = e.x - a.x, din = e.y - a.y;
            const double cout = n - cin;
            if (cin < 0.5 || cout < 0.5) continue;
            const float v = (float)(S * cin - n * din) * __builtin_amdgcn_rsqf((float)(cin * cout));
            if (v > best) { best = v; bidx = idx; }
        }
    }
    // block argmax: the largest value, then the smallest box index
    float wb = best;
    for (int d = 32; d > 0; d >>= 1) wb = fmaxf(wb, __shfl_xor(wb, d));
    int wi2 = (best == wb) ? bidx : 0x7fffffff;
    for (int d = 32; d > 0; d >>= 1) wi2 = min(wi2, __shfl_xor(wi2, d));
    if (lane == 0) { red_v[wave] = wb; red_i[wave] = wi2; }
    __syncthreads();
    if (tid != 0) return;
    float bv = 0.0f;
    int bi = 0x7fffffff;
    for (int w = 0; w < 4; ++w) {
        if (red_v[w] > bv) { bv = red_v[w]; bi = red_i[w]; }
        else if (red_v[w] == bv && red_i[w] < bi) bi = red_i[w];
    }
    float o_snr = 0.0f, o_depth = 0.0f;
    int32_t o_s = -1, o_w = -1;
    if (ok && bv > 0.0f && bi != 0x7fffffff) {
        const int log2nb = 31 - __builtin_clz(nb);
        const int wi = bi >> log2nb, s0 = bi & (nb - 1);
        const int w = wact[wi];
        const double2 a = pre[s0];
        double ec, ed;
        if (s0 + w <= nb) {
            ec = pre[s0 + w].x;
            ed = pre[s0 + w].y;
        } else {
            ec = pre[s0 + w - nb].x + tot.x;
            ed = pre[s0 + w - nb].y + tot.y;
        }
        const double nin = ec - a.x, din = ed - a.y;
        const double nout = n - nin;
        const double dep = (S - din) / nout - din / nin;
        o_snr = (float)(dep * sqrt(nin * nout / n) / sigma);
        o_depth = (float)dep;
        o_s = s0;
        o_w = w;
    }
    snr[kk] = o_snr;
    depth[kk] = o_depth;
    start[kk] = o_s;
    width[kk] = o_w;
}

// bf16 z-scored folds of materialised folds (nbins <= 256): one wave per row;
// bin means over non-empty bins, their mean and std (ddof 0) in FP64; empty
// bins and a zero spread give 0.
__global__ __launch_bounds__(256) void k_zfold_rows(const double* __restrict__ sums,
                                                    const int32_t* __restrict__ counts, int64_t k,
                                                    int32_t nb, uint16_t* __restrict__ zfold) {
    const int lane = threadIdx.x & 63;
    const int64_t kk = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (kk >= k) return;
    const double* srow = sums + kk * nb;
    const int32_t* crow = counts + kk * nb;
    double s1 = 0.0;
    int nz = 0;
    for (int b = lane; b < nb; b += 64)
        if (crow[b] > 0) { s1 += srow[b] / (double)crow[b]; ++nz; }
    s1 = wave_sum(s1);
    for (int o = 32; o > 0; o >>= 1) nz += __shfl_xor(nz, o, 64);
    const double mu = nz ? s1 / (double)nz : 0.0;
    double s2 = 0.0;
    for (int b = lane; b < nb; b += 64)
        if (crow[b] > 0) { const double d = srow[b] / (double)crow[b] - mu; s2 += d * d; }
    s2 = wave_sum(s2);
    const double sd = nz ? sqrt(s2 / (double)nz) : 0.0;
    for (int b = lane; b < nb; b += 64) {
        float z = 0.0f;
        if (crow[b] > 0 && sd > 0.0) z = (float)((srow[b] / (double)crow[b] - mu) / sd);
        zfold[kk * nb + b] = bf16_rne(z);
    }
}

// ------------------------------------------------------------------ launchers

hipError_t take_input_fault(int32_t* fault) {
    int32_t v = 0;
    hipError_t e = hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_input_fault), sizeof(v), 0,
                                       hipMemcpyDeviceToHost);
    if (e == hipSuccess && v) {
        const int32_t zero = 0;
        e = hipMemcpyToSymbol(HIP_SYMBOL(g_input_fault), &zero, sizeof(zero), 0,
                              hipMemcpyHostToDevice);
    }
    *fault = v;
    return e;
}

hipError_t launch_curve_stats(const double* t, const float* flux, int64_t n, CurveInfo* info,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_curve_stats, dim3(1), dim3(1024), 0, s, t, flux, (const int64_t*)nullptr,
                       n, info);
    return hipGetLastError();
}

int64_t fold_slice_len(int64_t n) {
    const int64_t q = kWaves * 2 * kBlk;
    const int64_t main = ((n > 0 ? n : 1) + q - 1) / q * q;
    return main / kWaves;
}

int64_t prepared_len(int64_t n) { return fold_slice_len(n) * kWaves + 2 * kBlk; }

int64_t slice_len(int64_t n) { return fold_slice_len(n); }

hipError_t launch_pack(const double* t, const float* flux, int64_t n, const CurveInfo* info,
                       Rec* rec, uint64_t* lo, hipStream_t s) {
    const int64_t total = prepared_len(n);
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_pack, dim3((unsigned)blocks), dim3(256), 0, s, t, flux,
                       (const int64_t*)nullptr, n, (const int64_t*)nullptr, total, info, rec, lo);
    return hipGetLastError();
}

static int log2_of(int32_t nbins) {
    int l = 0;
    while ((1 << l) < nbins) ++l;
    return l;
}

hipError_t launch_fold(const Rec* rec, const uint64_t* lo, int64_t n, const double* periods,
                       int64_t k, int32_t nbins, const CurveInfo* info, double* sums,
                       int32_t* counts, double* means, hipStream_t s) {
    if (k == 0) return hipSuccess;
    const int64_t blocks = (k + 63) / 64;
    hipLaunchKernelGGL(k_fold, dim3((unsigned)blocks), dim3(kThreads), 0, s, rec, lo,
                       fold_slice_len(n), periods, k, 8 - log2_of(nbins), info, sums, counts, means);
    return hipGetLastError();
}

hipError_t launch_fold_score(const Rec* rec, const uint64_t* lo, int64_t n,
                             const double* periods, int64_t k, int32_t nbins,
                             const CurveInfo* info, const Widths& widths, float* snr,
                             int32_t* start, int32_t* width, float* depth, uint16_t* zfold,
                             hipStream_t s) {
    if (k == 0) return hipSuccess;
    const int64_t blocks = (k + 63) / 64;
    hipLaunchKernelGGL(k_fold_score, dim3((unsigned)blocks), dim3(kThreads), 0, s, rec, lo,
                       fold_slice_len(n), periods, k, 8 - log2_of(nbins), info, widths, snr, start,
                       width, depth, zfold);
    return hipGetLastError();
}

hipError_t launch_fold_score_split(const Rec* rec, const uint64_t* lo, int64_t n,
                                   const double* periods, int64_t k, int32_t nbins,
                                   const CurveInfo* info, const Widths& widths, int32_t split,
                                   unsigned long long* gh, int32_t* arrivals, float* snr,
                                   int32_t* start, int32_t* width, float* depth, uint16_t* zfold,
                                   hipStream_t s) {
    if (k == 0) return hipSuccess;
    const int64_t tiles = (k + 63) / 64;
    const int64_t per = fold_slice_len(n);
    const int64_t q = 2 * kBlk;
    const int64_t per_s = ((per + split - 1) / split + q - 1) / q * q;
    hipLaunchKernelGGL(k_fold_score_split, dim3((unsigned)tiles, (unsigned)split), dim3(kThreads), 0, s,
                       rec, lo, per, per_s, periods, k, 8 - log2_of(nbins), info, widths, snr, start,
                       width, depth, zfold, gh, arrivals);
    return hipGetLastError();
}

hipError_t launch_fold_eqcount(const Rec* rec, const uint64_t* lo, int64_t n,
                               const double* periods, int64_t k, int32_t nbins,
                               const CurveInfo* info, double* means, uint16_t* zfold,
                               hipStream_t s) {
    if (k == 0) return hipSuccess;
    const int64_t blocks = (k + kEqPeriods - 1) / kEqPeriods;
    hipLaunchKernelGGL(k_fold_eqcount, dim3((unsigned)blocks), dim3(kThreads), 0, s, rec, lo,
                       fold_slice_len(n) * kWaves, periods, k, nbins, info, means, zfold);
    return hipGetLastError();
}

hipError_t launch_batch_prepare(const double* t, const float* flux, const int64_t* soff,
                                const int64_t* roff, int32_t n_curves, int64_t max_records,
                                CurveInfo* infos, Rec* rec, uint64_t* lo, hipStream_t s) {
    if (n_curves == 0) return hipSuccess;
    hipLaunchKernelGGL(k_curve_stats, dim3((unsigned)n_curves), dim3(1024), 0, s, t, flux, soff,
                       (int64_t)0, infos);
    const int64_t bx = std::min<int64_t>((max_records + 255) / 256, 64);
    hipLaunchKernelGGL(k_pack, dim3((unsigned)bx, (unsigned)n_curves), dim3(256), 0, s, t, flux, soff,
                       (int64_t)0, roff, (int64_t)0, infos, rec, lo);
    return hipGetLastError();
}

hipError_t launch_batch_fold_score(const Rec* rec, const uint64_t* lo, const BatchCurve* curves,
                                   const int2* items, int32_t n_items, int32_t* counter,
                                   const CurveInfo* infos, const double* periods, int32_t nbins,
                                   const Widths& widths, int32_t grid, float* snr, int32_t* start,
                                   int32_t* width, float* depth, uint16_t* zfold, hipStream_t s) {
    if (n_items == 0) return hipSuccess;
    hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(64), 0, s, counter, 0);
    hipLaunchKernelGGL(k_batch_fold_score, dim3((unsigned)std::min(grid, n_items)), dim3(kThreads), 0,
                       s, rec, lo, curves, items, n_items, counter, infos, periods,
                       8 - log2_of(nbins), widths, snr, start, width, depth, zfold);
    return hipGetLastError();
}

hipError_t launch_fold_f32(const Rec* rec, const uint64_t* lo, int64_t n, const double* periods,
                           int64_t k, int32_t nbins, int32_t compensated, const CurveInfo* info,
                           double* sums, int32_t* counts, double* means, hipStream_t s) {
    if (k == 0) return hipSuccess;
    const int64_t blocks = (k + 31) / 32;
    if (compensated)
        hipLaunchKernelGGL(k_fold_f32<true>, dim3((unsigned)blocks), dim3(kThreads), 0, s, rec, lo,
                           fold_slice_len(n), periods, k, 8 - log2_of(nbins), info, sums, counts, means);
    else
        hipLaunchKernelGGL(k_fold_f32<false>, dim3((unsigned)blocks), dim3(kThreads), 0, s, rec, lo,
                           fold_slice_len(n), periods, k, 8 - log2_of(nbins), info, sums, counts, means);
    return hipGetLastError();
}

hipError_t launch_score(const double* sums, const int32_t* counts, int64_t k, int32_t nbins,
                        double sigma, const Widths& widths, float* snr, int32_t* start,
                        int32_t* width, float* depth, hipStream_t s) {
    if (k == 0) return hipSuccess;
    const int64_t blocks = (k + 63) / 64;
    hipLaunchKernelGGL(k_score, dim3((unsigned)blocks), dim3(kThreads), 0, s, sums, counts, k,
                       nbins, sigma, widths, snr, start, width, depth);
    return hipGetLastError();
}

hipError_t launch_fold_wide(const Rec* rec, const uint64_t* lo, int64_t r0, int64_t r1,
                            const double* periods, int64_t k, int32_t nbins,
                            const CurveInfo* info, int32_t use_lo, int32_t first, uint32_t* cnt,
                            int64_t* shi, int64_t* slo, hipStream_t s) {
    if (k == 0) return hipSuccess;
    const int lg = log2_of(nbins);
    // fine bins: 256 up to nbins 256 (coarse bins are unions), else nbins
    const int logp = lg <= 8 ? 6 : 14 - lg;
    const int log2g = lg <= 8 ? 8 - lg : 0;
    const int64_t blocks = (k + (1 << logp) - 1) >> logp;
    switch (logp) {
#define GPFC_WIDE(L)                                                                              \
    case L:                                                                                       \
        hipLaunchKernelGGL(k_fold_wide<L>, dim3((unsigned)blocks), dim3(kThreads), 0, s, rec, lo, \
                           r0, r1, periods, k, log2g, info, use_lo, first, cnt, shi, slo);        \
        break;
        GPFC_WIDE(6)
        GPFC_WIDE(5)
        GPFC_WIDE(4)
        GPFC_WIDE(3)
        GPFC_WIDE(2)
#undef GPFC_WIDE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_wide_finish(const uint32_t* cnt, const int64_t* shi, const int64_t* slo,
                              const double* periods, int64_t k, int32_t nbins,
                              const CurveInfo* info, double* sums, int32_t* counts, double* means,
                              hipStream_t s) {
    const int64_t m = k * nbins;
    if (m == 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((m + 255) / 256, 65536);
    hipLaunchKernelGGL(k_wide_finish, dim3((unsigned)blocks), dim3(256), 0, s, cnt, shi, slo, periods,
                       k, nbins, info, sums, counts, means);
    return hipGetLastError();
}

hipError_t launch_score_wide(const double* sums, const int32_t* counts, int64_t k, int32_t nbins,
                             double sigma, const double* sigma_dev, const Widths& widths,
                             float* snr, int32_t* start, int32_t* width, float* depth,
                             hipStream_t s) {
    if (k == 0) return hipSuccess;
    if (k > 0x7fffffffLL) return hipErrorInvalidValue;
#define GPFC_SW(NB)                                                                                \
    hipLaunchKernelGGL(k_score_wide<NB>, dim3((unsigned)k), dim3(256), 0, s, sums, counts, k, nbins, \
                       sigma, sigma_dev, widths, snr, start, width, depth)
    if (nbins <= 256) GPFC_SW(256);
    else if (nbins <= 512) GPFC_SW(512);
    else if (nbins <= 1024) GPFC_SW(1024);
    else if (nbins <= 2048) GPFC_SW(2048);
    else GPFC_SW(4096);
#undef GPFC_SW
    return hipGetLastError();
}

hipError_t launch_zfold_rows(const double* sums, const int32_t* counts, int64_t k, int32_t nbins,
                             uint16_t* zfold, hipStream_t s) {
    if (k == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zfold_rows, dim3((unsigned)((k + 3) / 4)), dim3(256), 0, s, sums, counts, k,
                       nbins, zfold);
    return hipGetLastError();
}

hipError_t launch_fold_naive(const double* t, const float* flux, int64_t n,
                             const double* periods, int64_t k, int32_t nbins, double* sums,
                             int32_t* counts, hipStream_t s) {
    if (k == 0) return hipSuccess;
    const int64_t m = k * nbins;
    const int64_t zb = std::min<int64_t>((m + 255) / 256, 65536);
    hipLaunchKernelGGL(k_zero<double>, dim3((unsigned)zb), dim3(256), 0, s, sums, m);
    hipLaunchKernelGGL(k_zero<int32_t>, dim3((unsigned)zb), dim3(256), 0, s, counts, m);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fold_naive, dim3((unsigned)k), dim3(256), 0, s, t, flux, n, periods, nbins,
                       sums, counts);
    return hipGetLastError();
}

}  // namespace gpfc
