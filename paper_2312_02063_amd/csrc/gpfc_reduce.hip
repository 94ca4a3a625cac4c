// Per-curve reduction of periodograms: the best `top` (<= 64) scores of each
// row and their period indices (a curve's detection is its best score over
// the trial periods, Sec. 2.1; the maximum over periods is the statistic that
// is thresholded, Sec. 3.2).
//
// One block of 16 waves per row (or per part of a long row). Each wave
// streams a strided share of the row and keeps a `top`-entry candidate list,
// one entry per lane, plus the list's worst entry broadcast to every lane:
// an element enters only when it beats that worst entry, so after the first
// few hundred elements almost every chunk is rejected by one compare and one
// ballot. The 16 lists are then ranked in LDS: an entry's place is the
// number of entries that beat it (keys are unique because indices are).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "gpfc_internal.h"

namespace gpfc {
namespace {

constexpr int kTopWaves = 16;
constexpr int kTopThreads = kTopWaves * 64;

// Order: value descending, then index ascending.
__device__ __forceinline__ bool beats(float v, int64_t i, float w, int64_t j) {
    return v > w || (v == w && i < j);
}

__device__ __forceinline__ int64_t shfl64(int64_t x, int src) {
    const int lo = __shfl((int)(uint32_t)x, src);
    const int hi = __shfl((int)(x >> 32), src);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ int64_t shfl_xor64(int64_t x, int m) {
    const int lo = __shfl_xor((int)(uint32_t)x, m);
    const int hi = __shfl_xor((int)(x >> 32), m);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Block b takes part b % parts of row b / parts (parts > 1 splits a long
// row over many blocks; their lists are merged by a second launch over the
// parts' entries) and writes its best `top` to out[b][top]. With idx_in the
// entries carry their own indices (the merge; a negative index is an empty
// place), otherwise an entry's index is its position in the row.
// An entry's order as one 64-bit key, larger = better: the value's bits
// mapped to an unsigned order (-0 taken as +0, so equal values tie) in the
// high word, the complement of the index (< 2^32) in the low word. Key 0 is
// below every entry: an empty place.
__device__ __forceinline__ uint64_t top_key(float x, int64_t i) {
    const uint32_t u = __float_as_uint(x == 0.0f ? 0.0f : x);
    const uint32_t o = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return ((uint64_t)o << 32) | (uint32_t)~(uint32_t)i;
}

// Smallest key of the wave, in every lane: within each row of 16 lanes by
// DPP (swap neighbours, swap pairs, mirror 8, mirror 16), then across rows.
__device__ __forceinline__ uint64_t wave_min_key(uint64_t k) {
    auto dpp = [](uint64_t v, int ctrl) -> uint64_t {
        const int lo = (int)(uint32_t)v, hi = (int)(v >> 32);
        int rlo, rhi;
        switch (ctrl) {   // the control must be a constant
            case 0: rlo = __builtin_amdgcn_update_dpp(0, lo, 0xB1, 0xF, 0xF, false);
                    rhi = __builtin_amdgcn_update_dpp(0, hi, 0xB1, 0xF, 0xF, false); break;
            case 1: rlo = __builtin_amdgcn_update_dpp(0, lo, 0x4E, 0xF, 0xF, false);
                    rhi = __builtin_amdgcn_update_dpp(0, hi, 0x4E, 0xF, 0xF, false); break;
            case 2: rlo = __builtin_amdgcn_update_dpp(0, lo, 0x141, 0xF, 0xF, false);
                    rhi = __builtin_amdgcn_update_dpp(0, hi, 0x141, 0xF, 0xF, false); break;
            default: rlo = __builtin_amdgcn_update_dpp(0, lo, 0x140, 0xF, 0xF, false);
                     rhi = __builtin_amdgcn_update_dpp(0, hi, 0x140, 0xF, 0xF, false); break;
        }
        return ((uint64_t)(uint32_t)rhi << 32) | (uint32_t)rlo;
    };
    for (int c = 0; c < 4; ++c) {
        const uint64_t o = dpp(k, c);
        k = o < k ? o : k;
    }
    for (int d = 16; d < 64; d <<= 1) {
        const uint64_t o = (uint64_t)shfl_xor64((int64_t)k, d);
        k = o < k ? o : k;
    }
    return k;
}

// Block b takes part b % parts of row b / parts (parts > 1 splits a long
// row over many blocks; their lists are merged by a second launch over the
// parts' entries) and writes its best `top` to out[b][top]. With idx_in the
// entries carry their own indices (the merge; a negative index is an empty
// place), otherwise an entry's index is its position in the row.
__global__ __launch_bounds__(kTopThreads) void k_topk_rows(const float* __restrict__ values,
                                                           const float* __restrict__ gate,
                                                           float gate_min, int64_t len, int32_t top,
                                                           float* __restrict__ out_val,
                                                           int64_t* __restrict__ out_idx, int parts,
                                                           const int64_t* __restrict__ idx_in) {
    __shared__ uint64_t lk_s[kTopThreads];
    __shared__ float ov_s[64];
    __shared__ int64_t oi_s[64];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t row = blockIdx.x / parts;
    const int part = blockIdx.x - (int)row * parts;
    const int64_t chunk = ((len + parts - 1) / parts + 63) / 64 * 64;
    const int64_t lo = min(len, (int64_t)part * chunk), hi = min(len, lo + chunk);
    const float* v = values + row * len;
    const float* g = gate ? gate + row * len : nullptr;
    const int64_t* ix = idx_in ? idx_in + row * len : nullptr;
    // element p of the row: its value, key and whether it may enter
    auto fetch = [&](int64_t p, float& x, uint64_t& k) -> bool {
        if (p >= hi) return false;
        x = v[p];
        bool ok = !__builtin_isnan(x) && (!g || g[p] >= gate_min);
        int64_t i = p;
        if (ix) {
            i = ix[p];
            ok = ok && i >= 0;
        }
        k = top_key(x, i);
        return ok;
    };

    // The wave's list has `top` places, one per lane below `top`; lanes
    // above hold a key above every entry, so the list's worst is always a
    // real place and the threshold an element must beat is the top-th best
    // seen so far. With top = 64 the list starts as the wave's first 64
    // elements, one per lane.
    constexpr uint64_t kAbove = ~0ull;
    float lv = -INFINITY;        // this lane's list entry (value, key)
    uint64_t lk = lane < top ? 0 : kAbove;
    int64_t first = lo + (int64_t)wave * 64;
    if (top == 64) {
        float x;
        uint64_t k;
        if (fetch(first + lane, x, k)) { lv = x; lk = k; }
        first += kTopThreads;
    }
    uint64_t wk = wave_min_key(lk);   // the list's worst key and the lane holding it
    int wpos = __builtin_ctzll(__ballot(lk == wk));
    // kUnroll chunks of 64 per wave are loaded before any is examined, so
    // their memory latencies overlap
    constexpr int kUnroll = 8;
    for (int64_t base0 = first; base0 < hi; base0 += (int64_t)kTopThreads * kUnroll) {
      float xs[kUnroll];
      uint64_t ks[kUnroll];
      bool ok[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        xs[u] = 0.0f;
        ks[u] = 0;
        ok[u] = fetch(base0 + (int64_t)u * kTopThreads + lane, xs[u], ks[u]);
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        uint64_t m = __ballot(ok[u] && ks[u] > wk);
        while (m) {
            const int src = __builtin_ctzll(m);
            m &= m - 1;
            const uint64_t sk = (uint64_t)shfl64((int64_t)ks[u], src);
            if (sk <= wk) continue;                  // the list moved on meanwhile
            const float sv = __shfl(xs[u], src);
            if (lane == wpos) { lv = sv; lk = sk; }
            wk = wave_min_key(lk);
            wpos = __builtin_ctzll(__ballot(lk == wk));
        }
      }
    }
    // place of an entry = number of entries with a larger key (keys are
    // unique): each wave sorts its list by rank within the wave, then an
    // entry that can still place counts the larger keys of every other
    // wave's sorted list by binary search
    if (lk == kAbove) lk = 0;
    lk_s[threadIdx.x] = lk;
    if (threadIdx.x < 64) { ov_s[threadIdx.x] = -INFINITY; oi_s[threadIdx.x] = -1; }
    __syncthreads();
    // rank within the wave; equal keys (only empty places, key 0, can be
    // equal) are ordered by lane, so the ranks are a permutation of 0..63 and
    // the scatter below fills every slot of the wave's sorted list
    int lr = 0;
    for (int j = 0; j < 64; ++j) {
        const uint64_t o = lk_s[wave * 64 + j];
        lr += (o > lk || (o == lk && j < lane)) ? 1 : 0;
    }
    __syncthreads();
    lk_s[wave * 64 + lr] = lk;   // each wave's keys, descending
    __syncthreads();
    if (lk != 0 && lr < top) {
        int rank = lr;
        for (int w = 0; w < kTopWaves; ++w) {
            if (w == wave) continue;
            const uint64_t* a = lk_s + w * 64;
            int l = 0, h = 64;   // a[0, l) > lk >= a[h, 64)
            while (l < h) {
                const int mid = (l + h) >> 1;
                if (a[mid] > lk) l = mid + 1;
                else h = mid;
            }
            rank += l;
        }
        if (rank < top) { ov_s[rank] = lv; oi_s[rank] = (int64_t)(uint32_t)~(uint32_t)lk; }
    }
    __syncthreads();
    if (threadIdx.x < top) {
        out_val[(int64_t)blockIdx.x * top + threadIdx.x] = ov_s[threadIdx.x];
        out_idx[(int64_t)blockIdx.x * top + threadIdx.x] = oi_s[threadIdx.x];
    }
}

// ------------------------------------------------------------------ periodogram peaks
//
// One block of 16 waves per row: (1) count, sum and first maximum of the
// non-NaN scores, (2) the sum of squared deviations (two passes, FP64), so
// SDE = (max - mean) / sd; (3) runs above mean + nsigma sd: each thread scans
// a contiguous chunk, keeps its best internal runs (not touching the chunk
// ends) in a sorted list of kMaxPeaks and records the runs touching its ends;
// thread 0 joins those boundary runs across chunks in order; the per-thread
// lists are merged wave by wave and then with the joined runs. Peaks order by
// value descending, then index ascending, as the oracle.

constexpr int kMaxPeaks = 8;

struct Run {
    int64_t len;
    float mx;
    int64_t arg;
};

__device__ __forceinline__ Run join(Run a, Run b) {
    if (a.len == 0) return b;
    if (b.len == 0) return a;
    Run r;
    r.len = a.len + b.len;
    const bool tb = b.mx > a.mx;     // a comes first: it keeps ties
    r.mx = tb ? b.mx : a.mx;
    r.arg = tb ? b.arg : a.arg;
    return r;
}

struct PeakList {
    float v[kMaxPeaks];
    int64_t i[kMaxPeaks];
    int32_t w[kMaxPeaks];
    __device__ void init() {
        for (int a = 0; a < kMaxPeaks; ++a) { v[a] = -INFINITY; i[a] = INT64_MAX; w[a] = 0; }
    }
    // the entry walks down the list and changes places with every entry it
    // beats (the list stays sorted, its last entry drops out); fixed slots,
    // so the list stays in registers
    __device__ void insert(float pv, int64_t pi, int32_t pw) {
        if (!beats(pv, pi, v[kMaxPeaks - 1], i[kMaxPeaks - 1])) return;
#pragma unroll
        for (int a = 0; a < kMaxPeaks; ++a) {
            if (beats(pv, pi, v[a], i[a])) {
                const float tv = v[a];
                const int64_t ti = i[a];
                const int32_t tw = w[a];
                v[a] = pv;
                i[a] = pi;
                w[a] = pw;
                pv = tv;
                pi = ti;
                pw = tw;
            }
        }
    }
    // entry h (kMaxPeaks and above: an empty place), read by fixed slots
    __device__ void at(int h, float& ov, int64_t& oi, int32_t& ow) const {
        ov = -INFINITY;
        oi = INT64_MAX;
        ow = 0;
#pragma unroll
        for (int a = 0; a < kMaxPeaks; ++a)
            if (a == h) { ov = v[a]; oi = i[a]; ow = w[a]; }
    }
};

struct PeriodogramLds {
    double dred[kTopThreads / 64];
    int64_t cred[kTopThreads / 64];
    float mred[kTopThreads / 64];
    int64_t ared[kTopThreads / 64];
    int32_t nred[kTopThreads / 64];
    Run head[kTopThreads];
    Run tail[kTopThreads];
    uint8_t full[kTopThreads];
    float wv[kTopThreads / 64][kMaxPeaks];
    int64_t wi[kTopThreads / 64][kMaxPeaks];
    int32_t ww[kTopThreads / 64][kMaxPeaks];
    double mean, sd, thr;
    float mx;
    int64_t amx, m;
    // per wave: its threads' boundary runs joined (see join_block_runs)
    Run whead[kTopWaves], wtail[kTopWaves];
    uint8_t wfull[kTopWaves];
    int32_t wcnt[kTopWaves];
    float jv[kTopWaves][kMaxPeaks];
    int64_t ji[kTopWaves][kMaxPeaks];
    int32_t jw[kTopWaves][kMaxPeaks];
};

// Join the runs that cross the per-thread chunks, in chunk order: first each
// wave's lane 0 joins its 64 threads (runs completed inside the wave are
// counted and listed; the run touching the wave's first chunk start and the
// one touching its last chunk end are kept), then thread 0 joins the 16
// waves the same way. Called by every thread of the block; on thread 0 it
// adds the completed runs to fin / total and returns the block's head run
// (touching its first score), tail run (touching its last score) and
// whether every score of the block is above (then head is the whole block).
__device__ void join_block_runs(PeriodogramLds& sm, int32_t min_width, PeakList& fin, int32_t& total,
                                Run& bhead, Run& btail, bool& bfull) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const Run none{0, -INFINITY, INT64_MAX};
    if (lane == 0) {
        PeakList wl;
        wl.init();
        int32_t cnt = 0;
        Run open = none, head = none;
        bool first = true;
        for (int t = wave * 64; t < wave * 64 + 64; ++t) {
            if (sm.full[t]) {
                open = join(open, sm.head[t]);
            } else {
                const Run r = join(open, sm.head[t]);
                if (first) head = r;
                else if (r.len > min_width) { ++cnt; wl.insert(r.mx, r.arg, (int32_t)r.len); }
                first = false;
                open = sm.tail[t];
            }
        }
        sm.wfull[wave] = first ? 1 : 0;
        sm.whead[wave] = first ? open : head;
        sm.wtail[wave] = first ? none : open;
        sm.wcnt[wave] = cnt;
        for (int a = 0; a < kMaxPeaks; ++a) { sm.jv[wave][a] = wl.v[a]; sm.ji[wave][a] = wl.i[a]; sm.jw[wave][a] = wl.w[a]; }
    }
    __syncthreads();
    if (tid != 0) return;
    Run open = none, head = none;
    bool first = true;
    for (int w = 0; w < kTopWaves; ++w) {
        total += sm.wcnt[w];
        for (int a = 0; a < kMaxPeaks; ++a)
            if (sm.ji[w][a] != INT64_MAX) fin.insert(sm.jv[w][a], sm.ji[w][a], sm.jw[w][a]);
        if (sm.wfull[w]) {
            open = join(open, sm.whead[w]);
        } else {
            const Run r = join(open, sm.whead[w]);
            if (first) head = r;
            else if (r.len > min_width) { ++total; fin.insert(r.mx, r.arg, (int32_t)r.len); }
            first = false;
            open = sm.wtail[w];
        }
    }
    bfull = first;
    bhead = first ? open : head;
    btail = first ? none : open;
}

__global__ __launch_bounds__(kTopThreads) void k_periodogram(
    const float* __restrict__ values, const double* __restrict__ periods, int64_t len, float nsigma,
    int32_t min_width, int32_t max_peaks, float* __restrict__ sde, float* __restrict__ mean_out,
    float* __restrict__ sd_out, int32_t* __restrict__ n_peaks, float* __restrict__ pval,
    int64_t* __restrict__ pidx, int32_t* __restrict__ pwidth, int32_t* __restrict__ pharm) {
    __shared__ PeriodogramLds sm;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t row = blockIdx.x;
    const float* v = values + row * len;
    const int64_t cs = (len + kTopThreads - 1) / kTopThreads;
    const int64_t c0 = min(len, (int64_t)tid * cs), c1 = min(len, c0 + cs);
    // (1) count, sum, first maximum (strided: coalesced; the maximum's order
    // does not depend on the visiting order)
    int64_t m = 0;
    double s = 0.0;
    float mx = -INFINITY;
    int64_t amx = INT64_MAX;
    for (int64_t i0 = tid; i0 < len; i0 += 4 * kTopThreads) {
        float xs[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t i = i0 + (int64_t)u * kTopThreads;
            xs[u] = i < len ? v[i] : __builtin_nanf("");
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t i = i0 + (int64_t)u * kTopThreads;
            const float x = xs[u];
            if (__builtin_isnan(x)) continue;
            ++m;
            s += x;
            if (beats(x, i, mx, amx)) { mx = x; amx = i; }
        }
    }
    for (int d = 32; d > 0; d >>= 1) {
        m += __shfl_xor(m, d);
        s += __shfl_xor(s, d);
        const float om = __shfl_xor(mx, d);
        const int64_t oa = shfl_xor64(amx, d);
        if (beats(om, oa, mx, amx)) { mx = om; amx = oa; }
    }
    if (lane == 0) { sm.cred[wave] = m; sm.dred[wave] = s; sm.mred[wave] = mx; sm.ared[wave] = amx; }
    __syncthreads();
    if (tid == 0) {
        int64_t tm = 0;
        double ts = 0.0;
        float bm = -INFINITY;
        int64_t ba = INT64_MAX;
        for (int w = 0; w < kTopThreads / 64; ++w) {
            tm += sm.cred[w];
            ts += sm.dred[w];
            if (beats(sm.mred[w], sm.ared[w], bm, ba)) { bm = sm.mred[w]; ba = sm.ared[w]; }
        }
        sm.m = tm;
        sm.mean = tm ? ts / (double)tm : 0.0;
        sm.mx = bm;
        sm.amx = ba;
    }
    __syncthreads();
    // (2) squared deviations
    const double mean = sm.mean;
    double q = 0.0;
    for (int64_t i0 = tid; i0 < len; i0 += 4 * kTopThreads) {
        float xs[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t i = i0 + (int64_t)u * kTopThreads;
            xs[u] = i < len ? v[i] : __builtin_nanf("");
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (!__builtin_isnan(xs[u])) { const double d = xs[u] - mean; q += d * d; }
    }
    for (int d = 32; d > 0; d >>= 1) q += __shfl_xor(q, d);
    if (lane == 0) sm.dred[wave] = q;
    __syncthreads();
    if (tid == 0) {
        double tq = 0.0;
        for (int w = 0; w < kTopThreads / 64; ++w) tq += sm.dred[w];
        sm.sd = sm.m ? sqrt(tq / (double)sm.m) : 0.0;
        sm.thr = sm.mean + (double)nsigma * sm.sd;
    }
    __syncthreads();
    // (3) runs
    const double thr = sm.thr;
    PeakList pl;
    pl.init();
    int32_t np = 0;
    Run head{0, -INFINITY, INT64_MAX}, cur{0, -INFINITY, INT64_MAX};
    bool in_head = true;     // still inside a run that starts at c0
    for (int64_t i0 = c0; i0 < c1; i0 += 8) {
        float xs[8];     // loaded together so their latencies overlap
#pragma unroll
        for (int u = 0; u < 8; ++u) xs[u] = i0 + u < c1 ? v[i0 + u] : 0.0f;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t i = i0 + u;
            if (i >= c1) break;
            const float x = xs[u];
            const bool above = !__builtin_isnan(x) && (double)x > thr;
            if (above) {
                cur = join(cur, Run{1, x, i});
            } else {
                if (in_head) head = cur;
                else if (cur.len > min_width) { ++np; pl.insert(cur.mx, cur.arg, (int32_t)cur.len); }
                cur = Run{0, -INFINITY, INT64_MAX};
                in_head = false;
            }
        }
    }
    const bool full = in_head;     // every score of the chunk is above (an empty chunk too)
    sm.full[tid] = full ? 1 : 0;
    sm.head[tid] = full ? cur : head;
    sm.tail[tid] = full ? Run{0, -INFINITY, INT64_MAX} : cur;
    // merge the per-thread lists wave by wave: kMaxPeaks rounds of a wave argmax
    int h = 0;
    for (int rnd = 0; rnd < kMaxPeaks; ++rnd) {
        float bv;
        int64_t bi;
        int32_t bw;
        pl.at(h, bv, bi, bw);
        int bl = lane;
        for (int d = 32; d > 0; d >>= 1) {
            const float ov = __shfl_xor(bv, d);
            const int64_t oi = shfl_xor64(bi, d);
            const int ol = __shfl_xor(bl, d);
            if (beats(ov, oi, bv, bi) || (ov == bv && oi == bi && ol < bl)) { bv = ov; bi = oi; bl = ol; }
        }
        bw = __shfl(bw, bl);   // the winner's width
        if (lane == 0) { sm.wv[wave][rnd] = bv; sm.wi[wave][rnd] = bi; sm.ww[wave][rnd] = bw; }
        if (lane == bl) ++h;
    }
    for (int d = 32; d > 0; d >>= 1) np += __shfl_xor(np, d);
    if (lane == 0) sm.nred[wave] = np;
    __syncthreads();
    // join boundary runs across chunks, then merge everything (thread 0)
    PeakList fin;
    fin.init();
    int32_t total = 0;
    Run bhead, btail;
    bool bfull;
    join_block_runs(sm, min_width, fin, total, bhead, btail, bfull);
    if (tid != 0) return;
    for (int w = 0; w < kTopThreads / 64; ++w) {
        total += sm.nred[w];
        for (int a = 0; a < kMaxPeaks; ++a)
            if (sm.wi[w][a] != INT64_MAX) fin.insert(sm.wv[w][a], sm.wi[w][a], sm.ww[w][a]);
    }
    // the row's first and last runs are complete
    if (bhead.len > min_width) { ++total; fin.insert(bhead.mx, bhead.arg, (int32_t)bhead.len); }
    if (!bfull && btail.len > min_width) { ++total; fin.insert(btail.mx, btail.arg, (int32_t)btail.len); }
    const int64_t m_all = sm.m;
    const double sdv = sm.sd;
    sde[row] = (float)((m_all && sdv > 0.0) ? ((double)sm.mx - sm.mean) / sdv : 0.0);
    mean_out[row] = (float)sm.mean;
    sd_out[row] = (float)sdv;
    n_peaks[row] = total;
    const double p0 = (periods && fin.i[0] != INT64_MAX) ? periods[fin.i[0]] : 0.0;
#pragma unroll
    for (int a = 0; a < kMaxPeaks; ++a) {
        if (a >= max_peaks) break;
        const bool has = fin.i[a] != INT64_MAX;
        pval[row * max_peaks + a] = has ? fin.v[a] : -INFINITY;
        pidx[row * max_peaks + a] = has ? fin.i[a] : -1;
        pwidth[row * max_peaks + a] = has ? fin.w[a] : 0;
        int32_t code = 0;
        if (has && periods) {
            if (a == 0) code = 1;
            else {
                const double ratio = periods[fin.i[a]] / p0;
                for (int hh = 2; hh <= 3; ++hh) {
                    if (fabs(ratio - hh) <= 1e-3 * hh) code = hh;
                    if (fabs(1.0 / ratio - hh) <= 1e-3 * hh) code = -hh;
                }
            }
        }
        pharm[row * max_peaks + a] = code;
    }
}

// ---- the same for a few long rows, split over `parts` blocks per row:
// pass 1 and pass 2 write each part's count, sum, first maximum and sum of
// squared deviations; every later block derives the row's mean and sd from
// the parts in part order (the same values in every block); pass 3 finds
// each part's runs (its internal runs listed and counted, and the runs
// touching its ends); the last kernel joins those across the parts in order.
struct PartStats {
    int64_t m;
    double s, q;
    float mx;
    int64_t amx;
    Run head, tail;      // runs touching the part's first and last score
    int32_t full, np;    // every score of the part above; internal runs counted
    float pv[kMaxPeaks];
    int64_t pi[kMaxPeaks];
    int32_t pw[kMaxPeaks];
};

constexpr int kMaxParts = 256;   // parts per row in the split path

// A part's count and sums, copied to LDS by many threads at once so that
// the serial sums below read LDS rather than a chain of global loads.
struct PartSums {
    int64_t m;
    double s, q;
};

// Row count, mean and (with want_sd) standard deviation from the parts'
// records (PartStats or PartSums), summed in part order.
template <class S>
__device__ __forceinline__ void row_mean_sd(const S* ps, int parts, bool want_sd, int64_t& m,
                                            double& mean, double& sd) {
    m = 0;
    double ts = 0.0, tq = 0.0;
    for (int p = 0; p < parts; ++p) { m += ps[p].m; ts += ps[p].s; }
    mean = m ? ts / (double)m : 0.0;
    sd = 0.0;
    if (want_sd) {
        for (int p = 0; p < parts; ++p) tq += ps[p].q;
        sd = m ? sqrt(tq / (double)m) : 0.0;
    }
}

// pass 1 (stage 0) or pass 2 (stage 1) over one part of a row
__global__ __launch_bounds__(kTopThreads) void k_pgram_stats(const float* __restrict__ values, int64_t len,
                                                             int parts, int stage,
                                                             PartStats* __restrict__ ps) {
    __shared__ double dred[kTopWaves];
    __shared__ int64_t cred[kTopWaves];
    __shared__ float mred[kTopWaves];
    __shared__ int64_t ared[kTopWaves];
    __shared__ double mean_s;
    __shared__ PartSums psums[kMaxParts];
    if (parts > kMaxParts) return;   // the host splits a row into at most kMaxParts parts
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t row = blockIdx.x / parts;
    const int part = blockIdx.x - (int)row * parts;
    const int64_t chunk = ((len + parts - 1) / parts + 63) / 64 * 64;
    const int64_t lo = min(len, (int64_t)part * chunk), hi = min(len, lo + chunk);
    const float* v = values + row * len;
    PartStats* rp = ps + row * parts;
    if (stage == 1) {
        for (int p = tid; p < parts; p += kTopThreads) psums[p] = PartSums{rp[p].m, rp[p].s, 0.0};
        __syncthreads();
        if (tid == 0) {
            int64_t m;
            double mean, sd;
            row_mean_sd(psums, parts, false, m, mean, sd);
            mean_s = mean;
        }
        __syncthreads();
    }
    int64_t m = 0;
    double acc = 0.0;
    float mx = -INFINITY;
    int64_t amx = INT64_MAX;
    const double mean = stage == 1 ? mean_s : 0.0;
    for (int64_t i0 = lo + tid; i0 < hi; i0 += 4 * kTopThreads) {
        float xs[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t i = i0 + (int64_t)u * kTopThreads;
            xs[u] = i < hi ? v[i] : __builtin_nanf("");
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t i = i0 + (int64_t)u * kTopThreads;
            const float x = xs[u];
            if (__builtin_isnan(x)) continue;
            if (stage == 0) {
                ++m;
                acc += x;
                if (beats(x, i, mx, amx)) { mx = x; amx = i; }
            } else {
                const double d = x - mean;
                acc += d * d;
            }
        }
    }
    for (int d = 32; d > 0; d >>= 1) {
        m += __shfl_xor(m, d);
        acc += __shfl_xor(acc, d);
        const float om = __shfl_xor(mx, d);
        const int64_t oa = shfl_xor64(amx, d);
        if (beats(om, oa, mx, amx)) { mx = om; amx = oa; }
    }
    if (lane == 0) { cred[wave] = m; dred[wave] = acc; mred[wave] = mx; ared[wave] = amx; }
    __syncthreads();
    if (tid != 0) return;
    int64_t tm = 0;
    double ta = 0.0;
    float bm = -INFINITY;
    int64_t ba = INT64_MAX;
    for (int w = 0; w < kTopWaves; ++w) {
        tm += cred[w];
        ta += dred[w];
        if (beats(mred[w], ared[w], bm, ba)) { bm = mred[w]; ba = ared[w]; }
    }
    PartStats& o = rp[part];
    if (stage == 0) { o.m = tm; o.s = ta; o.mx = bm; o.amx = ba; }
    else o.q = ta;
}

// pass 3 over one part of a row
__global__ __launch_bounds__(kTopThreads) void k_pgram_runs(const float* __restrict__ values, int64_t len,
                                                            int parts, float nsigma, int32_t min_width,
                                                            PartStats* __restrict__ ps) {
    __shared__ PeriodogramLds sm;
    __shared__ PartSums psums[kMaxParts];
    if (parts > kMaxParts) return;   // the host splits a row into at most kMaxParts parts
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t row = blockIdx.x / parts;
    const int part = blockIdx.x - (int)row * parts;
    const int64_t chunk = ((len + parts - 1) / parts + 63) / 64 * 64;
    const int64_t lo = min(len, (int64_t)part * chunk), hi = min(len, lo + chunk);
    const float* v = values + row * len;
    PartStats* rp = ps + row * parts;
    for (int p = tid; p < parts; p += kTopThreads) psums[p] = PartSums{rp[p].m, rp[p].s, rp[p].q};
    __syncthreads();
    if (tid == 0) {
        int64_t m;
        double mean, sd;
        row_mean_sd(psums, parts, true, m, mean, sd);
        sm.thr = mean + (double)nsigma * sd;
    }
    __syncthreads();
    const double thr = sm.thr;
    const int64_t cs = (hi - lo + kTopThreads - 1) / kTopThreads;
    const int64_t c0 = min(hi, lo + (int64_t)tid * cs), c1 = min(hi, c0 + cs);
    PeakList pl;
    pl.init();
    int32_t np = 0;
    Run head{0, -INFINITY, INT64_MAX}, cur{0, -INFINITY, INT64_MAX};
    bool in_head = true;
    for (int64_t i0 = c0; i0 < c1; i0 += 8) {
        float xs[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) xs[u] = i0 + u < c1 ? v[i0 + u] : 0.0f;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t i = i0 + u;
            if (i >= c1) break;
            const float x = xs[u];
            const bool above = !__builtin_isnan(x) && (double)x > thr;
            if (above) {
                cur = join(cur, Run{1, x, i});
            } else {
                if (in_head) head = cur;
                else if (cur.len > min_width) { ++np; pl.insert(cur.mx, cur.arg, (int32_t)cur.len); }
                cur = Run{0, -INFINITY, INT64_MAX};
                in_head = false;
            }
        }
    }
    const bool full = in_head;
    sm.full[tid] = full ? 1 : 0;
    sm.head[tid] = full ? cur : head;
    sm.tail[tid] = full ? Run{0, -INFINITY, INT64_MAX} : cur;
    int h = 0;
    for (int rnd = 0; rnd < kMaxPeaks; ++rnd) {
        float bv;
        int64_t bi;
        int32_t bw;
        pl.at(h, bv, bi, bw);
        int bl = lane;
        for (int d = 32; d > 0; d >>= 1) {
            const float ov = __shfl_xor(bv, d);
            const int64_t oi = shfl_xor64(bi, d);
            const int ol = __shfl_xor(bl, d);
            if (beats(ov, oi, bv, bi) || (ov == bv && oi == bi && ol < bl)) { bv = ov; bi = oi; bl = ol; }
        }
        bw = __shfl(bw, bl);   // the winner's width
        if (lane == 0) { sm.wv[wave][rnd] = bv; sm.wi[wave][rnd] = bi; sm.ww[wave][rnd] = bw; }
        if (lane == bl) ++h;
    }
    for (int d = 32; d > 0; d >>= 1) np += __shfl_xor(np, d);
    if (lane == 0) sm.nred[wave] = np;
    __syncthreads();
    // the part's internal runs: those of the threads, and those joined
    // across threads that touch neither end of the part
    PeakList fin;
    fin.init();
    int32_t total = 0;
    Run bhead, btail;
    bool bfull;
    join_block_runs(sm, min_width, fin, total, bhead, btail, bfull);
    if (tid != 0) return;
    for (int w = 0; w < kTopWaves; ++w) {
        total += sm.nred[w];
        for (int a = 0; a < kMaxPeaks; ++a)
            if (sm.wi[w][a] != INT64_MAX) fin.insert(sm.wv[w][a], sm.wi[w][a], sm.ww[w][a]);
    }
    PartStats& o = rp[part];
    o.full = bfull ? 1 : 0;
    o.head = bhead;
    o.tail = btail;
    o.np = total;
    for (int a = 0; a < kMaxPeaks; ++a) { o.pv[a] = fin.v[a]; o.pi[a] = fin.i[a]; o.pw[a] = fin.w[a]; }
}

// last kernel: one wave per row. Lanes take parts lane, lane + 64, ...:
// the row's maximum, the parts' peak counts and internal peaks (into each
// lane's own list), and a copy of the part records in LDS; lane 0 then sums
// the statistics and joins the boundary runs in part order from that copy;
// the 64 lists merge into the row's best peaks by rounds of wave argmax (the
// same entries and order as one list fed everything). Results as
// k_periodogram writes them.
__global__ __launch_bounds__(64) void k_pgram_final(const PartStats* __restrict__ ps, int64_t rows, int parts,
                                                    const double* __restrict__ periods, int32_t min_width,
                                                    int32_t max_peaks, float* __restrict__ sde,
                                                    float* __restrict__ mean_out, float* __restrict__ sd_out,
                                                    int32_t* __restrict__ n_peaks, float* __restrict__ pval,
                                                    int64_t* __restrict__ pidx, int32_t* __restrict__ pwidth,
                                                    int32_t* __restrict__ pharm) {
    __shared__ PartStats sps[kMaxParts];
    const int64_t row = blockIdx.x;
    const int lane = threadIdx.x;
    if (row >= rows || parts > kMaxParts) return;
    const PartStats* rp = ps + row * parts;
    float mx = -INFINITY;
    int64_t amx = INT64_MAX;
    PeakList pl;
    pl.init();
    int32_t total = 0;
    for (int p = lane; p < parts; p += 64) {
        const PartStats& o = rp[p];
        sps[p] = o;
        if (beats(o.mx, o.amx, mx, amx)) { mx = o.mx; amx = o.amx; }
        total += o.np;
        for (int a = 0; a < kMaxPeaks; ++a)
            if (o.pi[a] != INT64_MAX) pl.insert(o.pv[a], o.pi[a], o.pw[a]);
    }
    __syncthreads();
    int64_t m = 0;
    double mean = 0.0, sdv = 0.0;
    if (lane == 0) {
        row_mean_sd(sps, parts, true, m, mean, sdv);
        Run open{0, -INFINITY, INT64_MAX};
        for (int p = 0; p < parts; ++p) {
            const PartStats& o = sps[p];
            if (o.full) {
                open = join(open, o.head);
            } else {
                const Run r = join(open, o.head);
                if (r.len > min_width) { ++total; pl.insert(r.mx, r.arg, (int32_t)r.len); }
                open = o.tail;
            }
        }
        if (open.len > min_width) { ++total; pl.insert(open.mx, open.arg, (int32_t)open.len); }
    }
    for (int d = 32; d > 0; d >>= 1) {
        total += __shfl_xor(total, d);
        const float ov = __shfl_xor(mx, d);
        const int64_t oa = shfl_xor64(amx, d);
        if (beats(ov, oa, mx, amx)) { mx = ov; amx = oa; }
    }
    PeakList fin;
    int h = 0;
#pragma unroll
    for (int rnd = 0; rnd < kMaxPeaks; ++rnd) {
        float bv;
        int64_t bi;
        int32_t bw;
        pl.at(h, bv, bi, bw);
        int bl = lane;
        for (int d = 32; d > 0; d >>= 1) {
            const float ov = __shfl_xor(bv, d);
            const int64_t oi = shfl_xor64(bi, d);
            const int ol = __shfl_xor(bl, d);
            if (beats(ov, oi, bv, bi) || (ov == bv && oi == bi && ol < bl)) { bv = ov; bi = oi; bl = ol; }
        }
        bw = __shfl(bw, bl);   // the winner's width
        fin.v[rnd] = bv;
        fin.i[rnd] = bi;
        fin.w[rnd] = bw;
        if (lane == bl) ++h;
    }
    if (lane != 0) return;
    sde[row] = (float)((m && sdv > 0.0) ? ((double)mx - mean) / sdv : 0.0);
    mean_out[row] = (float)mean;
    sd_out[row] = (float)sdv;
    n_peaks[row] = total;
    const double p0 = (periods && fin.i[0] != INT64_MAX) ? periods[fin.i[0]] : 0.0;
#pragma unroll
    for (int a = 0; a < kMaxPeaks; ++a) {
        if (a >= max_peaks) break;
        const bool has = fin.i[a] != INT64_MAX;
        pval[row * max_peaks + a] = has ? fin.v[a] : -INFINITY;
        pidx[row * max_peaks + a] = has ? fin.i[a] : -1;
        pwidth[row * max_peaks + a] = has ? fin.w[a] : 0;
        int32_t code = 0;
        if (has && periods) {
            if (a == 0) code = 1;
            else {
                const double ratio = periods[fin.i[a]] / p0;
                for (int hh = 2; hh <= 3; ++hh) {
                    if (fabs(ratio - hh) <= 1e-3 * hh) code = hh;
                    if (fabs(1.0 / ratio - hh) <= 1e-3 * hh) code = -hh;
                }
            }
        }
        pharm[row * max_peaks + a] = code;
    }
}

}  // namespace

hipError_t launch_periodogram(const float* values, int64_t rows, int64_t len, const double* periods,
                              float nsigma, int32_t min_width, int32_t max_peaks, float* sde,
                              float* mean, float* sd, int32_t* n_peaks, float* pval, int64_t* pidx,
                              int32_t* pwidth, int32_t* pharm, hipStream_t s) {
    if (rows == 0) return hipSuccess;
    // few long rows: each split over enough blocks to fill the chip (parts
    // of at least 16k scores), with stream-ordered scratch for the parts'
    // results; one block per row otherwise, and inside a graph capture
    int parts = 1;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone) {
        int dev = 0, n_cu = 256;
        if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
        const int64_t want = (2 * (int64_t)n_cu + rows - 1) / rows;
        parts = (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(want, kMaxParts), len / 16384));
    }
    if (parts <= 1) {
        hipLaunchKernelGGL(k_periodogram, dim3((unsigned)rows), dim3(kTopThreads), 0, s, values, periods,
                           len, nsigma, min_width, max_peaks, sde, mean, sd, n_peaks, pval, pidx, pwidth,
                           pharm);
        return hipGetLastError();
    }
    PartStats* ps = nullptr;
    hipError_t e = hipMallocAsync((void**)&ps, sizeof(PartStats) * rows * parts, s);
    if (e != hipSuccess) return e;
    const dim3 grid((unsigned)(rows * parts));
    hipLaunchKernelGGL(k_pgram_stats, grid, dim3(kTopThreads), 0, s, values, len, parts, 0, ps);
    hipLaunchKernelGGL(k_pgram_stats, grid, dim3(kTopThreads), 0, s, values, len, parts, 1, ps);
    hipLaunchKernelGGL(k_pgram_runs, grid, dim3(kTopThreads), 0, s, values, len, parts, nsigma, min_width, ps);
    hipLaunchKernelGGL(k_pgram_final, dim3((unsigned)rows), dim3(64), 0, s, (const PartStats*)ps,
                       rows, parts, periods, min_width, max_peaks, sde, mean, sd, n_peaks, pval, pidx, pwidth,
                       pharm);
    e = hipGetLastError();
    (void)hipFreeAsync(ps, s);
    return e;
}

hipError_t launch_topk(const float* values, int64_t rows, int64_t len, const float* gate,
                       float gate_min, int32_t top, float* out_val, int64_t* out_idx, hipStream_t s) {
    if (rows == 0) return hipSuccess;
    // few long rows: split each over enough blocks to fill the chip (each
    // part at least 8k scores), then merge the parts' lists; not inside a
    // graph capture (the split takes stream-ordered scratch memory)
    int parts = 1;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone) {
        int dev = 0, n_cu = 256;
        if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
        const int64_t want = (2 * (int64_t)n_cu + rows - 1) / rows;
        parts = (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(want, 256), len / 8192));
    }
    if (parts <= 1) {
        hipLaunchKernelGGL(k_topk_rows, dim3((unsigned)rows), dim3(kTopThreads), 0, s, values, gate,
                           gate_min, len, top, out_val, out_idx, 1, (const int64_t*)nullptr);
        return hipGetLastError();
    }
    const int64_t nc = rows * parts * top;
    float* cv = nullptr;
    int64_t* ci = nullptr;
    hipError_t e = hipMallocAsync((void**)&cv, sizeof(float) * nc, s);
    if (e == hipSuccess) e = hipMallocAsync((void**)&ci, sizeof(int64_t) * nc, s);
    if (e != hipSuccess) {
        if (cv) (void)hipFreeAsync(cv, s);
        return e;
    }
    hipLaunchKernelGGL(k_topk_rows, dim3((unsigned)(rows * parts)), dim3(kTopThreads), 0, s, values, gate,
                       gate_min, len, top, cv, ci, parts, (const int64_t*)nullptr);
    hipLaunchKernelGGL(k_topk_rows, dim3((unsigned)rows), dim3(kTopThreads), 0, s, (const float*)cv,
                       (const float*)nullptr, 0.0f, (int64_t)parts * top, top, out_val, out_idx, 1,
                       (const int64_t*)ci);
    e = hipGetLastError();
    (void)hipFreeAsync(cv, s);
    (void)hipFreeAsync(ci, s);
    return e;
}

}  // namespace gpfc
