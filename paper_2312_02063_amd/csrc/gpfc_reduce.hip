// Per-curve reduction of periodograms: the best `top` (<= 64) scores of each
// row and their period indices (a curve's detection is its best score over
// the trial periods, Sec. 2.1; the maximum over periods is the statistic that
// is thresholded, Sec. 3.2).
//
// One block of 16 waves per row. Each wave streams a strided share of the row
// and keeps a 64-entry candidate list, one entry per lane, plus the list's
// worst entry broadcast to every lane: an element enters only when it beats
// that worst entry, so after the first few hundred elements almost every
// chunk is rejected by one compare and one ballot. The 16 lists (1024
// entries) are then ranked in LDS: an entry's place is the number of entries
// that beat it (keys are unique because indices are).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gpfc_internal.h"

namespace gpfc {
namespace {

constexpr int kTopWaves = 16;
constexpr int kTopThreads = kTopWaves * 64;
constexpr int64_t kNoIndex = INT64_MAX;

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

__global__ __launch_bounds__(kTopThreads) void k_topk_rows(const float* __restrict__ values,
                                                           const float* __restrict__ gate,
                                                           float gate_min, int64_t len, int32_t top,
                                                           float* __restrict__ out_val,
                                                           int64_t* __restrict__ out_idx) {
    __shared__ float lv_s[kTopThreads];
    __shared__ int64_t li_s[kTopThreads];
    __shared__ float ov_s[64];
    __shared__ int64_t oi_s[64];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t row = blockIdx.x;
    const float* v = values + row * len;
    const float* g = gate ? gate + row * len : nullptr;

    float lv = -INFINITY;        // this lane's list entry
    int64_t li = kNoIndex;
    float wv = -INFINITY;        // the list's worst entry and the lane holding it
    int64_t wi = kNoIndex;
    int wpos = 0;
    for (int64_t base = (int64_t)wave * 64; base < len; base += kTopThreads) {
        const int64_t i = base + lane;
        float x = 0.0f;
        bool cand = false;
        if (i < len) {
            x = v[i];
            cand = !__builtin_isnan(x) && (!g || g[i] >= gate_min) && beats(x, i, wv, wi);
        }
        uint64_t m = __ballot(cand);
        while (m) {
            const int s = __builtin_ctzll(m);
            m &= m - 1;
            const float sv = __shfl(x, s);
            const int64_t si = shfl64(i, s);
            if (!beats(sv, si, wv, wi)) continue;     // the list moved on meanwhile
            if (lane == wpos) { lv = sv; li = si; }
            // new worst: the entry every other entry beats
            float rv = lv;
            int64_t ri = li;
            int rp = lane;
            for (int d = 1; d < 64; d <<= 1) {
                const float ov = __shfl_xor(rv, d);
                const int64_t oi = shfl_xor64(ri, d);
                const int op = __shfl_xor(rp, d);
                // keep the worse one; equal keys (sentinels only): lower lane
                const bool take = beats(rv, ri, ov, oi) || (rv == ov && ri == oi && op < rp);
                if (take) { rv = ov; ri = oi; rp = op; }
            }
            wv = rv;
            wi = ri;
            wpos = rp;
        }
    }
    lv_s[threadIdx.x] = lv;
    li_s[threadIdx.x] = li;
    if (threadIdx.x < 64) { ov_s[threadIdx.x] = -INFINITY; oi_s[threadIdx.x] = -1; }
    __syncthreads();
    if (li != kNoIndex) {
        int rank = 0;
        for (int j = 0; j < kTopThreads; ++j) rank += beats(lv_s[j], li_s[j], lv, li) ? 1 : 0;
        if (rank < top) { ov_s[rank] = lv; oi_s[rank] = li; }
    }
    __syncthreads();
    if (threadIdx.x < top) {
        out_val[row * top + threadIdx.x] = ov_s[threadIdx.x];
        out_idx[row * top + threadIdx.x] = oi_s[threadIdx.x];
    }
}

}  // namespace

hipError_t launch_topk(const float* values, int64_t rows, int64_t len, const float* gate,
                       float gate_min, int32_t top, float* out_val, int64_t* out_idx, hipStream_t s) {
    if (rows == 0) return hipSuccess;
    hipLaunchKernelGGL(k_topk_rows, dim3((unsigned)rows), dim3(kTopThreads), 0, s, values, gate,
                       gate_min, len, top, out_val, out_idx);
    return hipGetLastError();
}

}  // namespace gpfc
