// Learned scorer on gfx950: a 1-D CNN over noise-normalised folds (Sec. 2.5
// describes the paper's network: circular convolutions, max-pooling, fully
// connected ReLU layers, sigmoid output, cross-entropy, Adam). Layers here:
// 4 x [circular conv1d k5 -> ReLU -> max-pool 2] with 1->16->32->64->64
// channels over 256 positions, fully connected 1024->256->64->1, sigmoid.
//
// Convolutions 2-4 and the first two fully connected layers run as GEMMs on
// the matrix cores (v_mfma_f32_16x16x32_bf16 with FP32 accumulation, or
// v_mfma_f32_16x16x4_f32 in the FP32 mode); a convolution is an implicit
// GEMM whose operand loader gathers the five circularly shifted input rows.
// Activations are channels-last ([batch][position][channel]) so one lane
// fetches 8 consecutive channels at one position with a 16-byte load.
// Master weights, gradients and Adam moments are FP32 in the canonical
// layout (conv [Cout][Cin][5], fc [out][in], the flatten after block 4
// channel-major); the GEMMs read packed working copies.
//
// Inference of a bf16 network runs the four convolution blocks as one
// persistent kernel with every activation in LDS (k_convstack_bf16_w with
// wave-private inputs, or k_convstack_bf16 with tiles of 8) and the fully connected
// layers as LDS-tiled GEMMs (k_fc1_bf16, k_fc_bf16, the second with the
// output layer in its epilogue). A bf16 training step runs
// the same stack in a variant that also writes the activations and pooling
// masks to device memory, the backward data gradients down the blocks one
// kernel per block (k_convT_bf16, block 2's also giving block 1's weight
// gradients) and the other convolution weight gradients over LDS tiles of 8
// interleaved inputs (k_conv_dw_bf16, k_conv_dw_pipe_bf16); FP32
// networks and the layer path (gpfc_cnn_set_fused(0)) run layer by layer
// through device memory. A step can be replayed as one HIP graph. Every fused
// path gives the same bits as the layer path, except the convolution weight
// gradients, which differ only in FP32 summation order.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>

#include <algorithm>
#include <new>
#include <type_traits>
#include <string.h>

#include "../../include/gpfc.h"
#include "gpfc_internal.h"
#include "gpfc_mfma.h"

namespace gcnn {

constexpr int kNP = 312449;
constexpr int CH[5] = {1, 16, 32, 64, 64};
constexpr int LEN[5] = {256, 128, 64, 32, 16};
constexpr int64_t kConvW[5] = {0, 0, 96, 2688, 12992};
constexpr int64_t conv_b(int l) { return kConvW[l] + (int64_t)CH[l] * CH[l - 1] * 5; }
constexpr int64_t F1W = 33536, F1B = 295680, F2W = 295936, F2B = 312320, F3W = 312384, F3B = 312448;

// Bias-added pre-activations of a position pair -> the pooled activation:
// max(p0, p1, 0), i.e. ReLU then max-pool (one v_max3_f32). Every forward
// path (layer, fused, training) pools through this, so their outputs agree
// bit for bit; the training mask is taken from the same pair separately.
__device__ __forceinline__ float pool_relu(float p0, float p1) { return fmaxf(fmaxf(p0, p1), 0.0f); }

// Mask byte of one pooled output: bit 0 = the winning position (1: the odd
// one, chosen only when its ReLU output is strictly larger), bit 1 = the
// winner's pre-activation is > 0, which is the pooled value being > 0.
__device__ __forceinline__ uint32_t pool_mask(float p0, float p1, float pooled) {
    return (p1 > p0 && p1 > 0.0f ? 1u : 0u) | (pooled > 0.0f ? 2u : 0u);
}

// Implicit-GEMM rows of a circular conv input: row m = (b, x), k = dx*C + c
// -> act[b][(x + sgn*(dx - 2)) mod L][c]; sgn = +1 forward, -1 for the
// gradient with respect to the input.
template <class P>
struct ConvRows {
    using T = typename P::T;
    const T* act;
    int L, C, rows, sgn;
    __device__ __forceinline__ int64_t base(int m, int k) const {
        const int b = m / L, x = m - b * L;
        const int dx = k / C, c = k - dx * C;
        int pos = x + sgn * (dx - 2);
        pos = pos < 0 ? pos + L : (pos >= L ? pos - L : pos);
        return ((int64_t)b * L + pos) * C + c;
    }
    __device__ __forceinline__ bf16x8 frag8(int m, int k) const {
        if (m >= rows || k >= 5 * C) return bf16x8{};
        return *reinterpret_cast<const bf16x8*>(reinterpret_cast<const uint16_t*>(act) + base(m, k));
    }
    __device__ __forceinline__ float frag1(int m, int k) const {
        if (m >= rows || k >= 5 * C) return 0.0f;
        return P::to_f(act[base(m, k)]);
    }
};

// Weight-gradient operand of a conv: element (n = dx*Cin + ci, k = (b, x))
// = in[b][(x + dx - 2) mod L][ci].
template <class P>
struct ConvCols {
    using T = typename P::T;
    const T* act;
    int L, C, K;
    __device__ __forceinline__ float at(int n, int k) const {
        if (n >= 5 * C || k >= K) return 0.0f;
        const int b = k / L, x = k - b * L;
        const int dx = n / C, c = n - dx * C;
        int pos = x + dx - 2;
        pos = pos < 0 ? pos + L : (pos >= L ? pos - L : pos);
        return P::to_f(act[((int64_t)b * L + pos) * C + c]);
    }
    // bf16 elements are copied as they are (a bf16 -> float -> bf16 round trip
    // is exact); the index arithmetic is done once per fragment: k is a
    // multiple of 8 and L of 8, so the 8 positions lie in one input
    __device__ __forceinline__ bf16x8 frag8(int n, int k) const {
        u16x8 h;
        if (n < 5 * C && k + 8 <= K && (L & 7) == 0 && (k & 7) == 0) {
            const int b = k / L, x = k - b * L;
            const int dx = n / C, c = n - dx * C;
            const uint16_t* row = reinterpret_cast<const uint16_t*>(act) + (int64_t)b * L * C + c;
            for (int j = 0; j < 8; ++j) {
                int pos = x + j + dx - 2;
                pos = pos < 0 ? pos + L : (pos >= L ? pos - L : pos);
                h[j] = row[(int64_t)pos * C];
            }
        } else {
            for (int j = 0; j < 8; ++j) h[j] = f2bf(at(n, k + j));
        }
        return __builtin_bit_cast(bf16x8, h);
    }
    __device__ __forceinline__ float frag1(int n, int k) const { return at(n, k); }
};

// FP8 operand from a bf16 loader: scale, round to E4M3, pack 8 bytes.
template <class Base>
struct ActQ {
    Base base;
    float inv;
    __device__ __forceinline__ long frag8q(int m, int k) const {
        // whole-vector reinterpretation: a bit_cast of one vector element
        // (v[j]) is lowered as element 0 by this compiler
        const u16x8 v = __builtin_bit_cast(u16x8, base.frag8(m, k));
        uint64_t r = 0;
        for (int j = 0; j < 8; ++j) {
            const float f = bf2f(v[j]) * inv;
            r |= (uint64_t)f2e4m3(f) << (8 * j);
        }
        return (long)r;
    }
};

// FP8 weights stored as bytes, rows of ld.
struct WQ {
    const uint8_t* p;
    int rows, ld, K;
    __device__ __forceinline__ long frag8q(int n, int k) const {
        if (n >= rows || k + 8 > K) {
            uint64_t r = 0;
            for (int j = 0; j < 8; ++j)
                if (n < rows && k + j < K) r |= (uint64_t)p[(int64_t)n * ld + k + j] << (8 * j);
            return (long)r;
        }
        return *reinterpret_cast<const long*>(p + (int64_t)n * ld + k);
    }
};

// ---- epilogues

// Conv forward: rows are (b, x) positions (4 consecutive per lane), columns
// output channels. Bias, ReLU, max-pool over position pairs (both in the
// lane), store the pooled value and a mask byte (bit 0: the winning
// position's parity, bit 1: the winner's pre-activation is > 0).
template <class P>
struct EpConvFwd {
    using T = typename P::T;
    const float* bias;
    T* out;          // [b][L/2][C]
    uint8_t* mask;   // [b][L/2][C]
    int C;
    const float* colscale;   // FP8 mode: product of the two scales per column
    __device__ __forceinline__ void operator()(int m, int n, f32x4 a, int M, int N) const {
        if (n >= N) return;
        const float cs = colscale ? colscale[n] : 1.0f;
        for (int h = 0; h < 2; ++h) {
            const int mm = m + 2 * h;
            if (mm >= M) continue;
            const float p0 = a[2 * h] * cs + bias[n], p1 = a[2 * h + 1] * cs + bias[n];
            const int64_t o = (int64_t)(mm >> 1) * C + n;
            const float pooled = pool_relu(p0, p1);
            out[o] = P::from_f(pooled);
            if (mask) mask[o] = (uint8_t)pool_mask(p0, p1, pooled);
        }
    }
};

// Fully connected forward: rows batch, columns outputs; bias + ReLU.
template <class P>
struct EpFcFwd {
    using T = typename P::T;
    const float* bias;
    T* out;
    int ld;
    const float* colscale;
    __device__ __forceinline__ void operator()(int m, int n, f32x4 a, int M, int N) const {
        if (n >= N) return;
        const float cs = colscale ? colscale[n] : 1.0f;
        for (int i = 0; i < 4; ++i)
            if (m + i < M) out[(int64_t)(m + i) * ld + n] = P::from_f(fmaxf(a[i] * cs + bias[n], 0.0f));
    }
};

// Plain store of a data gradient, optionally masked by a ReLU output (> 0).
template <class P>
struct EpStore {
    using T = typename P::T;
    T* out;
    const T* relu_of;   // may be null
    int ld;
    __device__ __forceinline__ void operator()(int m, int n, f32x4 a, int M, int N) const {
        if (n >= N) return;
        for (int i = 0; i < 4; ++i)
            if (m + i < M) {
                const int64_t o = (int64_t)(m + i) * ld + n;
                float v = a[i];
                if (relu_of && !(P::to_f(relu_of[o]) > 0.0f)) v = 0.0f;
                out[o] = P::from_f(v);
            }
    }
};

// Weight gradient of conv layer l: rows co, columns n = dx*Cin + ci, written
// to the canonical [co][ci][dx] position (FP32).
struct EpConvDW {
    float* g;
    int Cin;
    __device__ __forceinline__ void store(int m, int n, float v) const {
        const int dx = n / Cin, ci = n - dx * Cin;
        g[((int64_t)m * Cin + ci) * 5 + dx] = v;
    }
    __device__ __forceinline__ void operator()(int m, int n, f32x4 a, int M, int N) const {
        if (n >= N) return;
        for (int i = 0; i < 4; ++i)
            if (m + i < M) store(m + i, n, a[i]);
    }
};

// Weight gradient of a fully connected layer: rows outputs, columns inputs.
// For fc1 the GEMM's input index j = x*64 + c maps to the canonical
// channel-major c*16 + x.
struct EpFcDW {
    float* g;
    int in;
    bool fc1;
    __device__ __forceinline__ void store(int m, int n, float v) const {
        const int i = fc1 ? ((n & 63) * 16 + (n >> 6)) : n;
        g[(int64_t)m * in + i] = v;
    }
    __device__ __forceinline__ void operator()(int m, int n, f32x4 a, int M, int N) const {
        if (n >= N) return;
        for (int r = 0; r < 4; ++r)
            if (m + r < M) store(m + r, n, a[r]);
    }
};

// Split-K partial sums: block z writes its tile to ws[z][m][n].
struct EpPartial {
    float* ws;
    __device__ __forceinline__ void operator()(int m, int n, f32x4 a, int M, int N) const {
        if (n >= N) return;
        float* w = ws + (int64_t)blockIdx.z * M * N;
        for (int r = 0; r < 4; ++r)
            if (m + r < M) w[(int64_t)(m + r) * N + n] = a[r];
    }
};

// Sum the split-K partials in z order (deterministic) and store through the
// weight-gradient epilogue.
template <class EP>
__global__ __launch_bounds__(256) void k_splitk_reduce(const float* __restrict__ ws, int S, int M,
                                                       int N, EP ep) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t mn = (int64_t)M * N;
    if (i >= mn) return;
    float v = 0.0f;
    for (int z = 0; z < S; ++z) v += ws[z * mn + i];
    ep.store((int)(i / N), (int)(i % N), v);
}

// The same for many partials: 64 consecutive outputs per block of 16 waves,
// one output per lane (each partial row is read coalesced); wave w adds
// partials w, w + 16, ... in that order, then the 16 wave sums are added in
// wave order (deterministic). Launch with ceil(M*N / 64) blocks of 1024.
template <class EP>
__global__ __launch_bounds__(1024) void k_splitk_reduce_w(const float* __restrict__ ws, int S, int M,
                                                          int N, EP ep) {
    __shared__ float red[16][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t mn = (int64_t)M * N;
    const int64_t i = (int64_t)blockIdx.x * 64 + lane;
    float v = 0.0f;
    if (i < mn)
        for (int z = wave; z < S; z += 16) v += ws[z * mn + i];
    red[wave][lane] = v;
    __syncthreads();
    if (wave == 0 && i < mn) {
        float t = 0.0f;
        for (int w = 0; w < 16; ++w) t += red[w][lane];
        ep.store((int)(i / N), (int)(i % N), t);
    }
}

// The same sums, 4 consecutive outputs per lane (16-byte loads of each
// partial row; M*N a multiple of 4): 256 outputs per block, each summed in
// exactly the order of k_splitk_reduce_w (same bits). Launch with
// ceil(M*N / 256) blocks of 1024.
template <class EP>
__global__ __launch_bounds__(1024) void k_splitk_reduce_w4(const float* __restrict__ ws, int S, int M, int N,
                                                           EP ep) {
    __shared__ float4 red[16][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t mn = (int64_t)M * N;
    const int64_t i = ((int64_t)blockIdx.x * 64 + lane) * 4;
    float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (i < mn)
        for (int z = wave; z < S; z += 16) {
            const float4 p = *reinterpret_cast<const float4*>(ws + z * mn + i);
            v.x += p.x;
            v.y += p.y;
            v.z += p.z;
            v.w += p.w;
        }
    red[wave][lane] = v;
    __syncthreads();
    if (wave == 0 && i < mn) {
        float t[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int w = 0; w < 16; ++w) {
            const float4 u = red[w][lane];
            t[0] += u.x;
            t[1] += u.y;
            t[2] += u.z;
            t[3] += u.w;
        }
        for (int c = 0; c < 4; ++c) ep.store((int)((i + c) / N), (int)((i + c) % N), t[c]);
    }
}

// k_splitk_reduce_w4 where the outputs allow it and still give it blocks
// enough to fill the chip, else k_splitk_reduce_w (4x the blocks).
template <class EP>
inline void reduce_partials_w(const float* ws, int S, int M, int N, EP ep, hipStream_t s) {
    const int64_t mn = (int64_t)M * N;
    if (mn % 4 == 0 && mn >= 512 * 256)
        hipLaunchKernelGGL((k_splitk_reduce_w4<EP>), dim3((unsigned)((mn + 255) / 256)), dim3(1024), 0, s, ws, S, M,
                           N, ep);
    else
        hipLaunchKernelGGL((k_splitk_reduce_w<EP>), dim3((unsigned)((mn + 63) / 64)), dim3(1024), 0, s, ws, S, M, N,
                           ep);
}

// Weight and bias gradients of a conv block reduced together: partial rows
// hold [COUT][5 CIN] weight sums, then COUT bias sums (M = 1, N = mn + COUT).
struct EpConvDWB {
    float* gw;
    float* gb;
    int Cin, mn;
    __device__ __forceinline__ void store(int, int j, float v) const {
        if (j >= mn) { gb[j - mn] = v; return; }
        const int m = j / (5 * Cin), n = j - m * (5 * Cin);
        const int dx = n / Cin, ci = n - dx * Cin;
        gw[((int64_t)m * Cin + ci) * 5 + dx] = v;
    }
};

// The weight and bias gradients of the convolution blocks of a bf16 training
// step reduced together: up to 4 jobs, each S partial rows of `row` floats
// ([COUT][5 CIN] weight sums, then COUT bias sums) in its own region. Pass 1
// (k_dw_seg) adds groups of kDwR consecutive rows into segment rows; pass 2
// (k_dw_final) adds a job's segments in order and stores through EpConvDWB:
// two launches for all the blocks, every sum in one fixed order.
constexpr int kDwR = 8;
struct DwJobs {
    const float* ws[4];
    float* seg[4];
    float* gw[4];
    float* gb[4];
    int S[4], row[4], cin[4];
    int ybase[5];   // pass 1: first segment (grid y) of each job
    int xbase[5];   // pass 2: first 64-column tile (grid x) of each job
    int n;
};

__device__ __forceinline__ int dw_job(const int* base, int n, int b) {
    int j = 0;
    while (j + 1 < n && b >= base[j + 1]) ++j;
    return j;
}

__global__ __launch_bounds__(256) void k_dw_seg(DwJobs J) {
    const int j = dw_job(J.ybase, J.n, blockIdx.y);
    const int y = blockIdx.y - J.ybase[j], S = J.S[j];
    const int64_t row = J.row[j];
    const int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
    if (i >= row) return;
    const float* ws = J.ws[j];
    const int z0 = y * kDwR;
    float4 p[kDwR];
#pragma unroll
    for (int u = 0; u < kDwR; ++u)
        p[u] = z0 + u < S ? *reinterpret_cast<const float4*>(ws + (z0 + u) * row + i)
                          : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
    for (int u = 0; u < kDwR; ++u) {
        v.x += p[u].x;
        v.y += p[u].y;
        v.z += p[u].z;
        v.w += p[u].w;
    }
    *reinterpret_cast<float4*>(J.seg[j] + y * row + i) = v;
}

__global__ __launch_bounds__(1024) void k_dw_final(DwJobs J) {
    __shared__ float red[16][64];
    const int j = dw_job(J.xbase, J.n, blockIdx.x);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = J.row[j], G = (J.S[j] + kDwR - 1) / kDwR;
    const int i = (blockIdx.x - J.xbase[j]) * 64 + lane;
    float v = 0.0f;
    if (i < row)
        for (int z = wave; z < G; z += 16) v += J.seg[j][(int64_t)z * row + i];
    red[wave][lane] = v;
    __syncthreads();
    if (wave == 0 && i < row) {
        float t = 0.0f;
        for (int w = 0; w < 16; ++w) t += red[w][lane];
        const int cin = J.cin[j], cout = row / (5 * cin + 1);
        EpConvDWB{J.gw[j], J.gb[j], cin, cout * 5 * cin}.store(0, i, t);
    }
}

// Weight and bias gradients of a dense layer reduced together: partial rows
// hold [M][N] weight sums (the weight-gradient epilogue's layout), then M
// bias sums (M = 1, N = M*N + M in the reduction's terms).
struct EpFcDWB {
    EpFcDW w;
    float* gb;
    int N, mn;
    __device__ __forceinline__ void store(int, int j, float v) const {
        if (j >= mn) { gb[j - mn] = v; return; }
        w.store(j / N, j - (j / N) * N, v);
    }
};

// ------------------------------------------------------------------ small kernels

// Conv block 1 (one input channel) on the vector units: x [B][256] (bf16
// bits or f32) -> pooled act1 [B][128][16] and mask.
template <class P>
__global__ __launch_bounds__(256) void k_conv1_fwd(const void* __restrict__ x, int xf32, int B,
                                                   const float* __restrict__ w /*[16][5]*/,
                                                   const float* __restrict__ bias,
                                                   typename P::T* __restrict__ out,
                                                   uint8_t* __restrict__ mask) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;   // (b, xp, co)
    if (idx >= (int64_t)B * 128 * 16) return;
    const int co = idx & 15;
    const int xp = (idx >> 4) & 127;
    const int b = (int)(idx >> 11);
    float pre[2];
    for (int h = 0; h < 2; ++h) {
        const int xx = 2 * xp + h;
        float s = bias[co];
        for (int dx = 0; dx < 5; ++dx) {
            const int pos = (xx + dx - 2) & 255;
            const int64_t o = (int64_t)b * 256 + pos;
            const float v = xf32 ? reinterpret_cast<const float*>(x)[o]
                                 : bf2f(reinterpret_cast<const uint16_t*>(x)[o]);
            s = __builtin_fmaf(w[co * 5 + dx], P::to_f(P::from_f(v)), s);
        }
        pre[h] = s;
    }
    const float pooled = pool_relu(pre[0], pre[1]);
    out[idx] = P::from_f(pooled);
    if (mask) mask[idx] = (uint8_t)pool_mask(pre[0], pre[1], pooled);
}

// Output layer of a training step, loss and its gradient (h2 [B][64] post-ReLU),
// in four passes with a fixed summation order (deterministic):
// k_head_rows: per input z = b3 + sum_i h2[i] w3[i] (the order of
//   k_head_infer), the logit if asked, dz = (sigmoid(z) - y) / B into
//   rows[0, B) and the loss term max(z, 0) - z y + log1p(exp(-|z|)) into
//   rows[B, 2B);
// k_head_dh2: dh2[b][i] = dz[b] w3[i] where h2[b][i] > 0, else 0;
// k_head_parts: sums of dz h2[.][i] (64), dz and the loss terms over parts
//   of kHeadRowsPerPart rows;
// k_head_final: the part sums added in part order into dW3, db3 and the loss.
template <class P>
__global__ __launch_bounds__(256) void k_head_rows(const typename P::T* __restrict__ h2, int B,
                                                   const float* __restrict__ w3,
                                                   const float* __restrict__ b3,
                                                   const float* __restrict__ labels,
                                                   float* __restrict__ logits, float* __restrict__ rows) {
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= B) return;
    float z = b3[0];
    for (int i = 0; i < 64; ++i) z += P::to_f(h2[(int64_t)b * 64 + i]) * w3[i];
    if (logits) logits[b] = z;
    const float y = labels[b];
    rows[B + b] = fmaxf(z, 0.0f) - z * y + log1pf(expf(-fabsf(z)));
    rows[b] = (1.0f / (1.0f + expf(-z)) - y) / (float)B;
}

template <class P>
__global__ __launch_bounds__(256) void k_head_dh2(const typename P::T* __restrict__ h2, int B,
                                                  const float* __restrict__ w3,
                                                  const float* __restrict__ rows,
                                                  typename P::T* __restrict__ dh2) {
    const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (o >= (int64_t)B * 64) return;
    const int i = (int)(o & 63);
    dh2[o] = P::from_f(P::to_f(h2[o]) > 0.0f ? rows[o >> 6] * w3[i] : 0.0f);
}

constexpr int kHeadSums = 66;   // dW3[64], db3, loss
constexpr int kHeadRowsPerPart = 128;   // rows per part: one part per block of the fused layer

// Block = one part of the rows; thread (row lane rl of 4, column i): sums over
// the part's rows rl, rl + 4, ...; lanes merged in order in LDS.
template <class P>
__global__ __launch_bounds__(256) void k_head_parts(const typename P::T* __restrict__ h2, int B,
                                                    const float* __restrict__ rows,
                                                    float* __restrict__ part_out) {
    __shared__ float red[4][kHeadSums];
    const int i = threadIdx.x & 63, rl = threadIdx.x >> 6;
    constexpr int64_t per = kHeadRowsPerPart;
    const int64_t r0 = (int64_t)blockIdx.x * per, r1 = min((int64_t)B, r0 + per);
    float sw = 0.0f, sb = 0.0f, sl = 0.0f;
    for (int64_t r = r0 + rl; r < r1; r += 4) {
        const float dz = rows[r];
        sw += dz * P::to_f(h2[r * 64 + i]);
        if (i == 0) { sb += dz; sl += rows[B + r]; }
    }
    red[rl][i] = sw;
    if (i == 0) { red[rl][64] = sb; red[rl][65] = sl; }
    __syncthreads();
    if (threadIdx.x < kHeadSums) {
        float t = 0.0f;
        for (int l = 0; l < 4; ++l) t += red[l][threadIdx.x];
        part_out[(int64_t)blockIdx.x * kHeadSums + threadIdx.x] = t;
    }
}

// One wave per sum j: lane l adds parts l, l + 64, ... in order, then the
// lanes are added by a fixed butterfly.
__device__ __forceinline__ float wave_sum_parts(const float* __restrict__ parts, int nparts, int n, int j,
                                                int lane) {
    float t = 0.0f;
    for (int p = lane; p < nparts; p += 64) t += parts[(int64_t)p * n + j];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    return t;
}

__global__ __launch_bounds__(256) void k_head_final(const float* __restrict__ parts, int nparts, int B,
                                                    float* __restrict__ grad, float* __restrict__ loss,
                                                    float* __restrict__ loss2) {
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (j >= kHeadSums) return;
    const float v = wave_sum_parts(parts, nparts, kHeadSums, j, lane);
    if (lane) return;
    if (j < 64) grad[F3W + j] = v;
    else if (j == 64) grad[F3B] = v;
    else {
        *loss = v / (float)B;
        if (loss2) *loss2 = v / (float)B;   // the caller's copy (no separate copy launch)
    }
}

// ------------------------------------------------------------------ fused inference
//
// The four convolution blocks of a bf16 network for inference, one persistent
// block per compute unit: the conv 2-4 weights (66 KB) are staged in LDS once,
// then tiles of kTileF inputs run conv1 on the vector units and conv2-4 as
// implicit GEMMs on the bf16 matrix cores with every activation kept in LDS
// (channels-last [fold][position][channel]); only the input (512 B) is read
// and the block-4 output (2 KB, position-major as the fc1 GEMM reads it) is
// written per input. Arithmetic and summation order are those of
// k_conv1_fwd and k_gemm with EpConvFwd, so the output is bit-identical to
// the layer-by-layer path.

constexpr int kTileF = 8;                       // inputs per tile
constexpr int kFusedThreads = 512;              // 8 waves
// LDS layouts. gfx950 serves a 16-byte-per-lane LDS read in four passes, over
// lanes {0-7, 24-31}, {8-15, 16-23}, {32-39, 56-63} and {40-47, 48-55} (found
// with bank-conflict counters on a probe of 20 access patterns); a pass is
// conflict-free when its 16 lanes hit distinct 16-byte slots modulo 256 bytes.
// An MFMA fragment load has lane (r, q) read row r, 16-byte chunk q, so:
// weight rows are padded to a stride of 32 mod 64 bytes (K padded to whole
// 32-steps plus 16), and activation rows keep their exact length with the
// chunks of a row XOR-swizzled (act_off): none for 32-byte rows (a1), chunk
// ^ 2*bit 2 of the row for 64-byte rows (a2), chunk ^ (row & 7) for 128-byte
// rows (a3).
constexpr int kW2Ld = 112, kW3Ld = 176, kW4Ld = 336;
constexpr int kA1Ld = 16, kA2Ld = 32, kA3Ld = 64;

struct ConvStackLds {
    uint16_t w2[32 * kW2Ld];
    uint16_t w3[64 * kW3Ld];
    uint16_t w4[64 * kW4Ld];
    float w1[16 * 5];
    float b1[16];
    uint16_t xs[kTileF * 256];                     // the tile's inputs (bf16)
    uint16_t buf0[kTileF * 32 * kA3Ld];            // a1 [F][128][16], then a3 [F][32][64]
    uint16_t buf1[kTileF * 64 * kA2Ld];            // a2 [F][64][32]
};
static_assert(kTileF * 128 * kA1Ld <= kTileF * 32 * kA3Ld, "a1 must fit where a3 goes");

// Element offset of (row, first channel ci0 of an 8-channel group) in an LDS
// activation buffer with rows of ILD channels (the swizzles above).
template <int ILD>
__device__ __forceinline__ int act_off(int row, int ci0) {
    static_assert(ILD == 16 || ILD == 32 || ILD == 64, "activation row lengths");
    if constexpr (ILD == 32) return row * 32 + (ci0 ^ (((row >> 2) & 1) << 4));
    if constexpr (ILD == 64) return row * 64 + (ci0 ^ ((row & 7) << 3));
    return row * 16 + ci0;
}
static_assert(sizeof(ConvStackLds) <= 160 * 1024, "LDS budget");

// One implicit-GEMM conv layer over the tile: rows (f, x) for x < L, columns
// output channels, k = dx*CIN + ci. Each wave takes 64 x 32 wave-tiles (4 x 2
// MFMA blocks of 16 x 16) and, per 32-step of k, loads 4 A and 2 B fragments
// from LDS. The epilogue adds the bias, applies ReLU and max-pools position
// pairs (both in the lane), then stores bf16 to `out` ([F][L/2][OLD] rows),
// skipping inputs >= nvalid when `to_global`.
template <int L, int CIN, int ILD, int COUT, int WLD, int OLD>
__device__ __forceinline__ void conv_tile(const uint16_t* __restrict__ in,
                                          const uint16_t* __restrict__ w,
                                          const float* __restrict__ bias, uint16_t* __restrict__ out,
                                          bool to_global, int nvalid) {
    constexpr int K = 5 * CIN;
    constexpr int KSTEPS = (K + 31) / 32;
    constexpr int M = kTileF * L;
    constexpr int NCT = COUT / 32;
    constexpr int NWT = (M / 64) * NCT;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int r = lane & 15, q = lane >> 4;
    for (int wt = wave; wt < NWT; wt += kFusedThreads / 64) {
        const int rt = wt / NCT, ct = wt - rt * NCT;
        f32x4 acc[4][2];
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < KSTEPS; ++ks) {
            const int k = ks * 32 + q * 8;
            const int dx = k / CIN, ci0 = k - dx * CIN;
            bf16x8 a[4], b[2];
            for (int i = 0; i < 4; ++i) {
                const int m = rt * 64 + i * 16 + r;
                const int f = m / L, x = m - f * L;
                int pos = x + dx - 2;
                pos = pos < 0 ? pos + L : (pos >= L ? pos - L : pos);
                a[i] = k < K ? *reinterpret_cast<const bf16x8*>(in + act_off<ILD>(f * L + pos, ci0)) : bf16x8{};
            }
            for (int j = 0; j < 2; ++j)
                b[j] = *reinterpret_cast<const bf16x8*>(w + (ct * 32 + j * 16 + r) * WLD + ks * 32 + q * 8);
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        for (int i = 0; i < 4; ++i) {
            const int m0 = rt * 64 + i * 16 + q * 4;      // 4 consecutive positions of one input
            const int f = m0 / L, x0 = m0 - f * L;
            if (to_global && f >= nvalid) continue;
            for (int j = 0; j < 2; ++j) {
                const int n = ct * 32 + j * 16 + r;
                const float bn = bias[n];
                for (int h = 0; h < 2; ++h) {
                    const float p0 = acc[i][j][2 * h] + bn, p1 = acc[i][j][2 * h + 1] + bn;
                    const int row = f * (L / 2) + (x0 >> 1) + h;
                    const int o = to_global ? row * OLD + n : act_off<OLD>(row, n & ~7) + (n & 7);
                    out[o] = f2bf(pool_relu(p0, p1));
                }
            }
        }
    }
}

// The tile's inputs as bf16 bits: thread t holds elements 4t .. 4t+3 of the
// [kTileF][256] tile (zeros past the last input).
__device__ __forceinline__ uint2 load_x4(const void* __restrict__ x, int xf32, int f0, int nvalid,
                                         int tid) {
    const int e = tid * 4;
    if ((e >> 8) >= nvalid) return make_uint2(0u, 0u);
    const int64_t o = (int64_t)f0 * 256 + e;
    if (xf32) {
        const float4 v = *reinterpret_cast<const float4*>(reinterpret_cast<const float*>(x) + o);
        return make_uint2((uint32_t)f2bf(v.x) | ((uint32_t)f2bf(v.y) << 16),
                          (uint32_t)f2bf(v.z) | ((uint32_t)f2bf(v.w) << 16));
    }
    return *reinterpret_cast<const uint2*>(reinterpret_cast<const uint16_t*>(x) + o);
}

__global__ __launch_bounds__(kFusedThreads, 1) void k_convstack_bf16(
    const void* __restrict__ x, int xf32, int B, const float* __restrict__ w1,
    const float* __restrict__ b1, const uint16_t* __restrict__ wf2, const float* __restrict__ b2,
    const uint16_t* __restrict__ wf3, const float* __restrict__ b3,
    const uint16_t* __restrict__ wf4, const float* __restrict__ b4, uint16_t* __restrict__ a4) {
    __shared__ __attribute__((aligned(16))) ConvStackLds sm;
    const int tid = threadIdx.x;
    for (int i = tid; i < 32 * kW2Ld; i += kFusedThreads) {
        const int n = i / kW2Ld, k = i - n * kW2Ld;
        sm.w2[i] = k < 80 ? wf2[n * 80 + k] : (uint16_t)0;
    }
    for (int i = tid; i < 64 * kW3Ld; i += kFusedThreads) {
        const int n = i / kW3Ld, k = i - n * kW3Ld;
        sm.w3[i] = k < 160 ? wf3[n * 160 + k] : (uint16_t)0;
    }
    for (int i = tid; i < 64 * kW4Ld; i += kFusedThreads) {
        const int n = i / kW4Ld, k = i - n * kW4Ld;
        sm.w4[i] = k < 320 ? wf4[n * 320 + k] : (uint16_t)0;
    }
    if (tid < 80) sm.w1[tid] = w1[tid];
    if (tid < 16) sm.b1[tid] = b1[tid];
    const int ntiles = (B + kTileF - 1) / kTileF;
    int tile = blockIdx.x;
    // 512 threads x 4 elements = one [8][256] tile
    uint2 xnext = tile < ntiles ? load_x4(x, xf32, tile * kTileF, min(kTileF, B - tile * kTileF), tid)
                                : make_uint2(0u, 0u);
    for (; tile < ntiles; tile += gridDim.x) {
        const int f0 = tile * kTileF;
        const int nvalid = min(kTileF, B - f0);
        reinterpret_cast<uint2*>(sm.xs)[tid] = xnext;
        __syncthreads();   // inputs and weights staged; the previous tile is done with buf0
        const int tn = tile + gridDim.x;   // prefetch the next tile's inputs
        if (tn < ntiles) xnext = load_x4(x, xf32, tn * kTileF, min(kTileF, B - tn * kTileF), tid);
        // conv1 (1 -> 16 channels) on the vector units, as k_conv1_fwd: thread
        // per (input, pooled position), all 16 channels
        for (int pi = tid; pi < kTileF * 128; pi += kFusedThreads) {
            const int f = pi >> 7, xp = pi & 127;
            float v[6];
            for (int d = 0; d < 6; ++d) v[d] = bf2f(sm.xs[f * 256 + ((2 * xp + d - 2) & 255)]);
            float pooled[16];
            for (int co = 0; co < 16; ++co) {
                float p0 = sm.b1[co], p1 = sm.b1[co];
                for (int dx = 0; dx < 5; ++dx) {
                    p0 = __builtin_fmaf(sm.w1[co * 5 + dx], v[dx], p0);
                    p1 = __builtin_fmaf(sm.w1[co * 5 + dx], v[dx + 1], p1);
                }
                pooled[co] = pool_relu(p0, p1);
            }
            uint32_t packed[8];
            for (int j = 0; j < 8; ++j) packed[j] = f2bf2(pooled[2 * j], pooled[2 * j + 1]);
            const int row = f * 128 + xp;
            uint4* dst = reinterpret_cast<uint4*>(sm.buf0 + row * kA1Ld);
            dst[0] = make_uint4(packed[0], packed[1], packed[2], packed[3]);
            dst[1] = make_uint4(packed[4], packed[5], packed[6], packed[7]);
        }
        __syncthreads();
        conv_tile<128, 16, kA1Ld, 32, kW2Ld, kA2Ld>(sm.buf0, sm.w2, b2, sm.buf1, false, nvalid);
        __syncthreads();
        conv_tile<64, 32, kA2Ld, 64, kW3Ld, kA3Ld>(sm.buf1, sm.w3, b3, sm.buf0, false, nvalid);
        __syncthreads();
        conv_tile<32, 64, kA3Ld, 64, kW4Ld, 64>(sm.buf0, sm.w4, b4, a4 + (int64_t)f0 * 1024, true,
                                                nvalid);
        __syncthreads();   // conv4 has read buf0 and every thread is done with xs
    }
}

// Variant of the fused convolution stack in which every wave takes whole
// inputs through all four blocks on its own: the block shares only the
// weights staged in LDS, each wave has a private slice of LDS for one input's
// activations, and nothing inside the loop waits for another wave, so one
// wave's vector work (conv1, epilogues) overlaps others' matrix work. Same
// arithmetic and summation order: bit-identical output.
constexpr int kWP = 8;                           // waves (inputs in flight) per block

struct WaveSlice {
    uint16_t xs[256];                            // the input (bf16)
    uint16_t buf0[32 * kA3Ld];                   // a1 [128][16], then a3 [32][64] (swizzled rows)
    uint16_t buf1[64 * kA2Ld];                   // a2 [64][32], then a4 [16][64] (swizzled rows)
    uint8_t mk[64 * 32];                         // a training step's pooling masks of one block
};

struct ConvStackLdsW {
    uint16_t w2[32 * kW2Ld];
    uint16_t w3[64 * kW3Ld];
    uint16_t w4[64 * kW4Ld];
    float bias[32 + 64 + 64];                    // blocks 2, 3, 4 (LDS reads: no wait on HBM stores)
    WaveSlice wv[kWP];
};
static_assert(128 * kA1Ld <= 32 * kA3Ld, "a1 must fit where a3 goes");
static_assert(sizeof(ConvStackLdsW) <= 160 * 1024, "LDS budget");

// LDS writes of this wave become visible to its later LDS reads.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One conv layer of one input by one wave: rows x < L, tiles of RB x CB MFMA
// blocks, as conv_tile (same k order, same epilogue). The pooled output goes
// to out (LDS, act_off rows of OLD channels); with kTrain each output's mask
// byte (bit 0: the winning position's parity, bit 1: the winner's
// pre-activation is > 0, as EpConvFwd stores it) goes to mlds [L/2][COUT].
template <int L, int CIN, int ILD, int COUT, int WLD, int OLD, int RB, int CB, bool kTrain = false>
__device__ __forceinline__ void conv_one(const uint16_t* __restrict__ in, const uint16_t* __restrict__ w,
                                         const float* __restrict__ bias, uint16_t* __restrict__ out,
                                         uint8_t* __restrict__ mlds = nullptr) {
    constexpr int K = 5 * CIN;
    constexpr int KSTEPS = (K + 31) / 32;
    constexpr int NRT = L / (16 * RB), NCT = COUT / (16 * CB);
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, q = lane >> 4;
    for (int t = 0; t < NRT * NCT; ++t) {
        const int rt = t / NCT, ct = t - rt * NCT;
        f32x4 acc[RB][CB];
        for (int i = 0; i < RB; ++i)
            for (int j = 0; j < CB; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < KSTEPS; ++ks) {
            const int k = ks * 32 + q * 8;
            const int dx = k / CIN, ci0 = k - dx * CIN;
            bf16x8 a[RB], b[CB];
            for (int i = 0; i < RB; ++i) {
                const int x = rt * 16 * RB + i * 16 + r;
                int pos = x + dx - 2;
                pos = pos < 0 ? pos + L : (pos >= L ? pos - L : pos);
                a[i] = k < K ? *reinterpret_cast<const bf16x8*>(in + act_off<ILD>(pos, ci0)) : bf16x8{};
            }
            for (int j = 0; j < CB; ++j)
                b[j] = *reinterpret_cast<const bf16x8*>(w + (ct * 16 * CB + j * 16 + r) * WLD + ks * 32 + q * 8);
            for (int i = 0; i < RB; ++i)
                for (int j = 0; j < CB; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        for (int i = 0; i < RB; ++i) {
            const int x0 = rt * 16 * RB + i * 16 + q * 4;
            for (int j = 0; j < CB; ++j) {
                const int n = ct * 16 * CB + j * 16 + r;
                const float bn = bias[n];
                for (int h = 0; h < 2; ++h) {
                    const float p0 = acc[i][j][2 * h] + bn, p1 = acc[i][j][2 * h + 1] + bn;
                    const int row = (x0 >> 1) + h;
                    const float pooled = pool_relu(p0, p1);
                    out[act_off<OLD>(row, n & ~7) + (n & 7)] = f2bf(pooled);
                    if constexpr (kTrain) mlds[row * COUT + n] = (uint8_t)pool_mask(p0, p1, pooled);
                }
            }
        }
    }
}

// One wave copies a pooled activation [ROWS][C] from LDS (act_off rows of C
// channels) to g [ROWS][C] in HBM, 16 bytes per lane and store.
template <int ROWS, int C>
__device__ __forceinline__ void act_to_hbm(const uint16_t* __restrict__ lds, uint16_t* __restrict__ g) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int t = lane; t < ROWS * C / 8; t += 64) {
        const int row = t / (C / 8), c0 = (t - row * (C / 8)) * 8;
        *reinterpret_cast<uint4*>(g + row * C + c0) = *reinterpret_cast<const uint4*>(lds + act_off<C>(row, c0));
    }
}

// One wave copies BYTES bytes (a multiple of 16) from LDS to HBM.
template <int BYTES>
__device__ __forceinline__ void bytes_to_hbm(const uint8_t* __restrict__ lds, uint8_t* __restrict__ g) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int t = lane; t < BYTES / 16; t += 64)
        reinterpret_cast<uint4*>(g)[t] = reinterpret_cast<const uint4*>(lds)[t];
}

// kTrain: the forward pass of a training step: besides a4, every block's
// pooled activations (a1 [B][128][16], a2 [B][64][32], a3 [B][32][64]) and
// pooling masks (m1 ... m4, the same layouts) go to HBM for the backward
// pass, with the values k_conv1_fwd and the EpConvFwd GEMMs would store.
// kXF32: the inputs are FP32 (rounded to bf16 when staged), else bf16 (a
// template flag: a branch between the two loads made the compiler wait for
// every store of the previous input before staging the next one).
template <bool kTrain, bool kXF32>
__global__ __launch_bounds__(kWP * 64, 1) void k_convstack_bf16_w(
    const void* __restrict__ x, int B, const float* __restrict__ w1,
    const float* __restrict__ b1, const uint16_t* __restrict__ wf2, const float* __restrict__ b2,
    const uint16_t* __restrict__ wf3, const float* __restrict__ b3,
    const uint16_t* __restrict__ wf4, const float* __restrict__ b4, uint16_t* __restrict__ a4,
    uint16_t* __restrict__ a1g, uint16_t* __restrict__ a2g, uint16_t* __restrict__ a3g,
    uint8_t* __restrict__ m1, uint8_t* __restrict__ m2, uint8_t* __restrict__ m3,
    uint8_t* __restrict__ m4) {
    __shared__ __attribute__((aligned(16))) ConvStackLdsW sm;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < 32 * kW2Ld; i += kWP * 64) {
        const int n = i / kW2Ld, k = i - n * kW2Ld;
        sm.w2[i] = k < 80 ? wf2[n * 80 + k] : (uint16_t)0;
    }
    for (int i = tid; i < 64 * kW3Ld; i += kWP * 64) {
        const int n = i / kW3Ld, k = i - n * kW3Ld;
        sm.w3[i] = k < 160 ? wf3[n * 160 + k] : (uint16_t)0;
    }
    for (int i = tid; i < 64 * kW4Ld; i += kWP * 64) {
        const int n = i / kW4Ld, k = i - n * kW4Ld;
        sm.w4[i] = k < 320 ? wf4[n * 320 + k] : (uint16_t)0;
    }
    // the biases too: read from HBM in the loop, their waits would also wait
    // for the stores issued before them
    if (tid < 160) sm.bias[tid] = tid < 32 ? b2[tid] : (tid < 96 ? b3[tid - 32] : b4[tid - 96]);
    __syncthreads();   // the only block-wide wait: weights staged
    WaveSlice& ws = sm.wv[wave];
    const int64_t stride = (int64_t)gridDim.x * kWP;
    // the wave's inputs: blockIdx * kWP + wave, + stride, ...; the next one's
    // 8 bytes per lane are loaded while the current one is computed
    int64_t fi = (int64_t)blockIdx.x * kWP + wave;
    // (FP32 inputs are kept as loaded and rounded when staged, so the load
    // is not waited for where it is issued)
    using XT = typename std::conditional<kXF32, float4, uint2>::type;
    auto load_in = [&](int64_t f) -> XT {
        f = f < B ? f : B - 1;   // (past the batch: read again, never used)
        const int64_t o = f * 256 + lane * 4;
        if constexpr (kXF32) {
            const u32x4v v = *reinterpret_cast<const u32x4v*>(reinterpret_cast<const float*>(x) + o);
            return make_float4(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z),
                               __uint_as_float(v.w));
        } else {
            return *reinterpret_cast<const uint2*>(reinterpret_cast<const uint16_t*>(x) + o);
        }
    };
    XT xnext = load_in(fi);
    for (; fi < B; fi += stride) {
        if constexpr (kXF32)
            reinterpret_cast<uint2*>(ws.xs)[lane] =
                make_uint2((uint32_t)f2bf(xnext.x) | ((uint32_t)f2bf(xnext.y) << 16),
                           (uint32_t)f2bf(xnext.z) | ((uint32_t)f2bf(xnext.w) << 16));
        else
            reinterpret_cast<uint2*>(ws.xs)[lane] = xnext;
        xnext = load_in(fi + stride);
        wave_lds_sync();
        // conv1: lane = 2 pooled positions, all 16 channels (as k_conv1_fwd;
        // weights and biases are wave-uniform: scalar loads)
        for (int xp = lane; xp < 128; xp += 64) {
            float v[6];
            for (int d = 0; d < 6; ++d) v[d] = bf2f(ws.xs[(2 * xp + d - 2) & 255]);
            float pooled[16];
            uint32_t mk[4] = {0u, 0u, 0u, 0u};
            for (int co = 0; co < 16; ++co) {
                float p0 = b1[co], p1 = b1[co];
                for (int dx = 0; dx < 5; ++dx) {
                    p0 = __builtin_fmaf(w1[co * 5 + dx], v[dx], p0);
                    p1 = __builtin_fmaf(w1[co * 5 + dx], v[dx + 1], p1);
                }
                pooled[co] = pool_relu(p0, p1);
                if constexpr (kTrain) mk[co >> 2] |= pool_mask(p0, p1, pooled[co]) << (8 * (co & 3));
            }
            uint32_t packed[8];
            for (int j = 0; j < 8; ++j) packed[j] = f2bf2(pooled[2 * j], pooled[2 * j + 1]);
            uint4* dst = reinterpret_cast<uint4*>(ws.buf0 + xp * kA1Ld);
            dst[0] = make_uint4(packed[0], packed[1], packed[2], packed[3]);
            dst[1] = make_uint4(packed[4], packed[5], packed[6], packed[7]);
            if constexpr (kTrain) {
                const int64_t o = (fi * 128 + xp) * 16;
                uint4* g = reinterpret_cast<uint4*>(a1g + o);
                g[0] = make_uint4(packed[0], packed[1], packed[2], packed[3]);
                g[1] = make_uint4(packed[4], packed[5], packed[6], packed[7]);
                *reinterpret_cast<uint4*>(m1 + o) = make_uint4(mk[0], mk[1], mk[2], mk[3]);
            }
        }
        wave_lds_sync();
        // each block's pooled output (and, training, its masks) is formed in
        // LDS, then copied to HBM in 16-byte stores
        conv_one<128, 16, kA1Ld, 32, kW2Ld, kA2Ld, 8, 2, kTrain>(ws.buf0, sm.w2, sm.bias, ws.buf1, ws.mk);
        wave_lds_sync();
        if constexpr (kTrain) {
            act_to_hbm<64, 32>(ws.buf1, a2g + fi * 2048);
            bytes_to_hbm<2048>(ws.mk, m2 + fi * 2048);
            wave_lds_sync();
        }
        conv_one<64, 32, kA2Ld, 64, kW3Ld, kA3Ld, 4, 4, kTrain>(ws.buf1, sm.w3, sm.bias + 32, ws.buf0, ws.mk);
        wave_lds_sync();
        if constexpr (kTrain) {
            act_to_hbm<32, 64>(ws.buf0, a3g + fi * 2048);
            bytes_to_hbm<2048>(ws.mk, m3 + fi * 2048);
            wave_lds_sync();
        }
        conv_one<32, 64, kA3Ld, 64, kW4Ld, kA3Ld, 2, 4, kTrain>(ws.buf0, sm.w4, sm.bias + 96, ws.buf1, ws.mk);
        wave_lds_sync();
        act_to_hbm<16, 64>(ws.buf1, a4 + fi * 1024);
        if constexpr (kTrain) bytes_to_hbm<1024>(ws.mk, m4 + fi * 1024);
        wave_lds_sync();   // buf0, buf1, mk and xs are reused by the next input
    }
}

// Fully connected layer for bf16 inference: out[m][n] = ReLU(bias[n] +
// sum_k A[m][k] W[n][k]) with A [M][K] activations and W [N][K] weights,
// both row-major bf16. Block tile 128 x BN, 4 waves of 64 x BN/2; K advances
// in steps of 64 through double-buffered LDS tiles (rows padded by 16
// elements) filled from registers loaded one step ahead. Each output's MFMA
// chain runs k in the same 32-steps as k_gemm, so results are bit-identical.
constexpr int kFcBK = 64, kFcLd = kFcBK + 16;   // rows of 160 bytes: conflict-free fragment reads

// EPI selects the epilogue: kFcRelu (bias + ReLU, the forward layer),
// kFcStore (plain store: a data gradient, as EpStore) or kFcHead (bias +
// ReLU of the second dense layer, then the output layer on the block's rows:
// hw holds the 64 output weights and the bias, logits receives one value per
// row, out is not written; needs BN = 64 and one column tile) or
// kFcHeadTrain (the same layer of a training step: the output layer, the
// loss and its gradient on the block's 128 rows, as k_head_rows, k_head_dh2
// and k_head_parts with parts of 128 rows do them: out receives dh2 [M][64],
// parts the block's kHeadSums sums; labels as k_head_rows). Blocks along y
// take further column tiles of BN.
constexpr int kFcRelu = 0, kFcStore = 1, kFcHead = 2, kFcHeadTrain = 3;
template <int BN, int EPI = kFcRelu>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_fc_bf16(int M, int K, const uint16_t* __restrict__ A,
                                                 const uint16_t* __restrict__ W,
                                                 const float* __restrict__ bias,
                                                 uint16_t* __restrict__ out, int ldo,
                                                 const float* __restrict__ hw, float* __restrict__ logits,
                                                 const float* __restrict__ labels = nullptr,
                                                 float* __restrict__ parts = nullptr) {
    constexpr int BM = 128;
    constexpr int WN = BN / 2;                 // columns per wave
    constexpr int NJ = WN / 16;                // MFMA column blocks per wave
    constexpr int ACH = BM * kFcBK / 8 / 256;  // 16-byte chunks of A per thread per step (4)
    constexpr int BCH = BN * kFcBK / 8 / 256;  // ... of W (4 or 2)
    __shared__ __attribute__((aligned(16))) uint16_t sa[2][BM * kFcLd];
    __shared__ __attribute__((aligned(16))) uint16_t sb[2][BN * kFcLd];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, q = lane >> 4;
    const int wm = wave & 1, wn = wave >> 1;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    uint4 ra[ACH], rb[BCH];
    auto load = [&](int k0) {
#pragma unroll
        for (int c = 0; c < ACH; ++c) {
            const int idx = tid + c * 256, row = idx >> 3, col = (idx & 7) * 8;
            ra[c] = (m0 + row < M) ? *reinterpret_cast<const uint4*>(A + (int64_t)(m0 + row) * K + k0 + col)
                                   : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int c = 0; c < BCH; ++c) {
            const int idx = tid + c * 256, row = idx >> 3, col = (idx & 7) * 8;
            rb[c] = ld_u4(W + (int64_t)(n0 + row) * K + k0 + col);
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int c = 0; c < ACH; ++c) {
            const int idx = tid + c * 256, row = idx >> 3, col = (idx & 7) * 8;
            *reinterpret_cast<uint4*>(&sa[buf][row * kFcLd + col]) = ra[c];
        }
#pragma unroll
        for (int c = 0; c < BCH; ++c) {
            const int idx = tid + c * 256, row = idx >> 3, col = (idx & 7) * 8;
            *reinterpret_cast<uint4*>(&sb[buf][row * kFcLd + col]) = rb[c];
        }
    };
    f32x4 acc[4][NJ];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < NJ; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    load(0);
    store(0);
    __syncthreads();
    const int steps = K / kFcBK;
    for (int st = 0; st < steps; ++st) {
        const int buf = st & 1;
        if (st + 1 < steps) load((st + 1) * kFcBK);
#pragma unroll
        for (int kk = 0; kk < kFcBK; kk += 32) {
            bf16x8 a[4], b[NJ];
            for (int i = 0; i < 4; ++i)
                a[i] = *reinterpret_cast<const bf16x8*>(&sa[buf][(wm * 64 + i * 16 + r) * kFcLd + kk + q * 8]);
            for (int j = 0; j < NJ; ++j)
                b[j] = *reinterpret_cast<const bf16x8*>(&sb[buf][(wn * WN + j * 16 + r) * kFcLd + kk + q * 8]);
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < NJ; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        if (st + 1 < steps) {
            store(buf ^ 1);   // the other buffer was last read in step st - 1
            __syncthreads();
        }
    }
    if constexpr (EPI == kFcHead) {
        static_assert(BN == 64, "the output layer reads whole 64-wide rows");
        // the block's 128 x 64 bf16 activations in LDS, rows of 144 bytes
        // (16 consecutive rows hit distinct 16-byte slots), then one thread
        // per row sums bias + h[i] w[i] over i in index order, the same
        // FP32 sequence as k_head_infer
        constexpr int kHLd = 72;
        static_assert(BM * kHLd <= BM * kFcLd, "fits the first A buffer");
        uint16_t* hs = sa[0];
        __syncthreads();   // every wave has finished its last fragment reads
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < NJ; ++j) {
                const int n = wn * WN + j * 16 + r;
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    hs[(wm * 64 + i * 16 + q * 4 + e) * kHLd + n] = f2bf(fmaxf(acc[i][j][e] + bias[n], 0.0f));
            }
        __syncthreads();
        if (tid < BM && m0 + tid < M) {
            float z = hw[64];
#pragma unroll
            for (int c8 = 0; c8 < 8; ++c8) {
                const uint4 v = *reinterpret_cast<const uint4*>(&hs[tid * kHLd + c8 * 8]);
                const uint32_t u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    z += bf2f((uint16_t)(u[k] & 0xFFFFu)) * hw[c8 * 8 + 2 * k];
                    z += bf2f((uint16_t)(u[k] >> 16)) * hw[c8 * 8 + 2 * k + 1];
                }
            }
            logits[m0 + tid] = z;
        }
    } else if constexpr (EPI == kFcHeadTrain) {
        static_assert(BN == 64, "the output layer reads whole 64-wide rows");
        constexpr int kHLd = 72;
        uint16_t* hs = sa[0];
        float* rowv = reinterpret_cast<float*>(sb[0]);   // dz [128], loss terms [128], then [4][kHeadSums]
        static_assert(256 + 4 * kHeadSums <= BN * kFcLd / 2, "fits the first W buffer");
        __syncthreads();   // every wave has finished its last fragment reads
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < NJ; ++j) {
                const int n = wn * WN + j * 16 + r;
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    hs[(wm * 64 + i * 16 + q * 4 + e) * kHLd + n] = f2bf(fmaxf(acc[i][j][e] + bias[n], 0.0f));
            }
        __syncthreads();
        if (tid < BM) {
            float dz = 0.0f, lt = 0.0f;
            if (m0 + tid < M) {
                float z = hw[64];
                for (int i = 0; i < 64; ++i) z += bf2f(hs[tid * kHLd + i]) * hw[i];
                if (logits) logits[m0 + tid] = z;
                const float y = labels[m0 + tid];
                lt = fmaxf(z, 0.0f) - z * y + log1pf(expf(-fabsf(z)));
                dz = (1.0f / (1.0f + expf(-z)) - y) / (float)M;
            }
            rowv[tid] = dz;
            rowv[BM + tid] = lt;
        }
        __syncthreads();
        for (int k = 0; k < BM * 64 / 256; ++k) {
            const int idx = tid + k * 256, row = idx >> 6, i = idx & 63;
            if (m0 + row < M)
                out[(int64_t)(m0 + row) * 64 + i] =
                    f2bf(bf2f(hs[row * kHLd + i]) > 0.0f ? rowv[row] * hw[i] : 0.0f);
        }
        float* red = rowv + 2 * BM;
        {
            const int i = tid & 63, rl = tid >> 6;
            const int nrows = min(BM, M - m0);
            float sw = 0.0f, sbias = 0.0f, sl = 0.0f;
            for (int rr = rl; rr < nrows; rr += 4) {
                const float dz = rowv[rr];
                sw += dz * bf2f(hs[rr * kHLd + i]);
                if (i == 0) { sbias += dz; sl += rowv[BM + rr]; }
            }
            red[rl * kHeadSums + i] = sw;
            if (i == 0) { red[rl * kHeadSums + 64] = sbias; red[rl * kHeadSums + 65] = sl; }
        }
        __syncthreads();
        if (tid < kHeadSums) {
            float t = 0.0f;
            for (int l = 0; l < 4; ++l) t += red[l * kHeadSums + tid];
            parts[(int64_t)blockIdx.x * kHeadSums + tid] = t;
        }
    } else {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int n = n0 + wn * WN + j * 16 + r;
            const int mb = m0 + wm * 64 + i * 16 + q * 4;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float v = acc[i][j][e];
                if constexpr (EPI == kFcRelu) v = fmaxf(v + bias[n], 0.0f);
                if (mb + e < M) out[(int64_t)(mb + e) * ldo + n] = f2bf(v);
            }
        }
    }
}

// The first fully connected layer for bf16 inference (N = 256 outputs): one
// block of 16 waves computes 256 rows x all 256 columns (waves 4 x 4, each
// 64 x 64), so every activation row is read once and the weights once per
// 256 rows. K advances in steps of 32 through four LDS stages filled straight
// from global memory (global_load_lds_dwordx4: a wave's 64 lanes write 1 KB of
// LDS in lane order, no registers in between), issued three steps ahead with
// one block barrier per step: 48 KB of activations in flight per CU, which
// the HBM stream needs (two steps of 128-row tiles kept too little of it in
// flight). A row of a stage is 64 B of 16-byte chunks stored XOR-swizzled
// (chunk c of row r at slot c ^ 2*bit 2 of r), conflict-free for the fragment
// reads. Same MFMA chains and epilogue as k_gemm with EpFcFwd: bit-identical
// output.
// s_waitcnt immediate that waits for vector memory operations only, until at
// most n (< 64) remain: vmcnt bits 3:0 at 3:0 and 5:4 at 15:14, expcnt (6:4)
// and lgkmcnt (11:8) at their maxima (no wait).
constexpr int vmcnt_imm(int n) { return 0x0F70 | (n & 15) | ((n >> 4) & 3) << 14; }
typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void glb_void_t;
constexpr int kF1BN = 256, kF1BK = 32;

// BM = 256 (16 waves), 128 (8 waves) or 64 (4 waves): the largest whose
// blocks fill the chip.
// Smaller row tiles keep more stages (LDS allowing), so that about as many
// bytes stay in flight per CU.
template <int BM>
__global__ __launch_bounds__(BM * 4, 1) void k_fc1_bf16(int M, int K, const uint16_t* __restrict__ A,
                                                      const uint16_t* __restrict__ W,
                                                      const float* __restrict__ bias,
                                                      uint16_t* __restrict__ out) {
    constexpr int kF1Stages = BM == 64 ? 7 : (BM == 128 ? 5 : 4);
    constexpr int kWaves = BM / 16;                   // 16 rows of A per wave per step
    constexpr int kWLoads = kF1BN / 16 / kWaves;      // W loads per wave per step
    constexpr int kLoads = 1 + kWLoads;               // loads per wave per step
    constexpr int kStageA = BM * kF1BK * 2, kStageB = kF1BN * kF1BK * 2;   // bytes per stage
    static_assert((kF1Stages - 2) * kLoads <= 63, "vmcnt range");
    __shared__ __attribute__((aligned(1024))) char smem[kF1Stages * (kStageA + kStageB)];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, q = lane >> 4;
    const int wm = wave % (BM / 64), wn = wave / (BM / 64);
    const int m0 = blockIdx.x * BM;
    // a wave's 1 KB load is 16 rows x 4 chunks: this lane's row is
    // 16 w + (lane >> 2) of load w, its slot lane & 3, holding global chunk
    // (lane & 3) ^ 2*bit 2 of the row
    const int lr = lane >> 2;
    const int lchunk = (lane & 3) ^ (((lr >> 2) & 1) << 1);
    const uint16_t* ga = A + (int64_t)min(m0 + wave * 16 + lr, M - 1) * K + lchunk * 8;   // rows past M: never stored
    // W is k-blocked ([K/32][256][32]): a step's slice is contiguous
    const uint16_t* gw[kWLoads];
    for (int j = 0; j < kWLoads; ++j) gw[j] = W + ((wave * kWLoads + j) * 16 + lr) * kF1BK + lchunk * 8;
    auto stage_a = [&](int st) { return smem + st * (kStageA + kStageB); };
    auto stage_b = [&](int st) { return smem + st * (kStageA + kStageB) + kStageA; };
    auto issue = [&](int step) {
        const int st = step % kF1Stages, k0 = step * kF1BK;
        __builtin_amdgcn_global_load_lds((glb_void_t*)(ga + k0), (lds_void_t*)(stage_a(st) + wave * 1024), 16, 0, 0);
        for (int j = 0; j < kWLoads; ++j)
            __builtin_amdgcn_global_load_lds((glb_void_t*)(gw[j] + (int64_t)step * kF1BN * kF1BK),
                                             (lds_void_t*)(stage_b(st) + (wave * kWLoads + j) * 1024), 16, 0, 0);
    };
    auto frag = [&](const char* base, int rw, int chunk) {
        return *reinterpret_cast<const bf16x8*>(base + rw * 64 + ((chunk ^ (((rw >> 2) & 1) << 1)) << 4));
    };
    f32x4 acc[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const int steps = K / kF1BK;
    for (int i = 0; i < kF1Stages - 1 && i < steps; ++i) issue(i);
    for (int st = 0; st < steps; ++st) {
        // this wave's loads of step st are done (kLoads per step; those of
        // the next steps may still be in flight), then every wave's, and
        // every wave is done reading the stage that step st + stages - 1
        // refills (a bare barrier: __syncthreads' fence would also wait for
        // the later loads)
        // (s_waitcnt's vmcnt is 6 bits: bits 3:0 of the immediate, then 15:14)
        const int ahead = min(kF1Stages - 2, steps - 1 - st);   // later steps already issued
        switch (ahead) {
            case 5: __builtin_amdgcn_s_waitcnt(vmcnt_imm(5 * kLoads)); break;
            case 4: __builtin_amdgcn_s_waitcnt(vmcnt_imm(4 * kLoads)); break;
            case 3: __builtin_amdgcn_s_waitcnt(vmcnt_imm(3 * kLoads)); break;
            case 2: __builtin_amdgcn_s_waitcnt(vmcnt_imm(2 * kLoads)); break;
            case 1: __builtin_amdgcn_s_waitcnt(vmcnt_imm(kLoads)); break;
            default: __builtin_amdgcn_s_waitcnt(vmcnt_imm(0)); break;
        }
        static_assert(kF1Stages - 2 <= 5, "waits listed above");
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_sched_barrier(0);
        if (st + kF1Stages - 1 < steps) issue(st + kF1Stages - 1);
        const char* sa = stage_a(st % kF1Stages);
        const char* sb = stage_b(st % kF1Stages);
        bf16x8 a[4], b[4];
        for (int i = 0; i < 4; ++i) a[i] = frag(sa, wm * 64 + i * 16 + r, q);
        for (int j = 0; j < 4; ++j) b[j] = frag(sb, wn * 64 + j * 16 + r, q);
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            const int n = wn * 64 + j * 16 + r;
            const float bn = bias[n];
            const int mb = m0 + wm * 64 + i * 16 + q * 4;
            for (int e = 0; e < 4; ++e)
                if (mb + e < M) out[(int64_t)(mb + e) * kF1BN + n] = f2bf(fmaxf(acc[i][j][e] + bn, 0.0f));
        }
}

// Output layer for inference: one thread per input, same summation order as
// k_head.
template <class P>
__global__ __launch_bounds__(256) void k_head_infer(const typename P::T* __restrict__ h2, int B,
                                                    const float* __restrict__ w3,
                                                    const float* __restrict__ b3,
                                                    float* __restrict__ logits) {
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= B) return;
    float z = b3[0];
    for (int i = 0; i < 64; ++i) z += P::to_f(h2[(int64_t)b * 64 + i]) * w3[i];
    logits[b] = z;
}

// Route a pooled-level gradient to the pre-activation positions with the
// forward mask: dpre[b][x][c] = dact[b][x/2][c] if x is the winner and its
// pre-activation was > 0, else 0.
template <class P>
__global__ __launch_bounds__(256) void k_unpool(const typename P::T* __restrict__ dact,
                                                const uint8_t* __restrict__ mask, int64_t npool,
                                                int C, typename P::T* __restrict__ dpre) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;   // pooled index (b, xp, c)
    if (i >= npool) return;
    const int c = (int)(i % C);
    const int64_t bx = i / C;                                      // b * Lp + xp
    const uint8_t mk = mask[i];
    const typename P::T g = (mk & 2) ? dact[i] : P::from_f(0.0f);
    const typename P::T z = P::from_f(0.0f);
    dpre[(2 * bx + (mk & 1)) * C + c] = g;
    dpre[(2 * bx + 1 - (mk & 1)) * C + c] = z;
}

// Bias gradient: g[o] = sum over rows of d[row][o] (rows x C, FP32 out).
// Block (c-group, part): 256 threads = 256 / C' row lanes x C' channels
// (C' = min(C, 64) consecutive channels, coalesced), rows split over
// gridDim.y parts; each part writes its sums to part_out[part][c], summed in
// part order by k_sum_parts (deterministic).
template <class P>
__global__ __launch_bounds__(256) void k_bias_grad(const typename P::T* __restrict__ d, int64_t rows,
                                                   int C, float* __restrict__ part_out) {
    __shared__ float red[256];
    const int cg = C < 64 ? C : 64;                  // channels per block
    const int lanes = 256 / cg;                      // row lanes per block
    const int c = blockIdx.x * cg + threadIdx.x % cg;
    const int rl = threadIdx.x / cg;
    const int64_t per = (rows + gridDim.y - 1) / gridDim.y;
    const int64_t r0 = (int64_t)blockIdx.y * per, r1 = min(rows, r0 + per);
    float s = 0.0f;
    if (rl < lanes)
        for (int64_t r = r0 + rl; r < r1; r += lanes) s += P::to_f(d[r * C + c]);
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < cg) {
        float t = 0.0f;
        for (int j = 0; j < lanes; ++j) t += red[j * cg + threadIdx.x];
        part_out[(int64_t)blockIdx.y * C + c] = t;
    }
}

// out[i] = sum_p parts[p][i] for p = 0 .. nparts-1, one wave per output in
// a fixed order (wave_sum_parts): deterministic. Launch with 4 outputs per
// 256-thread block.
__global__ __launch_bounds__(256) void k_sum_parts(const float* __restrict__ parts, int nparts, int n,
                                                   float* __restrict__ out) {
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (i >= n) return;
    const float t = wave_sum_parts(parts, nparts, n, i, lane);
    if (lane == 0) out[i] = t;
}

// Conv block 1 weight gradient: dW[co][dx] = sum_{b,x} dpre[b][x][co] x[b][(x+dx-2) mod 256].
// Thread = one position of one part of the batch, all 16 x 5 products at
// once (the 16 channel gradients are 32 contiguous bytes); the block's 80
// sums are reduced in LDS and written to part_out[part][co*5+dx], summed in
// part order by k_sum_parts.
template <class P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_conv1_dw(
    const typename P::T* __restrict__ dpre,
                                                  const void* __restrict__ x, int xf32, int B,
                                                  float* __restrict__ part_out) {
    __shared__ float red[80][33];
    const int64_t total = (int64_t)B * 256;
    const int64_t per = (total + gridDim.x - 1) / gridDim.x;
    const int64_t e0 = (int64_t)blockIdx.x * per, e1 = min(total, e0 + per);
    float acc[80];
    for (int j = 0; j < 80; ++j) acc[j] = 0.0f;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
        const int b = (int)(e >> 8), xx = (int)(e & 255);
        float xv[5];
        for (int dx = 0; dx < 5; ++dx) {
            const int64_t o = (int64_t)b * 256 + ((xx + dx - 2) & 255);
            const float v = xf32 ? reinterpret_cast<const float*>(x)[o]
                                 : bf2f(reinterpret_cast<const uint16_t*>(x)[o]);
            xv[dx] = P::to_f(P::from_f(v));
        }
        for (int co = 0; co < 16; ++co) {
            const float dv = P::to_f(dpre[e * 16 + co]);
            for (int dx = 0; dx < 5; ++dx) acc[co * 5 + dx] += dv * xv[dx];
        }
    }
    // wave sums, then the block's 4 waves... via LDS columns of 32 (8 threads per slot)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j = 0; j < 80; ++j) {
        float v = acc[j];
        for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d);
        if (lane == 0) red[j][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x < 80) {
        float t = 0.0f;
        for (int w = 0; w < 4; ++w) t += red[threadIdx.x][w];
        part_out[(int64_t)blockIdx.x * 80 + threadIdx.x] = t;
    }
}

// ------------------------------------------------------------------ fused backward of the convolution blocks (bf16)
//
// Data gradients, one kernel per block (k_convT_bf16): one wave per input
// unpools the block's pooled gradient with its mask into LDS, runs the
// transposed circular convolution on MFMA with the backward weights (k in the
// same 32-steps as k_gemm with ConvRows and sgn -1, rounded as EpStore
// rounds: the result is bit-identical to the layer path) and writes the
// result, the pooled gradient of the block below, to HBM, where the block's
// weight gradient and the next kernel read it. LDS layouts as in the forward
// stack: unpooled gradients in rows of their exact length with the act_off
// chunk swizzle; backward weights [Cin][5 Cout] in rows padded to a stride of
// 32 mod 64 bytes.
constexpr int kB4Ld = 336, kB3Ld = 336, kB2Ld = 176;  // rows of the backward weights

// The transposed conv of one input by one wave. dpre [L][PLD = COUT]
// (act_off rows): gradient at the block's COUT pre-activations; w
// [CIN][WLD]: backward weights, k = dx*COUT + co. Output (x, ci) = sum_k
// dpre[(x - dx + 2) mod L][co] w[ci][k], rounded to bf16, stored to gout
// [L][CIN]. The MFMA takes the weights as its first operand, so a lane ends
// with 4 consecutive channels of one position (8-byte stores); the products
// and their k order are those of k_gemm with ConvRows (sgn -1), whose output
// is the transpose.
template <int L, int CIN, int COUT, int PLD, int WLD, int RB, int CB>
__device__ __forceinline__ void convT_one(const uint16_t* __restrict__ dpre, const uint16_t* __restrict__ w,
                                          uint16_t* __restrict__ gout) {
    constexpr int K = 5 * COUT;
    static_assert(K % 32 == 0 && COUT % 8 == 0, "k steps within one dx");
    constexpr int KSTEPS = K / 32;
    constexpr int NRT = L / (16 * RB), NCT = CIN / (16 * CB);
    static_assert(NRT * 16 * RB == L && NCT * 16 * CB == CIN, "tiles cover the output");
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, q = lane >> 4;
    for (int t = 0; t < NRT * NCT; ++t) {
        const int rt = t / NCT, ct = t - rt * NCT;
        f32x4 acc[CB][RB];
        for (int j = 0; j < CB; ++j)
            for (int i = 0; i < RB; ++i) acc[j][i] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < KSTEPS; ++ks) {
            const int k = ks * 32 + q * 8;
            const int dx = k / COUT, c0 = k - dx * COUT;
            bf16x8 a[RB], b[CB];
            for (int i = 0; i < RB; ++i) {
                int pos = rt * 16 * RB + i * 16 + r - dx + 2;
                pos = pos < 0 ? pos + L : (pos >= L ? pos - L : pos);
                a[i] = *reinterpret_cast<const bf16x8*>(dpre + act_off<PLD>(pos, c0));
            }
            for (int j = 0; j < CB; ++j)
                b[j] = *reinterpret_cast<const bf16x8*>(w + (ct * 16 * CB + j * 16 + r) * WLD + k);
            for (int j = 0; j < CB; ++j)
                for (int i = 0; i < RB; ++i)
                    acc[j][i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[j], a[i], acc[j][i], 0, 0, 0);
        }
        for (int j = 0; j < CB; ++j) {
            const int n0 = ct * 16 * CB + j * 16 + q * 4;   // 4 channels n0 .. n0 + 3
            for (int i = 0; i < RB; ++i) {
                const int xx = rt * 16 * RB + i * 16 + r;
                *reinterpret_cast<uint2*>(gout + xx * CIN + n0) =
                    make_uint2(f2bf2(acc[j][i][0], acc[j][i][1]), f2bf2(acc[j][i][2], acc[j][i][3]));
            }
        }
    }
}

// Unpool 8 channels of one pooled position: g = 8 bf16 gradients, k = their
// 8 mask bytes; e0 / e1 receive the values at the even / odd position.
__device__ __forceinline__ void unpool8(uint4 g, uint2 k, uint4& e0, uint4& e1) {
    const uint32_t gv[4] = {g.x, g.y, g.z, g.w};
    uint32_t r0[4], r1[4];
    for (int j = 0; j < 4; ++j) {
        const uint32_t kb = (j < 2 ? k.x : k.y) >> (16 * (j & 1));
        const uint32_t ma = kb & 3u, mb = (kb >> 8) & 3u;
        const uint32_t lo = gv[j] & 0xffffu, hi = gv[j] & 0xffff0000u;
        r0[j] = (ma == 2u ? lo : 0u) | (mb == 2u ? hi : 0u);
        r1[j] = (ma == 3u ? lo : 0u) | (mb == 3u ? hi : 0u);
    }
    e0 = make_uint4(r0[0], r0[1], r0[2], r0[3]);
    e1 = make_uint4(r1[0], r1[1], r1[2], r1[3]);
}

// One block's data gradient: each kernel holds only its block's backward
// weights and one unpooled gradient per wave (4-8 KB), 16 waves per CU (a
// single kernel for all three blocks held all their weights and 18 KB per
// wave: 5 waves). d [B][LP][COUT], m [B][LP][COUT] (pooled gradient and mask
// of the block's output) -> dout [B][2 LP][CIN] (pooled gradient of the
// block below).
constexpr int kTW = 16;   // waves per block
// Block 2's kernel (C1 = 1: bf16 input, 2: FP32 input) also takes the
// weight and bias gradients of conv block 1, whose pre-activation gradient is
// its output (the pooled gradient of block 1) unpooled with block 1's mask:
// per input an MFMA product G[16 ch][256 positions] x X[256][16], X[p][dx] =
// x[(p + dx - 2) mod 256] for dx < 5, 1 in column 5 (the bias), 0 beyond;
// G goes to the wave's LDS slice transposed (channel rows of 528 bytes:
// conflict-free writes, fragment reads with at most 2 lanes per bank) and
// x as two copies offset by one element, so every lane's 8-position window
// is 4-byte aligned. A wave adds its inputs' products in order; the block
// sums its waves in order into part_out[block][co*5+dx, then 80+co], added
// up in block order with the other blocks' rows (k_dw_seg, k_dw_final). The
// block-1 gradient itself is not written.
constexpr int kXsDw = 136;   // dwords per x copy (268 elements used)
template <int LP, int COUT, int CIN, int WLD, int RB, int CB, int C1>
struct ConvTLds {
    uint16_t w[CIN * WLD];
    uint16_t dp[kTW][2 * LP * COUT + (C1 ? 128 : 0)];   // unpooled gradient [2 LP][COUT] (act_off rows)
    uint32_t xs[C1 ? kTW : 1][2][kXsDw];
};

template <int LP, int COUT, int CIN, int WLD, int RB, int CB, int C1 = 0>
__global__ __launch_bounds__(kTW * 64, 1) void k_convT_bf16(int B, const uint16_t* __restrict__ wb,
                                                        const uint16_t* __restrict__ d,
                                                        const uint8_t* __restrict__ m,
                                                        uint16_t* __restrict__ dout,
                                                        const uint8_t* __restrict__ m1 = nullptr,
                                                        const void* __restrict__ x = nullptr,
                                                        float* __restrict__ part_out = nullptr) {
    constexpr int L = 2 * LP, K = 5 * COUT, E = LP * COUT, U = E / 512;   // 8 values per lane and unit
    static_assert(E % 512 == 0 && sizeof(ConvTLds<LP, COUT, CIN, WLD, RB, CB, C1>) <= 160 * 1024, "shapes");
    static_assert(!C1 || (L == 128 && CIN == 16 && RB == 8 && CB == 1), "block-1 gradient: block 2's shape");
    __shared__ __attribute__((aligned(16))) ConvTLds<LP, COUT, CIN, WLD, RB, CB, C1> sm;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, q = lane >> 4;
    for (int i = tid; i < CIN * WLD; i += kTW * 64) {
        const int n = i / WLD, k = i - n * WLD;
        sm.w[i] = k < K ? wb[n * K + k] : (uint16_t)0;
    }
    __syncthreads();   // weights staged
    uint16_t* dp = sm.dp[wave];
    const int64_t stride = (int64_t)gridDim.x * kTW;
    int64_t fi = (int64_t)blockIdx.x * kTW + wave;
    uint4 ng[U];
    uint2 nk[U];
    // block 1: the input (4 positions per lane) and the mask words (tile i:
    // position 16 i + r, channels 4q .. 4q + 3)
    uint32_t nx[2], nm1[C1 ? 8 : 1];
    auto load = [&](int64_t f) {   // (unconditional: past the batch, read again and never used)
        f = f < B ? f : B - 1;
        for (int h = 0; h < U; ++h) {
            ng[h] = ld_u4(d + f * E + h * 512 + lane * 8);
            nk[h] = *reinterpret_cast<const uint2*>(m + f * E + h * 512 + lane * 8);
        }
        if constexpr (C1 != 0) {
            for (int i = 0; i < 8; ++i)
                nm1[i] = *reinterpret_cast<const uint32_t*>(m1 + f * 2048 + (16 * i + r) * 16 + 4 * q);
            if constexpr (C1 == 2) {
                const float4 v =
                    *reinterpret_cast<const float4*>(reinterpret_cast<const float*>(x) + f * 256 + lane * 4);
                nx[0] = f2bf2(v.x, v.y);
                nx[1] = f2bf2(v.z, v.w);
            } else {
                const uint2 v =
                    *reinterpret_cast<const uint2*>(reinterpret_cast<const uint16_t*>(x) + f * 256 + lane * 4);
                nx[0] = v.x;
                nx[1] = v.y;
            }
        }
    };
    f32x4 g1 = f32x4{0.0f, 0.0f, 0.0f, 0.0f};   // block 1: D[ch 4q..4q+3][column r]
    load(fi);
    for (; fi < B; fi += stride) {
        for (int h = 0; h < U; ++h) {
            const int e0 = h * 512 + lane * 8, xp = e0 / COUT, c0 = e0 - xp * COUT;
            uint4 ev, od;
            unpool8(ng[h], nk[h], ev, od);
            *reinterpret_cast<uint4*>(dp + act_off<COUT>(2 * xp, c0)) = ev;
            *reinterpret_cast<uint4*>(dp + act_off<COUT>(2 * xp + 1, c0)) = od;
        }
        if constexpr (C1 == 0) {
            __builtin_amdgcn_sched_barrier(0);
            load(fi + stride);
            wave_lds_sync();
            convT_one<L, CIN, COUT, COUT, WLD, RB, CB>(dp, sm.w, dout + fi * (L * CIN));
        } else {
            const uint32_t cx0 = nx[0], cx1 = nx[1];
            uint32_t cm1[8];
            for (int i = 0; i < 8; ++i) cm1[i] = nm1[i];
            // the lane's row and group, copied each input through an opaque move so
            // that the LDS offsets below are worked out here, not held in
            // registers across the loop
            int r, q;
            asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "v"(lane & 15));
            asm volatile("v_mov_b32 %0, %1" : "=v"(q) : "v"(lane >> 4));
            // x copies: xs[0][j] = x[(j - 4) mod 256], xs[1][j] = x[(j - 3) mod 256];
            // lane l holds x[4l .. 4l + 3] and writes both copies' words 2l + 2, 2l + 3
            // (lane 63 also words 0, 1 and lanes 0, 1 words 130 .. 133: the wrap)
            {
                const uint32_t nwx = __shfl(cx0, (lane + 1) & 63);   // x[4l + 4], x[4l + 5]
                const uint2 c0v = make_uint2(cx0, cx1);
                const uint2 c1v = make_uint2((cx0 >> 16) | (cx1 << 16), (cx1 >> 16) | (nwx << 16));
                uint32_t* x0 = sm.xs[C1 ? wave : 0][0];
                uint32_t* x1 = sm.xs[C1 ? wave : 0][1];
                *reinterpret_cast<uint2*>(x0 + 2 * lane + 2) = c0v;
                *reinterpret_cast<uint2*>(x1 + 2 * lane + 2) = c1v;
                if (lane == 63) {
                    *reinterpret_cast<uint2*>(x0) = c0v;
                    *reinterpret_cast<uint2*>(x1) = c1v;
                }
                if (lane < 2) {
                    *reinterpret_cast<uint2*>(x0 + 130 + 2 * lane) = c0v;
                    *reinterpret_cast<uint2*>(x1 + 130 + 2 * lane) = c1v;
                }
            }
            __builtin_amdgcn_sched_barrier(0);
            load(fi + stride);
            wave_lds_sync();
            // the data gradient as convT_one computes it (same products in the
            // same order), in two halves of 4 row tiles so that fewer
            // accumulators and operands are live; kept as bf16 pairs
            uint32_t pk[8][2];   // tile i: channels (4q, 4q + 1), (4q + 2, 4q + 3) at position 16 i + r
            for (int h = 0; h < 2; ++h) {
                f32x4 acc[4];
                for (int i = 0; i < 4; ++i) acc[i] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int ks = 0; ks < K / 32; ++ks) {
                    const int k = ks * 32 + q * 8;
                    const int dx = k / COUT, c0 = k - dx * COUT;
                    bf16x8 a[4];
                    for (int i = 0; i < 4; ++i) {
                        int pos = (4 * h + i) * 16 + r - dx + 2;
                        pos = pos < 0 ? pos + L : (pos >= L ? pos - L : pos);
                        a[i] = *reinterpret_cast<const bf16x8*>(dp + act_off<COUT>(pos, c0));
                    }
                    const bf16x8 b = *reinterpret_cast<const bf16x8*>(sm.w + r * WLD + k);
                    for (int i = 0; i < 4; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b, a[i], acc[i], 0, 0, 0);
                }
                for (int i = 0; i < 4; ++i) {
                    pk[4 * h + i][0] = f2bf2(acc[i][0], acc[i][1]);
                    pk[4 * h + i][1] = f2bf2(acc[i][2], acc[i][3]);
                }
            }
            wave_lds_sync();   // the wave's reads of dp are done
            // block 1's pre-activation gradient, transposed: row ch (132 words)
            // holds 256 positions; word pos of a row is pooled position pos
            // (its even and odd position)
            uint32_t* gt = reinterpret_cast<uint32_t*>(dp);
            for (int i = 0; i < 8; ++i) {
                const uint32_t v01 = pk[i][0], v23 = pk[i][1];
                const int pos = 16 * i + r;
                for (int e = 0; e < 4; ++e) {
                    const int ch = 4 * q + e;
                    const uint32_t g = ((e < 2 ? v01 : v23) >> (16 * (e & 1))) & 0xffffu;
                    const uint32_t mb = (cm1[i] >> (8 * e)) & 3u;
                    const uint32_t wv = (mb & 2u) ? ((mb & 1u) ? g << 16 : g) : 0u;
                    gt[ch * 132 + pos] = wv;
                }
            }
            wave_lds_sync();
            const uint32_t* xsw = sm.xs[C1 ? wave : 0][0];
            const int nn = r < 4 ? r : 4, dl = nn - 2, par = dl & 1;
            for (int st = 0; st < 8; ++st) {
                // row r, positions 32 st + 8 q .. + 7
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(gt + r * 132 + 16 * st + 4 * q);
                const int j0 = 32 * st + 8 * q + dl + 4 - par;   // even
                const uint32_t* xw = xsw + par * kXsDw + (j0 >> 1);
                uint32_t bw[4] = {xw[0], xw[1], xw[2], xw[3]};
                for (int t = 0; t < 4; ++t) bw[t] = r < 5 ? bw[t] : (r == 5 ? 0x3F803F80u : 0u);
                const bf16x8 b = __builtin_bit_cast(bf16x8, make_uint4(bw[0], bw[1], bw[2], bw[3]));
                g1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, g1, 0, 0, 0);
            }
        }
        wave_lds_sync();   // dp is reused by the next input
    }
    if constexpr (C1 != 0) {
        // the block's waves in order (the wave tiles go where the gradients were)
        __syncthreads();
        float* red = reinterpret_cast<float*>(&sm.dp[0][0]);
        for (int e = 0; e < 4; ++e) red[wave * 256 + (4 * q + e) * 16 + r] = g1[e];
        __syncthreads();
        if (tid < 96) {
            const int ch = tid < 80 ? tid / 5 : tid - 80, col = tid < 80 ? tid - 5 * ch : 5;
            float t = 0.0f;
            for (int w = 0; w < kTW; ++w) t += red[w * 256 + ch * 16 + col];
            part_out[(int64_t)blockIdx.x * 96 + tid] = t;
        }
    }
}

// Weight and bias gradients of conv block l = 2 .. 4 (bf16). The batch is cut
// into groups of 8 inputs and each block takes a contiguous range of groups.
// An item is 32 output positions of one group: the gradient at the block's
// pre-activations there (its pooled gradient unpooled with the mask) and the
// block's input at those positions -2 .. +2, staged in LDS with the 8 inputs
// innermost ([position][channel][8]), so that an MFMA k-step is 4 positions x
// 8 inputs and every operand fragment is one aligned 16-byte read. Channel
// slots are XOR-swizzled within groups of 8 by the position, which keeps both
// the transposing writes and the fragment reads free of most bank conflicts.
// In k_conv_dw_bf16 a block of 4 waves stages an item, then runs its MFMAs
// (several blocks per CU overlap one's loads with another's matrix work).
// The waves split the output columns (n = dx*CIN + ci) in WN parts and the
// k-steps in WK; each block writes one row of FP32 sums to part_out:
// [COUT][5 CIN] weight sums, then COUT bias sums; the rows are added up in
// block order (deterministic).
__device__ __forceinline__ int dw_slot(int pos, int c, int C) {
    return pos * C + (c ^ (((c >> 3) + pos) & 7));
}

// out[j] = channel j of the 8 inputs in v (v[s] = 8 channels of input s).
__device__ __forceinline__ uint4 tr8(const uint4 (&v)[8], int j) {
    uint32_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t a = (&v[2 * k].x)[j >> 1], b = (&v[2 * k + 1].x)[j >> 1];
        w[k] = (j & 1) ? ((a >> 16) | (b & 0xffff0000u)) : ((a & 0xffffu) | (b << 16));
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
}

template <int L, int CIN, int COUT, int WN, int WK>
struct DwShape {
    static constexpr int MT = COUT / 16, NT = 5 * CIN / 16, NTW = NT / WN;
    static constexpr int DQ = 32 * COUT * 8, AQ = 36 * CIN * 8;           // bf16 elements
    static constexpr int RED = (WK - 1) * WN * MT * NTW * 256;            // floats
    static constexpr int STAGE = 2 * (DQ + AQ), REDB = 4 * RED, DBB = 4 * 256 * 4;
    static constexpr int BYTES = STAGE > REDB ? (STAGE > DBB ? STAGE : DBB) : (REDB > DBB ? REDB : DBB);
};

template <int L, int CIN, int COUT, int WN, int WK>
__global__ __launch_bounds__(256, CIN == 16 ? 3 : 2) void k_conv_dw_bf16(int B, int groups_per_block,
                                                         const uint16_t* __restrict__ dact,
                                                         const uint8_t* __restrict__ mask,
                                                         const uint16_t* __restrict__ act,
                                                         float* __restrict__ part_out) {
    using S = DwShape<L, CIN, COUT, WN, WK>;
    constexpr int MT = S::MT, NTW = S::NTW;
    constexpr int NA = 36 * (CIN / 8), ND = 16 * (COUT / 4);   // staging units per chunk
    static_assert(NA <= 256 && ND <= 256, "one unit of each kind per thread");
    // CIN 32: both units' loads issued together (two blocks per CU); CIN 16:
    // one unit after the other, in the registers three blocks per CU allow
    constexpr bool kHoist = CIN == 32;
    static_assert(WN * WK == 4 && S::NT % WN == 0, "wave split");
    static_assert(L % 32 == 0 && CIN % 16 == 0 && COUT % 16 == 0, "tile shapes");
    __shared__ __attribute__((aligned(16))) uint8_t smem[S::BYTES];
    uint16_t* dq = reinterpret_cast<uint16_t*>(smem);
    uint16_t* aq = dq + S::DQ;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, q = lane >> 4;
    const int nw = wave % WN, kw = wave / WN;
    f32x4 acc[MT][NTW];
    for (int i = 0; i < MT; ++i)
        for (int j = 0; j < NTW; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float db[4] = {0, 0, 0, 0};
    // byte offsets of the lane's A and B fragments for k-steps kw and kw + WK
    int abase[2][MT], bbase[2][NTW];
    for (int hm = 0; hm < 2; ++hm) {
        const int p = (kw + hm * WK) * 4 + q;   // position within the chunk
        for (int i = 0; i < MT; ++i) abase[hm][i] = dw_slot(p, i * 16 + r, COUT) * 16;
        for (int j = 0; j < NTW; ++j) {
            const int n = (nw * NTW + j) * 16 + r;
            const int dx = n / CIN, ci = n - dx * CIN;
            bbase[hm][j] = S::DQ * 2 + dw_slot(p + dx, ci, CIN) * 16;
        }
    }
    const int ngroups = (B + 7) / 8;
    const int g0 = blockIdx.x * groups_per_block;
    const int g1 = min(ngroups, g0 + groups_per_block);
#pragma unroll 1
    for (int g = g0; g < g1; ++g) {
#pragma unroll 1
        for (int c = 0; c < L / 32; ++c) {
            if constexpr (kHoist) {
                // a thread has at most one input unit (8 inputs x 8 channels at
                // one of positions c*32 - 2 ... c*32 + 33, circular) and one
                // gradient unit (8 inputs x 4 channels of one pooled position);
                // both are loaded before either is used (indices past the units
                // or the batch are clamped and their values dropped), so one
                // memory latency is paid per chunk
                const int ta = min(tid, NA - 1), td = min(tid, ND - 1);
                const int pi = ta / (CIN / 8), cg = ta - pi * (CIN / 8);
                int pos = c * 32 + pi - 2;
                pos = pos < 0 ? pos + L : (pos >= L ? pos - L : pos);
                const int xi = td / (COUT / 4), og = td - xi * (COUT / 4);
                uint4 v[8];
                uint2 gv[8];
                uint32_t kv[8];
    #pragma unroll
                for (int s = 0; s < 8; ++s) {
                    const int64_t b = min<int64_t>((int64_t)g * 8 + s, B - 1);
                    v[s] = *reinterpret_cast<const uint4*>(act + (b * L + pos) * CIN + cg * 8);
                    const int64_t o = (b * (L / 2) + c * 16 + xi) * COUT + og * 4;
                    gv[s] = *reinterpret_cast<const uint2*>(dact + o);
                    kv[s] = *reinterpret_cast<const uint32_t*>(mask + o);
                }
                const int nval = (int)min<int64_t>(8, (int64_t)B - (int64_t)g * 8);
    #pragma unroll
                for (int s = 0; s < 8; ++s)
                    if (s >= nval) {
                        v[s] = make_uint4(0u, 0u, 0u, 0u);
                        kv[s] = 0u;   // a zero mask keeps nothing
                    }
                __syncthreads();   // the previous chunk's fragments are read
                if (tid < NA)
    #pragma unroll
                    for (int j = 0; j < 8; ++j)
                        *reinterpret_cast<uint4*>(aq + dw_slot(pi, cg * 8 + j, CIN) * 8) = tr8(v, j);
                // gradient at pre-activation positions c*32 ... c*32 + 31: the
                // even positions' values are formed and stored, then the odd ones'
                if (tid < ND) {
    #pragma unroll
                    for (int s = 0; s < 8; ++s)
    #pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const uint32_t h = (j < 2 ? gv[s].x : gv[s].y) >> (16 * (j & 1));
                            db[j] += (kv[s] >> (8 * j) & 2u) ? bf2f((uint16_t)h) : 0.0f;
                        }
    #pragma unroll
                    for (int par = 0; par < 2; ++par) {
                        const uint32_t sel = 2u | (uint32_t)par;
                        uint32_t e[8][4];
    #pragma unroll
                        for (int s = 0; s < 8; ++s)
    #pragma unroll
                            for (int j = 0; j < 4; ++j) {
                                const uint32_t h = ((j < 2 ? gv[s].x : gv[s].y) >> (16 * (j & 1))) & 0xffffu;
                                e[s][j] = ((kv[s] >> (8 * j)) & 3u) == sel ? h : 0u;
                            }
    #pragma unroll
                        for (int j = 0; j < 4; ++j)
                            *reinterpret_cast<uint4*>(dq + dw_slot(2 * xi + par, og * 4 + j, COUT) * 8) =
                                make_uint4(e[0][j] | (e[1][j] << 16), e[2][j] | (e[3][j] << 16),
                                           e[4][j] | (e[5][j] << 16), e[6][j] | (e[7][j] << 16));
                    }
                }
            } else {
                __syncthreads();   // the previous chunk's fragments are read
                // input positions c*32 - 2 ... c*32 + 33 (circular)
    #pragma unroll 1
                for (int t = tid; t < 36 * (CIN / 8); t += 256) {
                    const int pi = t / (CIN / 8), cg = t - pi * (CIN / 8);
                    int pos = c * 32 + pi - 2;
                    pos = pos < 0 ? pos + L : (pos >= L ? pos - L : pos);
                    uint4 v[8];
                    for (int s = 0; s < 8; ++s) {
                        const int64_t b = (int64_t)g * 8 + s;
                        v[s] = b < B ? *reinterpret_cast<const uint4*>(act + (b * L + pos) * CIN + cg * 8)
                                     : make_uint4(0u, 0u, 0u, 0u);
                    }
    #pragma unroll
                    for (int j = 0; j < 8; ++j)
                        *reinterpret_cast<uint4*>(aq + dw_slot(pi, cg * 8 + j, CIN) * 8) = tr8(v, j);
                }
                // gradient at pre-activation positions c*32 ... c*32 + 31, 4
                // channels of one pooled position per task: the even positions'
                // values are formed and stored, then the odd ones'
    #pragma unroll 1
                for (int t = tid; t < 16 * (COUT / 4); t += 256) {
                    const int xi = t / (COUT / 4), og = t - xi * (COUT / 4);
                    const int xp = c * 16 + xi;
                    uint2 gv[8];
                    uint32_t kv[8];
    #pragma unroll
                    for (int s = 0; s < 8; ++s) {
                        const int64_t b = (int64_t)g * 8 + s;
                        gv[s] = make_uint2(0u, 0u);
                        kv[s] = 0u;
                        if (b < B) {
                            const int64_t o = (b * (L / 2) + xp) * COUT + og * 4;
                            gv[s] = *reinterpret_cast<const uint2*>(dact + o);
                            kv[s] = *reinterpret_cast<const uint32_t*>(mask + o);
                        }
                    }
    #pragma unroll
                    for (int s = 0; s < 8; ++s)
    #pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const uint32_t h = (j < 2 ? gv[s].x : gv[s].y) >> (16 * (j & 1));
                            db[j] += (kv[s] >> (8 * j) & 2u) ? bf2f((uint16_t)h) : 0.0f;
                        }
    #pragma unroll
                    for (int par = 0; par < 2; ++par) {
                        const uint32_t sel = 2u | (uint32_t)par;
                        uint32_t e[8][4];
    #pragma unroll
                        for (int s = 0; s < 8; ++s)
    #pragma unroll
                            for (int j = 0; j < 4; ++j) {
                                const uint32_t h = ((j < 2 ? gv[s].x : gv[s].y) >> (16 * (j & 1))) & 0xffffu;
                                e[s][j] = ((kv[s] >> (8 * j)) & 3u) == sel ? h : 0u;
                            }
    #pragma unroll
                        for (int j = 0; j < 4; ++j)
                            *reinterpret_cast<uint4*>(dq + dw_slot(2 * xi + par, og * 4 + j, COUT) * 8) =
                                make_uint4(e[0][j] | (e[1][j] << 16), e[2][j] | (e[3][j] << 16),
                                           e[4][j] | (e[5][j] << 16), e[6][j] | (e[7][j] << 16));
                    }
                }
            }
            __syncthreads();
            // wave kw takes k-steps kw + m*WK (4 positions each); steps m and
            // m + 2 are 8*WK positions apart and use the same swizzle, so the
            // fragment addresses are two per-lane bases plus constant offsets
#pragma unroll 2
            for (int m = 0; m < 8 / WK; ++m) {
                const int hm = m & 1, step = (m >> 1) * 8 * WK * 16;   // 8 WK positions, 16 bytes a slot
                bf16x8 a[MT], bb[NTW];
                for (int i = 0; i < MT; ++i)
                    a[i] = *reinterpret_cast<const bf16x8*>(smem + abase[hm][i] + step * COUT);
                for (int j = 0; j < NTW; ++j)
                    bb[j] = *reinterpret_cast<const bf16x8*>(smem + bbase[hm][j] + step * CIN);
                for (int i = 0; i < MT; ++i)
                    for (int j = 0; j < NTW; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bb[j], acc[i][j], 0, 0, 0);
            }
        }
    }
    __syncthreads();   // staging space becomes reduction space
    float* red = reinterpret_cast<float*>(smem);
    constexpr int TILES = MT * NTW;
    if constexpr (WK > 1) {
        if (kw > 0)
            for (int i = 0; i < MT; ++i)
                for (int j = 0; j < NTW; ++j)
                    for (int e = 0; e < 4; ++e)
                        red[(((kw - 1) * WN + nw) * TILES + i * NTW + j) * 256 + e * 64 + lane] = acc[i][j][e];
        __syncthreads();
    }
    if (kw == 0) {
        float* out = part_out + (int64_t)blockIdx.x * (COUT * (5 * CIN) + COUT);
        for (int i = 0; i < MT; ++i)
            for (int j = 0; j < NTW; ++j)
                for (int e = 0; e < 4; ++e) {
                    float v = acc[i][j][e];
                    for (int z = 1; z < WK; ++z) v += red[(((z - 1) * WN + nw) * TILES + i * NTW + j) * 256 + e * 64 + lane];
                    const int m = i * 16 + q * 4 + e, n = (nw * NTW + j) * 16 + r;
                    out[m * (5 * CIN) + n] = v;
                }
    }
    __syncthreads();
    for (int j = 0; j < 4; ++j) red[tid * 4 + j] = db[j];
    __syncthreads();
    if (tid < COUT) {
        const int og = tid >> 2, j = tid & 3;
        float s = 0.0f;
        for (int t = og; t < 256; t += COUT / 4) s += red[t * 4 + j];
        part_out[(int64_t)blockIdx.x * (COUT * (5 * CIN) + COUT) + COUT * (5 * CIN) + tid] = s;
    }
}

// k_conv_dw_pipe_bf16: the same items, sums and output rows, with a block of
// 8 waves: waves 4-7 stage item i + 1 into one of two LDS stages (its loads
// issued while item i - 1's matrix work runs) while waves 0-3 run item i's
// MFMAs on the other, one barrier per item; the bias sums are formed by the
// staging waves.
template <int L, int CIN, int COUT, int WN, int WK>
struct DwPipeShape {
    static constexpr int MT = COUT / 16, NT = 5 * CIN / 16, NTW = NT / WN;
    static constexpr int DQ = 32 * COUT * 8, AQ = 36 * CIN * 8;           // bf16 elements per stage
    static constexpr int STAGE = 2 * (DQ + AQ);                          // bytes per stage
    static constexpr int RED = (WK - 1) * WN * MT * NTW * 256;            // floats
    static constexpr int REDB = 4 * RED, DBB = 4 * 256 * 4;
    static constexpr int BYTES = 2 * STAGE > REDB ? (2 * STAGE > DBB ? 2 * STAGE : DBB) : (REDB > DBB ? REDB : DBB);
    // staging units per item: input positions -2 .. 33 of the item (for a
    // 32-position block, whose one item wraps around, its 32 positions, each
    // also written to the halo slots it lands in); gradient units
    static constexpr bool WRAP = L == 32;
    static constexpr int NA = (WRAP ? 32 : 36) * (CIN / 8), ND = 16 * (COUT / 4);
    static constexpr int UA = (NA + 255) / 256, UD = (ND + 255) / 256;    // per staging thread
};

template <int L, int CIN, int COUT, int WN, int WK>
__global__ __launch_bounds__(512, 1) void k_conv_dw_pipe_bf16(
    int B, int groups_per_block, const uint16_t* __restrict__ dact, const uint8_t* __restrict__ mask,
    const uint16_t* __restrict__ act, float* __restrict__ part_out) {
    using S = DwPipeShape<L, CIN, COUT, WN, WK>;
    constexpr int MT = S::MT, NTW = S::NTW, CH = L / 32;
    static_assert(WN * WK == 4 && S::NT % WN == 0, "wave split");
    static_assert(L % 32 == 0 && CIN % 16 == 0 && COUT % 16 == 0, "tile shapes");
    __shared__ __attribute__((aligned(16))) uint8_t smem[S::BYTES];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const bool stager = wave >= 4;
    const int st = tid - 256;   // staging thread index
    const int ngroups = (B + 7) / 8;
    const int g0 = blockIdx.x * groups_per_block;
    const int n_it = max(0, min(ngroups, g0 + groups_per_block) - g0) * CH;
    float db[4] = {0, 0, 0, 0};
    // Staging. A thread holds up to UA input units (8 inputs x 8 channels)
    // and UD gradient units (8 inputs x 4 channels) of one item in
    // registers: load() issues every load of item `it` unconditionally
    // (indices past the item's units or the batch are clamped, and their
    // values dropped at use), so the waits count exactly; stage() turns them
    // into item it's LDS stage. The loads of item i + 2 are issued right
    // after item i + 1 is staged, so their latency passes during the matrix
    // work of item i.
    uint4 va[S::UA][8];
    uint2 gv[S::UD][8];
    uint32_t kv[S::UD][8];
    auto load = [&](int it) {
        const int g = g0 + it / CH, c = it - (it / CH) * CH;
#pragma unroll
        for (int u = 0; u < S::UA; ++u) {
            const int t = min(st + u * 256, S::NA - 1);
            const int pi = t / (CIN / 8), cg = t - pi * (CIN / 8);
            int pos = S::WRAP ? pi : c * 32 + pi - 2;
            pos = pos < 0 ? pos + L : (pos >= L ? pos - L : pos);
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const int64_t b = min<int64_t>((int64_t)g * 8 + s, B - 1);
                va[u][s] = *reinterpret_cast<const uint4*>(act + (b * L + pos) * CIN + cg * 8);
            }
        }
#pragma unroll
        for (int u = 0; u < S::UD; ++u) {
            const int t = min(st + u * 256, S::ND - 1);
            const int xi = t / (COUT / 4), og = t - xi * (COUT / 4);
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const int64_t b = min<int64_t>((int64_t)g * 8 + s, B - 1);
                const int64_t o = (b * (L / 2) + c * 16 + xi) * COUT + og * 4;
                gv[u][s] = *reinterpret_cast<const uint2*>(dact + o);
                kv[u][s] = *reinterpret_cast<const uint32_t*>(mask + o);
            }
        }
    };
    auto stage = [&](int it) {
        const int g = g0 + it / CH;
        uint16_t* dq = reinterpret_cast<uint16_t*>(smem + (it & 1) * S::STAGE);
        uint16_t* aq = dq + S::DQ;
        // inputs past the batch contribute zeros
        const int nval = (int)min<int64_t>(8, (int64_t)B - (int64_t)g * 8);
#pragma unroll
        for (int s = 0; s < 8; ++s)
            if (s >= nval) {
#pragma unroll
                for (int u = 0; u < S::UA; ++u) va[u][s] = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
                for (int u = 0; u < S::UD; ++u) kv[u][s] = 0u;
            }
#pragma unroll
        for (int u = 0; u < S::UA; ++u) {
            const int t = st + u * 256;
            if (t < S::NA) {
                const int pi = t / (CIN / 8), cg = t - pi * (CIN / 8);
                if constexpr (S::WRAP) {
                    // position p sits at slot p + 2, and at p + 34 or p - 30
                    // when that is a halo slot (0, 1, 34, 35)
                    const int p2 = pi < 2 ? pi + 34 : (pi >= 30 ? pi - 30 : -1);
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const uint4 w = tr8(va[u], j);
                        *reinterpret_cast<uint4*>(aq + dw_slot(pi + 2, cg * 8 + j, CIN) * 8) = w;
                        if (p2 >= 0) *reinterpret_cast<uint4*>(aq + dw_slot(p2, cg * 8 + j, CIN) * 8) = w;
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < 8; ++j)
                        *reinterpret_cast<uint4*>(aq + dw_slot(pi, cg * 8 + j, CIN) * 8) = tr8(va[u], j);
                }
            }
        }
        // gradient at pre-activation positions c*32 ... c*32 + 31, 4 channels
        // of one pooled position per unit (a zero mask keeps nothing): the
        // even positions' values, then the odd ones'
#pragma unroll
        for (int u = 0; u < S::UD; ++u) {
            const int t = st + u * 256;
            if (t < S::ND) {
                const int xi = t / (COUT / 4), og = t - xi * (COUT / 4);
#pragma unroll
                for (int s = 0; s < 8; ++s)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const uint32_t h = (j < 2 ? gv[u][s].x : gv[u][s].y) >> (16 * (j & 1));
                        db[j] += (kv[u][s] >> (8 * j) & 2u) ? bf2f((uint16_t)h) : 0.0f;
                    }
#pragma unroll
                for (int par = 0; par < 2; ++par) {
                    const uint32_t sel = 2u | (uint32_t)par;
                    uint32_t e[8][4];
#pragma unroll
                    for (int s = 0; s < 8; ++s)
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const uint32_t h = ((j < 2 ? gv[u][s].x : gv[u][s].y) >> (16 * (j & 1))) & 0xffffu;
                            e[s][j] = ((kv[u][s] >> (8 * j)) & 3u) == sel ? h : 0u;
                        }
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        *reinterpret_cast<uint4*>(dq + dw_slot(2 * xi + par, og * 4 + j, COUT) * 8) =
                            make_uint4(e[0][j] | (e[1][j] << 16), e[2][j] | (e[3][j] << 16),
                                       e[4][j] | (e[5][j] << 16), e[6][j] | (e[7][j] << 16));
                }
            }
        }
    };
    f32x4 acc[MT][NTW];
    for (int i = 0; i < MT; ++i)
        for (int j = 0; j < NTW; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const int r = lane & 15, q = lane >> 4;
    const int nw = wave % WN, kw = (wave & 3) / WN;
    // byte offsets (within a stage) of the lane's A and B fragments for
    // k-steps kw and kw + WK
    int abase[2][MT], bbase[2][NTW];
    for (int hm = 0; hm < 2; ++hm) {
        const int p = (kw + hm * WK) * 4 + q;   // position within the item
        for (int i = 0; i < MT; ++i) abase[hm][i] = dw_slot(p, i * 16 + r, COUT) * 16;
        for (int j = 0; j < NTW; ++j) {
            const int n = (nw * NTW + j) * 16 + r;
            const int dx = n / CIN, ci = n - dx * CIN;
            bbase[hm][j] = S::DQ * 2 + dw_slot(p + dx, ci, CIN) * 16;
        }
    }
    if (stager && n_it > 0) {
        load(0);
        stage(0);
        load(min(1, n_it - 1));
    }
    __syncthreads();
#pragma unroll 1
    for (int it = 0; it < n_it; ++it) {
        if (stager) {
            if (it + 1 < n_it) {
                stage(it + 1);
                load(min(it + 2, n_it - 1));   // (past the end: the last item again, never staged)
            }
        } else {
            // wave kw takes k-steps kw + m*WK (4 positions each); steps m and
            // m + 2 are 8*WK positions apart and use the same swizzle, so the
            // fragment addresses are two per-lane bases plus constant offsets
            const uint8_t* stg = smem + (it & 1) * S::STAGE;
#pragma unroll 2
            for (int m = 0; m < 8 / WK; ++m) {
                const int hm = m & 1, step = (m >> 1) * 8 * WK * 16;   // 8 WK positions, 16 bytes a slot
                bf16x8 a[MT], bb[NTW];
                for (int i = 0; i < MT; ++i)
                    a[i] = *reinterpret_cast<const bf16x8*>(stg + abase[hm][i] + step * COUT);
                for (int j = 0; j < NTW; ++j)
                    bb[j] = *reinterpret_cast<const bf16x8*>(stg + bbase[hm][j] + step * CIN);
                for (int i = 0; i < MT; ++i)
                    for (int j = 0; j < NTW; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bb[j], acc[i][j], 0, 0, 0);
            }
        }
        __syncthreads();   // stage it & 1 is free, stage (it + 1) & 1 is full
    }
    // (the stages become reduction space: every wave is past the last barrier)
    float* red = reinterpret_cast<float*>(smem);
    constexpr int TILES = MT * NTW;
    if constexpr (WK > 1) {
        if (!stager && kw > 0)
            for (int i = 0; i < MT; ++i)
                for (int j = 0; j < NTW; ++j)
                    for (int e = 0; e < 4; ++e)
                        red[(((kw - 1) * WN + nw) * TILES + i * NTW + j) * 256 + e * 64 + lane] = acc[i][j][e];
        __syncthreads();
    }
    if (!stager && kw == 0) {
        float* out = part_out + (int64_t)blockIdx.x * (COUT * (5 * CIN) + COUT);
        for (int i = 0; i < MT; ++i)
            for (int j = 0; j < NTW; ++j)
                for (int e = 0; e < 4; ++e) {
                    float v = acc[i][j][e];
                    for (int z = 1; z < WK; ++z) v += red[(((z - 1) * WN + nw) * TILES + i * NTW + j) * 256 + e * 64 + lane];
                    const int m = i * 16 + q * 4 + e, n = (nw * NTW + j) * 16 + r;
                    out[m * (5 * CIN) + n] = v;
                }
    }
    __syncthreads();
    if (stager)
        for (int j = 0; j < 4; ++j) red[st * 4 + j] = db[j];
    __syncthreads();
    if (tid < COUT) {
        const int og = tid >> 2, j = tid & 3;
        float t = 0.0f;
        for (int u = og; u < 256; u += COUT / 4) t += red[u * 4 + j];
        part_out[(int64_t)blockIdx.x * (COUT * (5 * CIN) + COUT) + COUT * (5 * CIN) + tid] = t;
    }
}

// Weight and bias gradients of a dense layer (bf16): C[m][n] = sum_b
// A[b][m] Bt[b][n] and c[m] = sum_b A[b][m] over a range of the batch, with
// A = the output gradient [K][M] and Bt = the layer's input [K][N], both
// row-major with the batch as rows. A block owns a BM x 128 tile and one
// batch range of kc rows; 64 rows at a time are loaded as 8 x 8 units (8
// rows of 16 bytes per thread, one step ahead in registers), transposed in
// registers and stored to LDS as [column][64 rows] (16-byte chunks XOR-
// swizzled by the column), double-buffered so that one barrier per step
// suffices. Blocks of the tiles' first column also sum A's columns (the bias
// gradient), each thread over its 8 rows in order, then over the 8 row
// groups in order. Block z of the batch writes ws[z][M*N + M]: the weight
// sums [M][N], then the bias sums (deterministic; added up in z order by the
// reduction). Blocks are mapped so that the tiles of one batch range share
// an XCD (its L2 holds the range's rows once).
template <int BM>
__global__ __launch_bounds__(256, 2) void k_fc_dw_bf16(int K, int M, int N, int kc, int tiles_n,
                                                       const uint16_t* __restrict__ A,
                                                       const uint16_t* __restrict__ Bt,
                                                       float* __restrict__ ws) {
    constexpr int BN = 128, BK = 64, ROWS = BM + BN;
    constexpr int AU = (BM / 8) * (BK / 8), BU = (BN / 8) * (BK / 8);   // 8 x 8 units per step
    static_assert(AU + BU <= 256, "one unit per thread");
    constexpr int WM = BM / 2, MT = WM / 16, NT = 4;                  // waves 2 x 2, 64 columns each
    __shared__ uint4 lds[2][ROWS * (BK / 8)];
    __shared__ float bred[8][BM];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, q = lane >> 4;
    const int wm = wave >> 1, wn = wave & 1;
    const int nb = gridDim.x, b = blockIdx.x;
    const int logical = (nb & 7) == 0 ? (b & 7) * (nb >> 3) + (b >> 3) : b;
    const int tiles = (M / BM) * tiles_n;
    const int tile = logical % tiles, z = logical / tiles;
    const int mt = tile / tiles_n, nt = tile - mt * tiles_n;
    const int k0 = z * kc, k1 = min(K, k0 + kc);
    // this thread's load unit: 8 rows x 8 columns of A or of Bt
    const bool isA = tid < AU, isB = !isA && tid < AU + BU;
    const int u = isA ? tid : tid - AU;
    const int cg = isA ? u % (BM / 8) : u % (BN / 8), kg = isA ? u / (BM / 8) : u / (BN / 8);
    // (threads without a unit read A's first columns and store nothing)
    const uint16_t* src = isA || !isB ? A + (int64_t)mt * BM + (isA ? cg * 8 : 0) : Bt + (int64_t)nt * BN + cg * 8;
    const int ld = isA || !isB ? M : N;
    const int row0 = isA ? cg * 8 : BM + cg * 8;   // LDS row of this unit's first column
    const bool bias = isA && nt == 0;
    float bsum[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    f32x4 acc[MT][NT];
    for (int i = 0; i < MT; ++i)
        for (int j = 0; j < NT; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    // two register sets: the loads for step st + 2 are issued while step st
    // is computed (about 64 KB in flight per block)
    const int steps = k1 > k0 ? (k1 - k0 + BK - 1) / BK : 0;
    // LDS row `row` keeps its 16-byte chunk c at c ^ swz(row): the fragment
    // reads (16 consecutive rows, one chunk) stay conflict-free and the
    // transposing writes (8 rows apart, one chunk per row group) are 2-way
    auto slot = [](int row, int c) { return row * 8 + (c ^ (((row >> 3) * 2 + (row >> 1) * 2) & 7)); };
    uint4 v0[8], v1[8];
    // loads are unconditional (rows past the range re-read its last row and
    // are zeroed at use), so the wait before a step covers only its own loads
    auto load = [&](uint4 (&v)[8], int st) {
        const int kb = k0 + st * BK;
        for (int s = 0; s < 8; ++s) {
            const int k = min(kb + kg * 8 + s, k1 - 1);
            v[s] = *reinterpret_cast<const uint4*>(src + (int64_t)k * ld);
        }
    };
    auto run_step = [&](uint4 (&v)[8], int st) {
        uint4* buf = lds[st & 1];
        const int kb = k0 + st * BK;
        for (int s = 0; s < 8; ++s) {
            const uint32_t keep = kb + kg * 8 + s < k1 ? ~0u : 0u;
            v[s] = make_uint4(v[s].x & keep, v[s].y & keep, v[s].z & keep, v[s].w & keep);
        }
        if (isA || isB) {
#pragma unroll
            for (int j = 0; j < 8; ++j) buf[slot(row0 + j, kg)] = tr8(v, j);
            if (bias)
#pragma unroll
                for (int s = 0; s < 8; ++s) {
                    const uint32_t w4[4] = {v[s].x, v[s].y, v[s].z, v[s].w};
#pragma unroll
                    for (int j = 0; j < 8; ++j) bsum[j] += bf2f((uint16_t)(w4[j >> 1] >> (16 * (j & 1))));
                }
        }
        __syncthreads();   // this step's tile is stored; the other buffer is free
        load(v, st + 2);   // (past the end: the range's last row again, never used)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            bf16x8 a[MT], bb[NT];
            for (int i = 0; i < MT; ++i) {
                a[i] = __builtin_bit_cast(bf16x8, buf[slot(wm * WM + i * 16 + r, ks * 4 + q)]);
            }
            for (int j = 0; j < NT; ++j) {
                bb[j] = __builtin_bit_cast(bf16x8, buf[slot(BM + wn * 64 + j * 16 + r, ks * 4 + q)]);
            }
            for (int i = 0; i < MT; ++i)
                for (int j = 0; j < NT; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bb[j], acc[i][j], 0, 0, 0);
        }
    };
    // every path issues the same loads, so the compiler's waits before a
    // step count only the loads that step needs (an odd count gets one step
    // of zero rows)
    if (steps > 0) {
        load(v0, 0);
        load(v1, 1);
    }
#pragma unroll 1
    for (int st = 0; st < steps; st += 2) {
        run_step(v0, st);
        run_step(v1, st + 1);
    }
    const int64_t mn = (int64_t)M * N;
    float* out = ws + (int64_t)z * (mn + M);
    for (int i = 0; i < MT; ++i)
        for (int j = 0; j < NT; ++j) {
            const int n = nt * BN + wn * 64 + j * 16 + r;
            for (int e = 0; e < 4; ++e) {
                const int m = mt * BM + wm * WM + i * 16 + q * 4 + e;
                out[(int64_t)m * N + n] = acc[i][j][e];
            }
        }
    if (nt == 0) {
        if (isA)
            for (int j = 0; j < 8; ++j) bred[kg][cg * 8 + j] = bsum[j];
        __syncthreads();
        if (tid < BM) {
            float t = 0.0f;
            for (int g = 0; g < 8; ++g) t += bred[g][tid];
            out[mn + mt * BM + tid] = t;
        }
    }
}

// Working copies of the weights from the FP32 masters: the copies of master
// parameter gi (value v already in the working type), if it is a weight of
// conv blocks 2-4 or of the two dense layers.
template <class P>
struct PackDst {
    typename P::T *wf2, *wb2, *wf3, *wb3, *wf4, *wb4, *f1f, *f1b, *f2f, *f2b, *f1k;
};

template <class P>
__device__ __forceinline__ void pack_one(int64_t gi, typename P::T v, const PackDst<P>& d) {
    // conv l = 2..4: canonical [co][ci][dx]
    typename P::T* wf[5] = {nullptr, nullptr, d.wf2, d.wf3, d.wf4};
    typename P::T* wb[5] = {nullptr, nullptr, d.wb2, d.wb3, d.wb4};
#pragma unroll
    for (int l = 2; l <= 4; ++l) {
        const int Cin = CH[l - 1], Cout = CH[l];
        const int64_t i = gi - kConvW[l];
        if (i >= 0 && i < (int64_t)Cout * Cin * 5) {
            const int dx = (int)(i % 5), ci = (int)((i / 5) % Cin), co = (int)(i / (5 * Cin));
            wf[l][(int64_t)co * (5 * Cin) + dx * Cin + ci] = v;
            wb[l][(int64_t)ci * (5 * Cout) + dx * Cout + co] = v;
        }
    }
    {
        const int64_t i = gi - F1W;
        if (i >= 0 && i < 256 * 1024) {
            const int o = (int)(i >> 10), ic = (int)(i & 1023);          // canonical c*16 + x
            const int j = (ic & 15) * 64 + (ic >> 4);                      // position-major x*64 + c
            d.f1f[(int64_t)o * 1024 + j] = v;
            d.f1b[(int64_t)j * 256 + o] = v;
            // k-blocked copy for k_fc1_bf16: [j / 32][o][j % 32], one 32-column
            // slice of the layer a contiguous 16 KB
            d.f1k[((int64_t)(j >> 5) * 256 + o) * 32 + (j & 31)] = v;
        }
    }
    {
        const int64_t i = gi - F2W;
        if (i >= 0 && i < 64 * 256) {
            const int o = (int)(i >> 8), ii = (int)(i & 255);
            d.f2f[i] = v;
            d.f2b[(int64_t)ii * 64 + o] = v;
        }
    }
}

template <class P>
__global__ __launch_bounds__(256) void k_pack(const float* __restrict__ w, PackDst<P> d) {
    const int64_t gi = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (gi < kNP) pack_one<P>(gi, P::from_f(w[gi]), d);
}

// Largest value of a non-negative bf16 activation tensor (float bits order
// like the values), accumulated into *out.
__global__ __launch_bounds__(256) void k_absmax(const uint16_t* __restrict__ a, int64_t n,
                                                uint32_t* __restrict__ out) {
    __shared__ uint32_t red[256];
    uint32_t mx = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        mx = max(mx, __float_as_uint(fabsf(bf2f(a[i]))));
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, red[0]);
}

// FP8 weights: one block per output row of a packed bf16 weight matrix
// [rows][K]; scale = max|w| / 448 (1 for an all-zero row); the column scale
// of the GEMM epilogue is scale * act_scale.
__global__ __launch_bounds__(256) void k_quant_rows(const uint16_t* __restrict__ w, int K,
                                                    uint8_t* __restrict__ q, float* __restrict__ colscale,
                                                    const uint32_t* __restrict__ act_max) {
    __shared__ float red[256];
    const int row = blockIdx.x;
    float mx = 0.0f;
    for (int k = threadIdx.x; k < K; k += 256) mx = fmaxf(mx, fabsf(bf2f(w[(int64_t)row * K + k])));
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    const float sw = red[0] > 0.0f ? red[0] / 448.0f : 1.0f;
    for (int k = threadIdx.x; k < K; k += 256)
        q[(int64_t)row * K + k] = f2e4m3(bf2f(w[(int64_t)row * K + k]) / sw);
    if (threadIdx.x == 0) {
        const float am = __uint_as_float(*act_max);
        const float sa = am > 0.0f ? am / 448.0f : 1.0f;
        colscale[row] = sw * sa;
    }
}

// Adam with the step count on the device (so a captured training step can be
// replayed). step[0] holds the steps taken; every block reads it, applies
// step t = step[0] + 1 (the bias corrections worked out once per block) to
// its stripes of the parameters, and the last block to finish (counted in
// step[1]) stores t and clears the count, so no block of this launch sees
// the new value. Launch with kAdamBlocks blocks (few: the count is one
// memory-side atomic per block, with no cache maintenance).
constexpr int kAdamBlocks = 256;
// PK: the updated weights' working copies are written too (as k_pack writes
// them), so the next forward pass need not re-pack.
template <class P, bool PK>
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, int64_t n,
                                              float lr, float b1, float b2, float eps,
                                              int32_t* __restrict__ step, PackDst<P> d) {
    __shared__ float corr[2];
    __shared__ int32_t t_sh;
    if (threadIdx.x == 0) {
        const int32_t t = __hip_atomic_load(step, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
        corr[0] = (float)(1.0 - pow((double)b1, (double)t));
        corr[1] = (float)(1.0 - pow((double)b2, (double)t));
        t_sh = t;
    }
    __syncthreads();
    const float c1 = corr[0], c2 = corr[1];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float pn = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        p[i] = pn;
        if constexpr (PK) pack_one<P>(i, P::from_f(pn), d);
    }
    // thread 0 read step[0] before the barrier above, so its block has read
    // it before it is counted
    if (threadIdx.x == 0) {
        const int32_t done = __hip_atomic_fetch_add(step + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (done == (int32_t)gridDim.x - 1) {
            __hip_atomic_store(step + 1, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(step, t_sh, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

__global__ void k_copy_f32(const float* __restrict__ src, float* __restrict__ dst, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// Adam's step count and its finished-block count back to zero.
__global__ void k_reset_step(int32_t* __restrict__ p) {
    if (threadIdx.x < 2 && blockIdx.x == 0) p[threadIdx.x] = 0;
}

__global__ __launch_bounds__(256) void k_fill(float* __restrict__ p, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

template <class P, class LA, class LB, class EP>
hipError_t gemm(int M, int N, int K, LA la, LB lb, EP ep, hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    dim3 grid((M + 63) / 64, (N + 63) / 64);
    const int kc = (K + P::KSTEP - 1) / P::KSTEP * P::KSTEP;
    hipLaunchKernelGGL((k_gemm<P, LA, LB, EP>), grid, dim3(256), 0, s, M, N, K, kc, la, lb, ep);
    return hipGetLastError();
}

// Bias gradient over `rows` rows of C channels into g[C]: enough row parts to
// fill the chip, partial sums in ws, summed in part order.
template <class P>
hipError_t bias_grad(const typename P::T* d, int64_t rows, int C, float* g, float* ws, hipStream_t s) {
    const int cg = C < 64 ? C : 64;
    const int groups = C / cg;
    const int parts = (int)std::max<int64_t>(1, std::min<int64_t>(2048 / groups, rows / 32));
    hipLaunchKernelGGL((k_bias_grad<P>), dim3((unsigned)groups, (unsigned)parts), dim3(256), 0, s, d, rows,
                       C, ws);
    hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((C + 3) / 4)), dim3(256), 0, s, ws, parts, C, g);
    return hipGetLastError();
}

// Split-K workspace (floats) every network holds.
constexpr int64_t kSplitWs = int64_t(8) << 20;
// The convolution weight-gradient workspace of a bf16 step: block 1's rows
// (one per data-gradient block), blocks 4, 3 and 2's partial rows (several
// blocks per CU each), then the segment rows of the two-pass reduction (an
// eighth of the rest, plus one per job).
constexpr int64_t kDwCap[4] = {int64_t(1) << 16, int64_t(6) << 20, int64_t(6) << 20, int64_t(3) << 20};
constexpr int64_t kDwWs = kDwCap[0] + kDwCap[1] + kDwCap[2] + kDwCap[3] +
                          (kDwCap[0] + kDwCap[1] + kDwCap[2] + kDwCap[3]) / 8 + 4 * 20544;

// Weight and bias gradients of a bf16 dense layer with M outputs and N
// inputs (M a multiple of 64, N of 128) from its output gradient d [B][M]
// and input act [B][N]: batch ranges over enough blocks to fill the chip
// (at least 256 rows each), then the partials summed in range order.
inline hipError_t fc_dw_bf16(int B, int M, int N, const uint16_t* d, const uint16_t* act, EpFcDW ep,
                             float* gb, float* ws, hipStream_t s) {
    const bool wide = M % 128 == 0;
    const int tiles_n = N / 128, tiles = (wide ? M / 128 : M / 64) * tiles_n;
    const int64_t row = (int64_t)M * N + M;
    int S = std::max(1, std::min(B / 256, std::max(1, 256 / tiles)));
    S = (int)std::min<int64_t>(S, kSplitWs / row);
    int kc = (B + S - 1) / S;
    kc = (kc + 63) / 64 * 64;
    S = (B + kc - 1) / kc;
    const dim3 grid((unsigned)(tiles * S));
    if (wide)
        hipLaunchKernelGGL(k_fc_dw_bf16<128>, grid, dim3(256), 0, s, B, M, N, kc, tiles_n, d, act, ws);
    else
        hipLaunchKernelGGL(k_fc_dw_bf16<64>, grid, dim3(256), 0, s, B, M, N, kc, tiles_n, d, act, ws);
    const EpFcDWB epb{ep, gb, N, M * N};
    if (S >= 16)
        reduce_partials_w(ws, S, 1, (int)row, epb, s);
    else
        hipLaunchKernelGGL(k_splitk_reduce<EpFcDWB>, dim3(blocks_for(row)), dim3(256), 0, s, ws, S, 1, (int)row,
                           epb);
    return hipGetLastError();
}

// Weight-gradient GEMM with a long K (the batch, or batch x positions): the
// K range is split over enough blocks to fill the chip, partial tiles go to
// `ws` and one pass sums them in a fixed order into the epilogue.
template <class P, class LA, class LB, class EP>
hipError_t gemm_splitk(int M, int N, int K, LA la, LB lb, EP ep, float* ws, hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
    int S = std::max(1, 2048 / tiles);                           // about 2048 blocks
    S = std::min<int64_t>(S, std::max(1, K / 512));             // at least 512 k per block
    S = (int)std::min<int64_t>(S, kSplitWs / ((int64_t)M * N));
    if (S <= 1) return gemm<P>(M, N, K, la, lb, ep, s);
    int kc = (K + S - 1) / S;
    kc = (kc + P::KSTEP - 1) / P::KSTEP * P::KSTEP;
    S = (K + kc - 1) / kc;
    dim3 grid((M + 63) / 64, (N + 63) / 64, S);
    hipLaunchKernelGGL((k_gemm<P, LA, LB, EpPartial>), grid, dim3(256), 0, s, M, N, K, kc, la, lb,
                       EpPartial{ws});
    if (S >= 16)
        reduce_partials_w(ws, S, M, N, ep, s);
    else
        hipLaunchKernelGGL((k_splitk_reduce<EP>), dim3(blocks_for((int64_t)M * N)), dim3(256), 0, s, ws,
                           S, M, N, ep);
    return hipGetLastError();
}

}  // namespace gcnn

// ------------------------------------------------------------------ C ABI

struct gpfc_cnn {
    int32_t device = 0;
    int32_t prec = 0;            // 0 bf16, 1 fp32
    int64_t max_batch = 0;
    int32_t* step_dev = nullptr;  // Adam step count (device)
    hipGraph_t train_graph = nullptr;
    hipGraphExec_t train_exec = nullptr;
    float* params = nullptr;     // FP32 masters, canonical layout
    float* grad = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    float* loss = nullptr;
    float* loss_out = nullptr;   // during one backward call: the caller's loss buffer
    float* ws = nullptr;         // split-K partial sums (kSplitWs floats)
    float* wsd = nullptr;        // convolution weight-gradient rows of a bf16 step (kDwWs floats)
    void* work = nullptr;        // packed weights + activations
    bool packed = false;
    bool fused = true;           // bf16 inference through the fused convolution stack
    int32_t fused_mode = 1;      // 1: wave-private inputs, 2: tiles of 8 inputs in lockstep
    int32_t n_cu = 256;
    // views into work (element type per prec)
    void *wf2, *wb2, *wf3, *wb3, *wf4, *wb4, *f1f, *f1b, *f2f, *f2b;
    void* f1k;                                // the first dense layer, k-blocked (k_fc1_bf16)
    void *a1, *a2, *a3, *a4, *h1, *h2;       // activations
    void *d_a, *d_b;                          // gradient scratch (largest activation size)
    uint8_t *m1, *m2, *m3, *m4;
    // FP8 inference (bf16 networks): E4M3 weights, per-column scales, activation maxima
    uint8_t *q2, *q3, *q4, *qf1, *qf2;
    float *cs2, *cs3, *cs4, *csf1, *csf2;
    uint32_t* act_max;                        // [5] float bits: inputs of conv2..4, fc1, fc2
    float act_max_host[5] = {0, 0, 0, 0, 0};
    bool calibrated = false, quantized = false;
};

int64_t gpfc::cnn_max_batch(const gpfc_cnn* c) { return c->max_batch; }

namespace {

thread_local char g_cnn_err[256] = "";

int32_t cnn_err(hipError_t e, const char* what) {
    snprintf(g_cnn_err, sizeof(g_cnn_err), "%s: %s", what, hipGetErrorString(e));
    return GPFC_EDEVICE;
}

template <class P>
gcnn::PackDst<P> pack_dst(gpfc_cnn* c) {
    using T = typename P::T;
    return gcnn::PackDst<P>{(T*)c->wf2, (T*)c->wb2, (T*)c->wf3, (T*)c->wb3, (T*)c->wf4, (T*)c->wb4,
                            (T*)c->f1f, (T*)c->f1b, (T*)c->f2f, (T*)c->f2b, (T*)c->f1k};
}

// True while `s` records into a graph: work enqueued now has not run yet, so
// the working copies it makes cannot be marked ready, and a graph must make
// its own (each replay then uses the network's current weights).
bool capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    return s && hipStreamIsCapturing(s, &st) == hipSuccess && st == hipStreamCaptureStatusActive;
}

template <class P>
int32_t pack(gpfc_cnn* c, hipStream_t s) {
    using T = typename P::T;
    hipLaunchKernelGGL((gcnn::k_pack<P>), dim3(gcnn::blocks_for(gcnn::kNP)), dim3(256), 0, s, c->params,
                       pack_dst<P>(c));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return cnn_err(e, "k_pack");
    c->packed = !capturing(s);   // a captured pack runs only when the graph does
    return GPFC_OK;
}

template <class P>
int32_t forward(gpfc_cnn* c, const void* x, int xf32, int B, float* logits, const float* labels,
                hipStream_t s) {
    using namespace gcnn;
    using T = typename P::T;
    hipError_t e;
    if (!c->packed || capturing(s)) {
        int32_t rc = pack<P>(c, s);
        if (rc != GPFC_OK) return rc;
    }
    const float* w = c->params;
    const bool train = labels != nullptr;   // pooling masks are kept for the backward pass only
    T* acts[5] = {nullptr, (T*)c->a1, (T*)c->a2, (T*)c->a3, (T*)c->a4};
    uint8_t* masks[5] = {nullptr, c->m1, c->m2, c->m3, c->m4};
    if (!train) masks[2] = masks[3] = masks[4] = nullptr;
    void* wfs[5] = {nullptr, nullptr, c->wf2, c->wf3, c->wf4};
    // a bf16 network runs the fused convolution stack (bit-identical to the
    // layer path); a training step's forward also writes the activations and
    // masks the backward pass reads
    const bool fused = __is_same(P, BF16) && (train || logits) && c->fused &&
                       ((uintptr_t)x & 15) == 0;   // the fused kernel loads 16-byte groups
    if (fused) {
        const int ntiles = (B + kTileF - 1) / kTileF;
        const dim3 wgrid((unsigned)std::min<int64_t>((B + kWP - 1) / kWP, c->n_cu));
        auto stack = [&](auto kernel, bool with_train_outputs) {
            hipLaunchKernelGGL(kernel, wgrid, dim3(kWP * 64), 0, s, x, B, w + kConvW[1], w + conv_b(1),
                               (const uint16_t*)c->wf2, w + conv_b(2), (const uint16_t*)c->wf3, w + conv_b(3),
                               (const uint16_t*)c->wf4, w + conv_b(4), (uint16_t*)c->a4,
                               with_train_outputs ? (uint16_t*)c->a1 : nullptr,
                               with_train_outputs ? (uint16_t*)c->a2 : nullptr,
                               with_train_outputs ? (uint16_t*)c->a3 : nullptr, with_train_outputs ? c->m1 : nullptr,
                               with_train_outputs ? c->m2 : nullptr, with_train_outputs ? c->m3 : nullptr,
                               with_train_outputs ? c->m4 : nullptr);
        };
        if (train)
            xf32 ? stack(k_convstack_bf16_w<true, true>, true) : stack(k_convstack_bf16_w<true, false>, true);
        else if (c->fused_mode == 1)
            xf32 ? stack(k_convstack_bf16_w<false, true>, false) : stack(k_convstack_bf16_w<false, false>, false);
        else
            hipLaunchKernelGGL(k_convstack_bf16, dim3((unsigned)std::min(ntiles, c->n_cu)),
                               dim3(kFusedThreads), 0, s, x, xf32, B, w + kConvW[1], w + conv_b(1),
                               (const uint16_t*)c->wf2, w + conv_b(2), (const uint16_t*)c->wf3,
                               w + conv_b(3), (const uint16_t*)c->wf4, w + conv_b(4), (uint16_t*)c->a4);
    } else {
    hipLaunchKernelGGL((k_conv1_fwd<P>), dim3(blocks_for((int64_t)B * 128 * 16)), dim3(256), 0, s, x,
                       xf32, B, w + kConvW[1], w + conv_b(1), (T*)c->a1, train ? c->m1 : nullptr);
    for (int l = 2; l <= 4; ++l) {
        const int Cin = CH[l - 1], Cout = CH[l], L = LEN[l - 1];
        ConvRows<P> la{acts[l - 1], L, Cin, B * L, +1};
        Rows<P> lb{(const T*)wfs[l], Cout, 5 * Cin, 5 * Cin};
        EpConvFwd<P> ep{w + conv_b(l), acts[l], masks[l], Cout};
        e = gemm<P>(B * L, Cout, 5 * Cin, la, lb, ep, s);
        if (e != hipSuccess) return cnn_err(e, "conv gemm");
    }
    }
    if (fused) {
        // tiles that keep the chip busy: 256 rows, 128 rows, or for small
        // batches 128 x 64 tiles of the generic staged kernel (same bits)
        if ((B + 255) / 256 >= c->n_cu)
            hipLaunchKernelGGL(k_fc1_bf16<256>, dim3((unsigned)((B + 255) / 256)), dim3(1024), 0, s, B, 1024,
                               (const uint16_t*)c->a4, (const uint16_t*)c->f1k, w + F1B, (uint16_t*)c->h1);
        else if ((B + 127) / 128 >= c->n_cu)
            hipLaunchKernelGGL(k_fc1_bf16<128>, dim3((unsigned)((B + 127) / 128)), dim3(512), 0, s, B, 1024,
                               (const uint16_t*)c->a4, (const uint16_t*)c->f1k, w + F1B, (uint16_t*)c->h1);
        else if ((B + 63) / 64 >= c->n_cu / 2)
            hipLaunchKernelGGL(k_fc1_bf16<64>, dim3((unsigned)((B + 63) / 64)), dim3(256), 0, s, B, 1024,
                               (const uint16_t*)c->a4, (const uint16_t*)c->f1k, w + F1B, (uint16_t*)c->h1);
        else
            hipLaunchKernelGGL((k_fc_bf16<64, kFcRelu>), dim3((unsigned)((B + 127) / 128), 4), dim3(256), 0, s, B,
                               1024, (const uint16_t*)c->a4, (const uint16_t*)c->f1f, w + F1B, (uint16_t*)c->h1, 256,
                               nullptr, nullptr);
        // inference: the output layer runs in the second dense layer's
        // epilogue (h2 never reaches memory); training: the output layer,
        // loss and dh2 in the same epilogue, then the part sums added up
        if (!train)
            hipLaunchKernelGGL((k_fc_bf16<64, kFcHead>), dim3((unsigned)((B + 127) / 128), 1), dim3(256), 0, s, B,
                               256, (const uint16_t*)c->h1, (const uint16_t*)c->f2f, w + F2B, nullptr, 64, w + F3W,
                               logits, nullptr, nullptr);
        else
            hipLaunchKernelGGL((k_fc_bf16<64, kFcHeadTrain>), dim3((unsigned)((B + 127) / 128), 1), dim3(256), 0, s,
                               B, 256, (const uint16_t*)c->h1, (const uint16_t*)c->f2f, w + F2B, (uint16_t*)c->d_a,
                               64, w + F3W, logits, labels, c->ws);
        e = hipGetLastError();
        if (e != hipSuccess) return cnn_err(e, "fc gemm");
    } else {
    e = gemm<P>(B, 256, 1024, Rows<P>{(const T*)c->a4, B, 1024, 1024},
                Rows<P>{(const T*)c->f1f, 256, 1024, 1024}, EpFcFwd<P>{w + F1B, (T*)c->h1, 256}, s);
    if (e != hipSuccess) return cnn_err(e, "fc1 gemm");
    e = gemm<P>(B, 64, 256, Rows<P>{(const T*)c->h1, B, 256, 256},
                Rows<P>{(const T*)c->f2f, 64, 256, 256}, EpFcFwd<P>{w + F2B, (T*)c->h2, 64}, s);
    if (e != hipSuccess) return cnn_err(e, "fc2 gemm");
    }
    if (train) {
        // parts of kHeadRowsPerPart rows; the fused layer left their sums at
        // the start of the workspace, the layer path keeps rows [2 B] there
        // and the part sums after them
        const int parts = (int)((B + kHeadRowsPerPart - 1) / kHeadRowsPerPart);
        float* psum = c->ws;
        if (!fused) {
            float* rows = c->ws;
            psum = c->ws + 2 * (int64_t)B;
            hipLaunchKernelGGL((k_head_rows<P>), dim3(blocks_for(B)), dim3(256), 0, s, (const T*)c->h2, B,
                               w + F3W, w + F3B, labels, logits, rows);
            hipLaunchKernelGGL((k_head_dh2<P>), dim3(blocks_for((int64_t)B * 64)), dim3(256), 0, s,
                               (const T*)c->h2, B, w + F3W, rows, (T*)c->d_a);
            hipLaunchKernelGGL((k_head_parts<P>), dim3((unsigned)parts), dim3(256), 0, s, (const T*)c->h2, B,
                               rows, psum);
        }
        hipLaunchKernelGGL(k_head_final, dim3((kHeadSums + 3) / 4), dim3(256), 0, s, psum, parts, B,
                           c->grad, c->loss, c->loss_out);
    } else if (logits && !fused)
        hipLaunchKernelGGL((k_head_infer<P>), dim3(blocks_for(B)), dim3(256), 0, s, (const T*)c->h2,
                           B, w + F3W, w + F3B, logits);
    e = hipGetLastError();
    return e == hipSuccess ? GPFC_OK : cnn_err(e, "k_head");
}

// Backward of the four convolution blocks of a bf16 network from the pooled
// gradient of block 4 (in d_a): the data gradients in one pass down the
// blocks, then each block's weight and bias gradients from its pooled
// gradient, mask and input.
template <int L, int CIN, int COUT, int WN, int WK>
int conv_dw_bf16(const gpfc_cnn* c, int B, const uint16_t* dact, const uint8_t* mask, const uint16_t* act,
                 float* ws, int64_t cap, hipStream_t s) {
    using namespace gcnn;
    const int64_t row = (int64_t)COUT * 5 * CIN + COUT;
    static_assert(COUT % 4 == 0, "rows of whole 16-byte units");
    const int groups = (B + 7) / 8;
    // block 4 (one 32-position item per group): the staged pipeline, one
    // block of 8 waves per CU; blocks 2 and 3: several 4-wave blocks per CU,
    // each staging and computing in turn (faster for their small items)
    constexpr bool kPipe = L == 32;
    const int per_cu = kPipe ? 1 : (CIN == 16 ? 3 : 2);
    int blocks = (int)std::min<int64_t>(std::min(groups, per_cu * c->n_cu), cap / row);
    const int gpb = (groups + blocks - 1) / blocks;
    blocks = (groups + gpb - 1) / gpb;
    if constexpr (kPipe)
        hipLaunchKernelGGL((k_conv_dw_pipe_bf16<L, CIN, COUT, WN, WK>), dim3((unsigned)blocks), dim3(512), 0, s, B,
                           gpb, dact, mask, act, ws);
    else
        hipLaunchKernelGGL((k_conv_dw_bf16<L, CIN, COUT, WN, WK>), dim3((unsigned)blocks), dim3(256), 0, s, B, gpb,
                           dact, mask, act, ws);
    return blocks;   // partial rows
}

int32_t backward_convs_bf16(gpfc_cnn* c, const void* x, int xf32, int B, hipStream_t s) {
    using namespace gcnn;
    float* g = c->grad;
    const uint16_t* d4 = (const uint16_t*)c->d_a;                 // [B][16][64]
    uint16_t* d3 = (uint16_t*)c->d_b;                              // [B][32][64]
    uint16_t* d2 = (uint16_t*)c->d_b + (int64_t)B * 2048;          // [B][64][32]
    // the data gradients down the blocks, one kernel per block
    const dim3 gt((unsigned)std::min<int64_t>((B + kTW - 1) / kTW, c->n_cu));
    hipLaunchKernelGGL((k_convT_bf16<16, 64, 64, kB4Ld, 2, 4>), gt, dim3(kTW * 64), 0, s, B,
                       (const uint16_t*)c->wb4, d4, c->m4, d3);
    hipLaunchKernelGGL((k_convT_bf16<32, 64, 32, kB3Ld, 4, 2>), gt, dim3(kTW * 64), 0, s, B,
                       (const uint16_t*)c->wb3, (const uint16_t*)d3, c->m3, d2);
    // block 2's data gradient also gives block 1's weight gradients (one row
    // of 96 sums per block)
    float* wd = c->wsd;
    const int64_t cap1 = kDwCap[0], capw[3] = {kDwCap[1], kDwCap[2], kDwCap[3]};
    if ((int64_t)gt.x * 96 > cap1) return GPFC_ERANGE;   // more data-gradient blocks than rows
    if (xf32)
        hipLaunchKernelGGL((k_convT_bf16<64, 32, 16, kB2Ld, 8, 1, 2>), gt, dim3(kTW * 64), 0, s, B,
                           (const uint16_t*)c->wb2, (const uint16_t*)d2, c->m2, (uint16_t*)nullptr, c->m1, x, wd);
    else
        hipLaunchKernelGGL((k_convT_bf16<64, 32, 16, kB2Ld, 8, 1, 1>), gt, dim3(kTW * 64), 0, s, B,
                           (const uint16_t*)c->wb2, (const uint16_t*)d2, c->m2, (uint16_t*)nullptr, c->m1, x, wd);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return cnn_err(e, "backward data gradients");
    // blocks 4, 3, 2: partial rows in their own regions, then one two-pass
    // reduction of all four blocks' rows
    float* r4 = wd + cap1;
    float* r3 = r4 + capw[0];
    float* r2 = r3 + capw[1];
    float* segs = r2 + capw[2];
    DwJobs J{};
    J.n = 4;
    J.ws[0] = wd;  J.S[0] = (int)gt.x;  J.row[0] = 96;      J.cin[0] = 1;
    J.gw[0] = g + kConvW[1];  J.gb[0] = g + kConvW[1] + 80;
    J.ws[1] = r4;  J.S[1] = conv_dw_bf16<32, 64, 64, 4, 1>(c, B, d4, c->m4, (const uint16_t*)c->a3, r4, capw[0], s);
    J.row[1] = 64 * 320 + 64;  J.cin[1] = 64;  J.gw[1] = g + kConvW[4];  J.gb[1] = g + conv_b(4);
    J.ws[2] = r3;  J.S[2] = conv_dw_bf16<64, 32, 64, 2, 2>(c, B, d3, c->m3, (const uint16_t*)c->a2, r3, capw[1], s);
    J.row[2] = 64 * 160 + 64;  J.cin[2] = 32;  J.gw[2] = g + kConvW[3];  J.gb[2] = g + conv_b(3);
    J.ws[3] = r2;  J.S[3] = conv_dw_bf16<128, 16, 32, 1, 4>(c, B, d2, c->m2, (const uint16_t*)c->a1, r2, capw[2], s);
    J.row[3] = 32 * 80 + 32;  J.cin[3] = 16;  J.gw[3] = g + kConvW[2];  J.gb[3] = g + conv_b(2);
    e = hipGetLastError();
    if (e != hipSuccess) return cnn_err(e, "k_conv_dw_bf16");
    int ymax = 0, xcols = 0;
    J.ybase[0] = 0;
    J.xbase[0] = 0;
    for (int j = 0; j < 4; ++j) {
        const int G = (J.S[j] + kDwR - 1) / kDwR;
        J.seg[j] = segs;
        segs += (int64_t)G * J.row[j];
        J.ybase[j + 1] = J.ybase[j] + G;
        J.xbase[j + 1] = J.xbase[j] + (J.row[j] + 63) / 64;
        ymax = std::max(ymax, (J.row[j] / 4 + 255) / 256);
        xcols = J.xbase[j + 1];
    }
    // (segment rows: sum of ceil(S_j / 8) row_j <= sum of cap_j / 8 + 4 rows <= what kDwWs leaves)
    hipLaunchKernelGGL(k_dw_seg, dim3((unsigned)ymax, (unsigned)J.ybase[4]), dim3(256), 0, s, J);
    hipLaunchKernelGGL(k_dw_final, dim3((unsigned)xcols), dim3(1024), 0, s, J);
    e = hipGetLastError();
    return e == hipSuccess ? GPFC_OK : cnn_err(e, "conv weight-gradient reduction");
}

template <class P>
int32_t backward(gpfc_cnn* c, const void* x, int xf32, int B, hipStream_t s) {
    using namespace gcnn;
    using T = typename P::T;
    hipError_t e;
    float* g = c->grad;
    // dh2 (already masked) is in d_a [B][64]
    T* dh2 = (T*)c->d_a;
    // bf16 (both paths): the staged weight-gradient kernel, bias sums included
    constexpr bool kBf = __is_same(P, BF16);
    if constexpr (kBf)
        e = fc_dw_bf16(B, 64, 256, (const uint16_t*)dh2, (const uint16_t*)c->h1, EpFcDW{g + F2W, 256, false},
                       g + F2B, c->ws, s);
    else
        e = gemm_splitk<P>(64, 256, B, Cols<P>{dh2, 64, 64, B}, Cols<P>{(const T*)c->h1, 256, 256, B},
                           EpFcDW{g + F2W, 256, false}, c->ws, s);
    if (e != hipSuccess) return cnn_err(e, "fc2 dW");
    if constexpr (!kBf) {
        e = bias_grad<P>(dh2, B, 64, g + F2B, c->ws, s);
        if (e != hipSuccess) return cnn_err(e, "fc2 bias grad");
    }
    T* dh1 = (T*)c->d_b;   // [B][256], masked by h1 > 0
    e = gemm<P>(B, 256, 64, Rows<P>{dh2, B, 64, 64}, Rows<P>{(const T*)c->f2b, 256, 64, 64},
                EpStore<P>{dh1, (const T*)c->h1, 256}, s);
    if (e != hipSuccess) return cnn_err(e, "fc2 dX");
    if constexpr (kBf)
        e = fc_dw_bf16(B, 256, 1024, (const uint16_t*)dh1, (const uint16_t*)c->a4, EpFcDW{g + F1W, 1024, true},
                       g + F1B, c->ws, s);
    else
        e = gemm_splitk<P>(256, 1024, B, Cols<P>{dh1, 256, 256, B},
                           Cols<P>{(const T*)c->a4, 1024, 1024, B}, EpFcDW{g + F1W, 1024, true}, c->ws, s);
    if (e != hipSuccess) return cnn_err(e, "fc1 dW");
    if constexpr (!kBf) {
        e = bias_grad<P>(dh1, B, 256, g + F1B, c->ws, s);
        if (e != hipSuccess) return cnn_err(e, "fc1 bias grad");
    }
    T* dact = (T*)c->d_a;  // [B][1024] = pooled gradient of block 4, position-major
    // bf16: the staged kernel (same MFMA chains and rounding as the GEMM)
    if (__is_same(P, BF16) && c->fused) {
        hipLaunchKernelGGL((k_fc_bf16<128, kFcStore>), dim3((unsigned)((B + 127) / 128), 8), dim3(256), 0, s, B,
                           256, (const uint16_t*)dh1, (const uint16_t*)c->f1b, nullptr, (uint16_t*)dact, 1024,
                           nullptr, nullptr);
        e = hipGetLastError();
    } else
        e = gemm<P>(B, 1024, 256, Rows<P>{dh1, B, 256, 256}, Rows<P>{(const T*)c->f1b, 1024, 256, 256},
                    EpStore<P>{dact, nullptr, 1024}, s);
    if (e != hipSuccess) return cnn_err(e, "fc1 dX");
    if constexpr (__is_same(P, BF16))
        if (c->fused && ((uintptr_t)x & 15) == 0)   // block 1 reads the input in aligned pairs
            return backward_convs_bf16(c, x, xf32, B, s);
    T* acts[5] = {nullptr, (T*)c->a1, (T*)c->a2, (T*)c->a3, (T*)c->a4};
    uint8_t* masks[5] = {nullptr, c->m1, c->m2, c->m3, c->m4};
    void* wbs[5] = {nullptr, nullptr, c->wb2, c->wb3, c->wb4};
    T* bufA = (T*)c->d_a;
    T* bufB = (T*)c->d_b;
    for (int l = 4; l >= 1; --l) {
        const int Cin = CH[l - 1], Cout = CH[l], L = LEN[l - 1];
        const int64_t npool = (int64_t)B * (L / 2) * Cout;
        T* dpre = (bufA == dact) ? bufB : bufA;
        hipLaunchKernelGGL((k_unpool<P>), dim3(blocks_for(npool)), dim3(256), 0, s, dact, masks[l],
                           npool, Cout, dpre);
        e = bias_grad<P>(dpre, (int64_t)B * L, Cout, g + conv_b(l), c->ws, s);
        if (e != hipSuccess) return cnn_err(e, "conv bias grad");
        if (l == 1) {
            const int parts = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (int64_t)B * 256 / 1024));
            hipLaunchKernelGGL((k_conv1_dw<P>), dim3(parts), dim3(256), 0, s, dpre, x, xf32, B, c->ws);
            hipLaunchKernelGGL(k_sum_parts, dim3(20), dim3(256), 0, s, c->ws, parts, 80, g + kConvW[1]);
            break;
        }
        e = gemm_splitk<P>(Cout, 5 * Cin, B * L, Cols<P>{dpre, Cout, Cout, B * L},
                           ConvCols<P>{acts[l - 1], L, Cin, B * L}, EpConvDW{g + kConvW[l], Cin},
                           c->ws, s);
        if (e != hipSuccess) return cnn_err(e, "conv dW");
        // gradient with respect to the block's input (pooled output of l-1)
        T* dnext = dact;   // reuse: dact is free once dpre exists
        e = gemm<P>(B * L, Cin, 5 * Cout, ConvRows<P>{dpre, L, Cout, B * L, -1},
                    Rows<P>{(const T*)wbs[l], Cin, 5 * Cout, 5 * Cout},
                    EpStore<P>{dnext, nullptr, Cin}, s);
        if (e != hipSuccess) return cnn_err(e, "conv dX");
        dact = dnext;
        bufA = dact;
        bufB = dpre;
    }
    e = hipGetLastError();
    return e == hipSuccess ? GPFC_OK : cnn_err(e, "backward");
}

size_t elt(const gpfc_cnn* c) { return c->prec ? 4 : 2; }

}  // namespace

extern "C" {

int32_t gpfc_cnn_nparams(void) { return gcnn::kNP; }

const char* gpfc_cnn_last_error(void) { return g_cnn_err; }

int32_t gpfc_cnn_create(gpfc_cnn** out, int32_t device, int32_t precision, int64_t max_batch) {
    if (!out) return GPFC_EINVAL;
    *out = nullptr;
    if (precision != GPFC_CNN_BF16 && precision != GPFC_CNN_FP32) return GPFC_EINVAL;
    if (max_batch < 1 || max_batch > (1 << 22)) return GPFC_EINVAL;
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return cnn_err(e, "hipSetDevice");
    gpfc_cnn* c = new (std::nothrow) gpfc_cnn();
    if (!c) return GPFC_ENOMEM;
    c->device = device;
    c->prec = precision;
    {
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
            ncu > 0)
            c->n_cu = ncu;
    }
    c->max_batch = max_batch;
    const size_t E = elt(c);
    const int64_t Bm = max_batch;
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    size_t wsz[11] = {32 * 80, 16 * 160, 64 * 160, 32 * 320, 64 * 320, 64 * 320,
                      256 * 1024, 1024 * 256, 64 * 256, 256 * 64, 256 * 1024};
    size_t asz[6] = {(size_t)Bm * 128 * 16, (size_t)Bm * 64 * 32, (size_t)Bm * 32 * 64,
                     (size_t)Bm * 16 * 64, (size_t)Bm * 256, (size_t)Bm * 64};
    const size_t dsz = (size_t)Bm * 256 * 16;   // largest pre-pool gradient (block 1)
    size_t total = 0;
    for (size_t z : wsz) total += al(z * E);
    for (size_t z : asz) total += al(z * E);
    total += 2 * al(dsz * E);
    for (int i = 0; i < 4; ++i) total += al(asz[i]);   // masks
    const size_t fsz = al(sizeof(float) * gcnn::kNP);
    // the reduction workspace also holds the output layer's rows and part sums
    const int64_t wsn = std::max<int64_t>(
        gcnn::kSplitWs, 2 * Bm + (Bm / gcnn::kHeadRowsPerPart + 1) * gcnn::kHeadSums);
    total += 4 * fsz + 256 + al(sizeof(float) * wsn) + al(sizeof(float) * gcnn::kDwWs);
    const size_t qsz[5] = {32 * 80, 64 * 160, 64 * 320, 256 * 1024, 64 * 256};
    const size_t csz[5] = {32, 64, 64, 256, 64};
    for (int i = 0; i < 5; ++i) total += al(qsz[i]) + al(csz[i] * sizeof(float));
    total += 2 * 256;                           // activation maxima, Adam step count
    void* base = nullptr;
    e = hipMalloc(&base, total);
    if (e != hipSuccess) {
        delete c;
        return e == hipErrorOutOfMemory ? GPFC_ENOMEM : cnn_err(e, "hipMalloc");
    }
    c->work = base;
    char* p = (char*)base;
    auto take = [&](size_t bytes) { void* r = p; p += al(bytes); return r; };
    c->params = (float*)take(sizeof(float) * gcnn::kNP);
    c->grad = (float*)take(sizeof(float) * gcnn::kNP);
    c->m = (float*)take(sizeof(float) * gcnn::kNP);
    c->v = (float*)take(sizeof(float) * gcnn::kNP);
    c->loss = (float*)take(256);
    c->ws = (float*)take(sizeof(float) * wsn);
    c->wsd = (float*)take(sizeof(float) * gcnn::kDwWs);
    void** wv[11] = {&c->wf2, &c->wb2, &c->wf3, &c->wb3, &c->wf4, &c->wb4, &c->f1f, &c->f1b, &c->f2f, &c->f2b,
                     &c->f1k};
    for (int i = 0; i < 11; ++i) *wv[i] = take(wsz[i] * E);
    void** av[6] = {&c->a1, &c->a2, &c->a3, &c->a4, &c->h1, &c->h2};
    for (int i = 0; i < 6; ++i) *av[i] = take(asz[i] * E);
    c->d_a = take(dsz * E);
    c->d_b = take(dsz * E);
    uint8_t** mv[4] = {&c->m1, &c->m2, &c->m3, &c->m4};
    for (int i = 0; i < 4; ++i) *mv[i] = (uint8_t*)take(asz[i]);
    uint8_t** qv[5] = {&c->q2, &c->q3, &c->q4, &c->qf1, &c->qf2};
    float** cv[5] = {&c->cs2, &c->cs3, &c->cs4, &c->csf1, &c->csf2};
    for (int i = 0; i < 5; ++i) {
        *qv[i] = (uint8_t*)take(qsz[i]);
        *cv[i] = (float*)take(csz[i] * sizeof(float));
    }
    c->act_max = (uint32_t*)take(256);
    c->step_dev = (int32_t*)take(256);
    if ((size_t)(p - (char*)base) > total) {   // the views must lie inside the allocation
        (void)hipFree(base);
        delete c;
        snprintf(g_cnn_err, sizeof(g_cnn_err), "gpfc_cnn_create: workspace layout exceeds its allocation");
        return GPFC_EDEVICE;
    }
    e = hipMemset(c->step_dev, 0, 256);   // no steps taken, no blocks counted
    if (e != hipSuccess) {
        (void)hipFree(base);
        delete c;
        return cnn_err(e, "hipMemset");
    }
    *out = c;
    return GPFC_OK;
}

int32_t gpfc_cnn_destroy(gpfc_cnn* c) {
    if (!c) return GPFC_OK;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    if (c->train_exec) (void)hipGraphExecDestroy(c->train_exec);
    if (c->train_graph) (void)hipGraphDestroy(c->train_graph);
    if (c->work) (void)hipFree(c->work);
    delete c;
    return GPFC_OK;
}

// After new parameters: Adam moments and step count back to zero, working
// copies to be re-packed.
static int32_t reset_after_params(gpfc_cnn* c, hipStream_t s) {
    const unsigned nb = gcnn::blocks_for(gcnn::kNP);
    hipLaunchKernelGGL(gcnn::k_fill, dim3(nb), dim3(256), 0, s, c->m, (int64_t)gcnn::kNP, 0.0f);
    hipLaunchKernelGGL(gcnn::k_fill, dim3(nb), dim3(256), 0, s, c->v, (int64_t)gcnn::kNP, 0.0f);
    hipLaunchKernelGGL(gcnn::k_reset_step, dim3(1), dim3(64), 0, s, c->step_dev);
    c->packed = false;
    c->quantized = false;
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? GPFC_OK : cnn_err(e, "set params");
}

int32_t gpfc_cnn_set_params(gpfc_cnn* c, const float* params, void* stream) {
    if (!c || !params) return GPFC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(c->params, params, sizeof(float) * gcnn::kNP,
                                  hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return cnn_err(e, "set params");
    return reset_after_params(c, s);
}

// Network file: 8-byte tag, int64 parameter count, then the FP32 parameters
// in the canonical order, little-endian.
static const char kCnnFileTag[8] = {'G', 'P', 'F', 'C', 'C', 'N', 'N', '1'};

int32_t gpfc_cnn_save(gpfc_cnn* c, const char* path, void* stream) {
    if (!c || !path) return GPFC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    float* h = new (std::nothrow) float[gcnn::kNP];
    if (!h) return GPFC_ENOMEM;
    hipError_t e = hipMemcpyAsync(h, c->params, sizeof(float) * gcnn::kNP, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { delete[] h; return cnn_err(e, "save"); }
    FILE* f = fopen(path, "wb");
    if (!f) { delete[] h; return GPFC_EIO; }
    const int64_t n = gcnn::kNP;
    bool ok = fwrite(kCnnFileTag, 1, 8, f) == 8 && fwrite(&n, sizeof(n), 1, f) == 1 &&
              fwrite(h, sizeof(float), (size_t)n, f) == (size_t)n;
    ok = (fclose(f) == 0) && ok;
    delete[] h;
    return ok ? GPFC_OK : GPFC_EIO;
}

int32_t gpfc_cnn_load(gpfc_cnn* c, const char* path, void* stream) {
    if (!c || !path) return GPFC_EINVAL;
    FILE* f = fopen(path, "rb");
    if (!f) return GPFC_EIO;
    char tag[8];
    int64_t n = 0;
    bool ok = fread(tag, 1, 8, f) == 8 && memcmp(tag, kCnnFileTag, 8) == 0 &&
              fread(&n, sizeof(n), 1, f) == 1 && n == gcnn::kNP;
    float* h = ok ? new (std::nothrow) float[gcnn::kNP] : nullptr;
    if (ok && !h) { fclose(f); return GPFC_ENOMEM; }
    ok = ok && fread(h, sizeof(float), (size_t)n, f) == (size_t)n && fgetc(f) == EOF;
    fclose(f);
    if (!ok) { delete[] h; return GPFC_EIO; }
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(c->params, h, sizeof(float) * gcnn::kNP, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);   // the host copy is freed next
    delete[] h;
    if (e != hipSuccess) return cnn_err(e, "load");
    return reset_after_params(c, s);
}

int32_t gpfc_cnn_set_fused(gpfc_cnn* c, int32_t on) {
    if (!c) return GPFC_EINVAL;
    if (on < 0 || on > 2) return GPFC_EINVAL;
    c->fused = on != 0;
    if (on) c->fused_mode = on;
    return GPFC_OK;
}

int32_t gpfc_cnn_get_params(gpfc_cnn* c, float* out, void* stream) {
    if (!c || !out) return GPFC_EINVAL;
    hipError_t e = hipMemcpyAsync(out, c->params, sizeof(float) * gcnn::kNP, hipMemcpyDeviceToDevice,
                                  (hipStream_t)stream);
    return e == hipSuccess ? GPFC_OK : cnn_err(e, "get params");
}

int32_t gpfc_cnn_forward(gpfc_cnn* c, const void* x, int32_t x_f32, int64_t B, float* logits,
                         void* stream) {
    if (!c || B < 0 || B > c->max_batch || (B > 0 && (!x || !logits))) return GPFC_EINVAL;
    if (B == 0) return GPFC_OK;
    hipStream_t s = (hipStream_t)stream;
    return c->prec ? forward<gcnn::F32>(c, x, x_f32, (int)B, logits, nullptr, s)
                   : forward<gcnn::BF16>(c, x, x_f32, (int)B, logits, nullptr, s);
}

int32_t gpfc_cnn_backward(gpfc_cnn* c, const void* x, int32_t x_f32, const float* labels, int64_t B,
                          float* loss_out, float* grad_out, void* stream) {
    if (!c || B < 1 || B > c->max_batch || !x || !labels) return GPFC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    // every gradient entry is stored (not accumulated) by exactly one kernel;
    // the loss also goes straight to loss_out
    c->loss_out = loss_out;
    int32_t rc = c->prec ? forward<gcnn::F32>(c, x, x_f32, (int)B, nullptr, labels, s)
                         : forward<gcnn::BF16>(c, x, x_f32, (int)B, nullptr, labels, s);
    c->loss_out = nullptr;
    if (rc != GPFC_OK) return rc;
    rc = c->prec ? backward<gcnn::F32>(c, x, x_f32, (int)B, s)
                 : backward<gcnn::BF16>(c, x, x_f32, (int)B, s);
    if (rc != GPFC_OK) return rc;
    hipError_t e = hipSuccess;
    if (grad_out)
        e = hipMemcpyAsync(grad_out, c->grad, sizeof(float) * gcnn::kNP, hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? GPFC_OK : cnn_err(e, "copy out");
}

static bool adam_args_ok(float lr, float beta1, float beta2) {
    return lr >= 0.0f && beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f;
}

static int32_t enqueue_adam(gpfc_cnn* c, float lr, float beta1, float beta2, float eps, hipStream_t s) {
    // outside a graph capture the update also writes the working copies (a
    // captured forward packs its own: each replay uses the current weights)
    const bool pk = !capturing(s);
    if (c->prec)
        if (pk)
            hipLaunchKernelGGL((gcnn::k_adam<gcnn::F32, true>), dim3(gcnn::kAdamBlocks), dim3(256), 0, s, c->params,
                               c->grad, c->m, c->v, (int64_t)gcnn::kNP, lr, beta1, beta2, eps, c->step_dev,
                               pack_dst<gcnn::F32>(c));
        else
            hipLaunchKernelGGL((gcnn::k_adam<gcnn::F32, false>), dim3(gcnn::kAdamBlocks), dim3(256), 0, s,
                               c->params, c->grad, c->m, c->v, (int64_t)gcnn::kNP, lr, beta1, beta2, eps,
                               c->step_dev, pack_dst<gcnn::F32>(c));
    else if (pk)
        hipLaunchKernelGGL((gcnn::k_adam<gcnn::BF16, true>), dim3(gcnn::kAdamBlocks), dim3(256), 0, s, c->params,
                           c->grad, c->m, c->v, (int64_t)gcnn::kNP, lr, beta1, beta2, eps, c->step_dev,
                           pack_dst<gcnn::BF16>(c));
    else
        hipLaunchKernelGGL((gcnn::k_adam<gcnn::BF16, false>), dim3(gcnn::kAdamBlocks), dim3(256), 0, s,
                           c->params, c->grad, c->m, c->v, (int64_t)gcnn::kNP, lr, beta1, beta2, eps,
                           c->step_dev, pack_dst<gcnn::BF16>(c));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return cnn_err(e, "k_adam");
    c->packed = pk;
    c->quantized = false;
    return GPFC_OK;
}

int32_t gpfc_cnn_adam(gpfc_cnn* c, float lr, float beta1, float beta2, float eps, void* stream) {
    if (!c || !adam_args_ok(lr, beta1, beta2)) return GPFC_EINVAL;
    return enqueue_adam(c, lr, beta1, beta2, eps, (hipStream_t)stream);
}

int32_t gpfc_cnn_train_step(gpfc_cnn* c, const void* x, int32_t x_f32, const float* labels,
                            int64_t B, float lr, float beta1, float beta2, float eps, float* loss_out,
                            void* stream) {
    if (!c || !adam_args_ok(lr, beta1, beta2)) return GPFC_EINVAL;
    const int32_t rc = gpfc_cnn_backward(c, x, x_f32, labels, B, loss_out, nullptr, stream);
    if (rc != GPFC_OK) return rc;
    return enqueue_adam(c, lr, beta1, beta2, eps, (hipStream_t)stream);
}

int32_t gpfc_cnn_train_capture(gpfc_cnn* c, const void* x, int32_t x_f32, const float* labels,
                               int64_t B, float lr, float beta1, float beta2, float eps,
                               float* loss_out, void* stream) {
    if (!c || B < 1 || B > c->max_batch || !x || !labels || !adam_args_ok(lr, beta1, beta2))
        return GPFC_EINVAL;
    if (!stream) return GPFC_EINVAL;   // the null stream cannot be captured
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return cnn_err(e, "hipSetDevice");
    if (c->train_exec) { (void)hipGraphExecDestroy(c->train_exec); c->train_exec = nullptr; }
    if (c->train_graph) { (void)hipGraphDestroy(c->train_graph); c->train_graph = nullptr; }
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return cnn_err(e, "hipStreamBeginCapture");
    int32_t rc = gpfc_cnn_backward(c, x, x_f32, labels, B, nullptr, nullptr, stream);
    if (rc == GPFC_OK) rc = enqueue_adam(c, lr, beta1, beta2, eps, s);
    if (rc == GPFC_OK && loss_out)
        hipLaunchKernelGGL(gcnn::k_copy_f32, dim3(1), dim3(256), 0, s, c->loss, loss_out, 1);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s, &g);
    if (rc != GPFC_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return cnn_err(e, "hipStreamEndCapture");
    c->train_graph = g;
    e = hipGraphInstantiate(&c->train_exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        c->train_exec = nullptr;
        return cnn_err(e, "hipGraphInstantiate");
    }
    return GPFC_OK;
}

int32_t gpfc_cnn_train_replay(gpfc_cnn* c, void* stream) {
    if (!c || !c->train_exec) return GPFC_EINVAL;
    hipError_t e = hipGraphLaunch(c->train_exec, (hipStream_t)stream);
    return e == hipSuccess ? GPFC_OK : cnn_err(e, "hipGraphLaunch");
}

int32_t gpfc_cnn_calibrate_fp8(gpfc_cnn* c, const void* x, int32_t x_f32, int64_t B, int32_t reset,
                               void* stream) {
    if (!c || c->prec != GPFC_CNN_BF16 || B < 1 || B > c->max_batch || !x) return GPFC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (reset || !c->calibrated)
        hipLaunchKernelGGL(gcnn::k_fill, dim3(1), dim3(256), 0, s, reinterpret_cast<float*>(c->act_max),
                           (int64_t)5, 0.0f);
    int32_t rc = forward<gcnn::BF16>(c, x, x_f32, (int)B, nullptr, nullptr, s);
    // forward with no labels and no logits still fills the activations
    if (rc != GPFC_OK) return rc;
    const void* acts[5] = {c->a1, c->a2, c->a3, c->a4, c->h1};
    const int64_t n[5] = {B * 128 * 16, B * 64 * 32, B * 32 * 64, B * 1024, B * 256};
    for (int i = 0; i < 5; ++i) {
        const unsigned nb = (unsigned)std::min<int64_t>((n[i] + 255) / 256, 1024);
        hipLaunchKernelGGL(gcnn::k_absmax, dim3(nb), dim3(256), 0, s, (const uint16_t*)acts[i], n[i],
                           c->act_max + i);
    }
    uint32_t h[5];
    hipError_t e = hipMemcpyAsync(h, c->act_max, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return cnn_err(e, "calibrate");
    for (int i = 0; i < 5; ++i) memcpy(&c->act_max_host[i], &h[i], 4);
    c->calibrated = true;
    c->quantized = false;
    return GPFC_OK;
}

int32_t gpfc_cnn_forward_fp8(gpfc_cnn* c, const void* x, int32_t x_f32, int64_t B, float* logits,
                             void* stream) {
    using namespace gcnn;
    if (!c || !c->calibrated || B < 0 || B > c->max_batch || (B > 0 && (!x || !logits)))
        return GPFC_EINVAL;
    if (B == 0) return GPFC_OK;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    const bool cap = capturing(s);
    if (!c->packed || cap) {
        int32_t rc = pack<BF16>(c, s);
        if (rc != GPFC_OK) return rc;
    }
    if (!c->quantized || cap) {
        const void* wsrc[5] = {c->wf2, c->wf3, c->wf4, c->f1f, c->f2f};
        const int rows[5] = {32, 64, 64, 256, 64};
        const int Ks[5] = {80, 160, 320, 1024, 256};
        uint8_t* qs[5] = {c->q2, c->q3, c->q4, c->qf1, c->qf2};
        float* cs[5] = {c->cs2, c->cs3, c->cs4, c->csf1, c->csf2};
        for (int i = 0; i < 5; ++i)
            hipLaunchKernelGGL(k_quant_rows, dim3(rows[i]), dim3(256), 0, s, (const uint16_t*)wsrc[i],
                               Ks[i], qs[i], cs[i], c->act_max + i);
        e = hipGetLastError();
        if (e != hipSuccess) return cnn_err(e, "k_quant_rows");
        c->quantized = !cap;
    }
    float inv[5];
    for (int i = 0; i < 5; ++i) inv[i] = c->act_max_host[i] > 0.0f ? 448.0f / c->act_max_host[i] : 1.0f;
    const float* w = c->params;
    using T = uint16_t;
    const int Bi = (int)B;
    hipLaunchKernelGGL((k_conv1_fwd<BF16>), dim3(blocks_for(B * 128 * 16)), dim3(256), 0, s, x, x_f32,
                       Bi, w + kConvW[1], w + conv_b(1), (T*)c->a1, (uint8_t*)nullptr);
    T* acts[5] = {nullptr, (T*)c->a1, (T*)c->a2, (T*)c->a3, (T*)c->a4};
    uint8_t* qw[5] = {nullptr, nullptr, c->q2, c->q3, c->q4};
    float* cs[5] = {nullptr, nullptr, c->cs2, c->cs3, c->cs4};
    for (int l = 2; l <= 4; ++l) {
        const int Cin = CH[l - 1], Cout = CH[l], L = LEN[l - 1];
        ActQ<ConvRows<BF16>> la{ConvRows<BF16>{acts[l - 1], L, Cin, Bi * L, +1}, inv[l - 2]};
        WQ lb{qw[l], Cout, 5 * Cin, 5 * Cin};
        EpConvFwd<BF16> ep{w + conv_b(l), acts[l], nullptr, Cout, cs[l]};
        e = gemm<FP8>(Bi * L, Cout, 5 * Cin, la, lb, ep, s);
        if (e != hipSuccess) return cnn_err(e, "conv gemm fp8");
    }
    e = gemm<FP8>(Bi, 256, 1024, ActQ<Rows<BF16>>{Rows<BF16>{(const T*)c->a4, Bi, 1024, 1024}, inv[3]},
                  WQ{c->qf1, 256, 1024, 1024}, EpFcFwd<BF16>{w + F1B, (T*)c->h1, 256, c->csf1}, s);
    if (e != hipSuccess) return cnn_err(e, "fc1 gemm fp8");
    e = gemm<FP8>(Bi, 64, 256, ActQ<Rows<BF16>>{Rows<BF16>{(const T*)c->h1, Bi, 256, 256}, inv[4]},
                  WQ{c->qf2, 64, 256, 256}, EpFcFwd<BF16>{w + F2B, (T*)c->h2, 64, c->csf2}, s);
    if (e != hipSuccess) return cnn_err(e, "fc2 gemm fp8");
    hipLaunchKernelGGL((k_head_infer<BF16>), dim3(blocks_for(B)), dim3(256), 0, s, (const T*)c->h2,
                       Bi, w + F3W, w + F3B, logits);
    e = hipGetLastError();
    return e == hipSuccess ? GPFC_OK : cnn_err(e, "k_head fp8");
}

}  // extern "C"
