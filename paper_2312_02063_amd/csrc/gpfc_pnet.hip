// The paper's own scoring network on gfx950 (Sec. 2.5, Fig. 5 of
// arXiv:2312.02063): the normalised fold of 256 bins read row-major as a
// 16 x 16 image; circular 2-D convolutions of 128 and then 256 filters
// (3 x 3, each followed by ReLU); a global max-pool over the 256 positions
// whose 256 values are read row-major as a new 16 x 16 image; the same
// sequence with 5 x 5 kernels; a fully connected layer of 128 ReLU units,
// dropout, and one sigmoid output unit. Kernel sizes, the reshape order and
// the hidden width are readings of a figure the text does not spell out.
//
// Convolutions are cross-correlations with wrap-around in both image axes:
//   y[f][r][c] = b[f] + sum_{i,u,v} w[f][i][u][v] x[i][(r+u-p) mod 16][(c+v-p) mod 16].
// The two wide convolutions (128 -> 256 channels, K = 9 x 128 and 25 x 128)
// run as implicit GEMMs on the matrix cores (bf16 with FP32 accumulation, or
// FP32 for checking): rows are (input, position), columns filters, k =
// (tap, channel) over channels-last activations. Their epilogue never stores
// the 256 x 256 pre-activations: it takes each column's maximum over the
// tile's rows and merges it into the input's pooled value with a 64-bit
// atomic max of (ordered value bits, complemented position), so the result
// is the first position of the maximum in row-major order, as the gradient
// routing needs. The one-channel convolutions (1 -> 128 filters) and the
// dense head run on the vector units.
//
// Training: the gradient of a global max-pool reaches one position per
// channel, so the backward pass of a wide convolution is sparse: its weight
// gradient is a sum over the batch of the input patches around each
// channel's routed position (one block per filter, batch in order), and its
// data gradient scatters the filter's weights around that position (one
// block per input, filters in order). Every sum runs in a fixed order, so a
// step is deterministic.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "../../include/gpfc.h"
#include "gpfc_mfma.h"

namespace gpnet {

using gcnn::BF16;
using gcnn::F32;
using gcnn::bf16x8;
using gcnn::f32x4;

constexpr int S = 16, NPOS = 256;
constexpr int F1 = 128, F2 = 256, F3 = 128, F4 = 256, K1 = 3, K2 = 5, H = 128;
// parameter layout (FP32 masters, the oracle's flat order)
constexpr int64_t W1 = 0, B1 = W1 + F1 * K1 * K1, W2 = B1 + F1, B2 = W2 + (int64_t)F2 * F1 * K1 * K1,
                  W3 = B2 + F2, B3 = W3 + F3 * K2 * K2, W4 = B3 + F3,
                  B4 = W4 + (int64_t)F4 * F3 * K2 * K2, W5 = B4 + F4, B5 = W5 + (int64_t)H * F4,
                  W6 = B5 + H, B6 = W6 + H, NP = B6 + 1;
static_assert(NP == 1152257, "parameter count");

__device__ __forceinline__ int wrap16(int v) { return v & (S - 1); }

// Order-preserving 32-bit image of a float (larger float -> larger unsigned).
__device__ __forceinline__ uint32_t ord_bits(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord_float(uint32_t o) {
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}
// Key of (value, position): the larger value wins, then the smaller position.
__device__ __forceinline__ uint64_t pool_key(float z, int pos) {
    return ((uint64_t)ord_bits(z) << 32) | (uint32_t)(0xffffffffu - (uint32_t)pos);
}

template <class P>
__device__ __forceinline__ float in_val(const void* x, int in_f32, int64_t i) {
    return in_f32 ? reinterpret_cast<const float*>(x)[i]
                  : gcnn::bf2f(reinterpret_cast<const uint16_t*>(x)[i]);
}

// ------------------------------------------------------------------ forward

// One-channel circular convolution + ReLU: one block per input image
// ([256] values, bf16 bits or FP32), one thread per position; F filters of
// side KS (weights [F][KS*KS] and biases, FP32, already rounded to the
// working precision) read from LDS. out [B][256][F] channels-last.
template <class P, int KS, int F>
__global__ __launch_bounds__(256) void k_conv1ch(const void* __restrict__ x, int in_f32,
                                                 const float* __restrict__ w,
                                                 const float* __restrict__ b,
                                                 typename P::T* __restrict__ out) {
    __shared__ float img[NPOS];
    __shared__ float ws[F * KS * KS];
    __shared__ float bs[F];
    const int tid = threadIdx.x;
    const int64_t inp = blockIdx.x;
    img[tid] = in_val<P>(x, in_f32, inp * NPOS + tid);
    for (int i = tid; i < F * KS * KS; i += 256) ws[i] = w[i];
    for (int i = tid; i < F; i += 256) bs[i] = b[i];
    __syncthreads();
    constexpr int p = (KS - 1) / 2;
    const int r = tid >> 4, c = tid & 15;
    float v[KS * KS];
#pragma unroll
    for (int u = 0; u < KS; ++u)
#pragma unroll
        for (int q = 0; q < KS; ++q) v[u * KS + q] = img[wrap16(r + u - p) * S + wrap16(c + q - p)];
    typename P::T* o = out + (inp * NPOS + tid) * F;
    for (int f0 = 0; f0 < F; f0 += 8) {
        float acc[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            float a = bs[f0 + j];
#pragma unroll
            for (int t = 0; t < KS * KS; ++t) a += ws[(f0 + j) * KS * KS + t] * v[t];
            acc[j] = fmaxf(a, 0.0f);
        }
        if constexpr (sizeof(typename P::T) == 2) {
            uint4 pk;
            pk.x = gcnn::f2bf2(acc[0], acc[1]);
            pk.y = gcnn::f2bf2(acc[2], acc[3]);
            pk.z = gcnn::f2bf2(acc[4], acc[5]);
            pk.w = gcnn::f2bf2(acc[6], acc[7]);
            *reinterpret_cast<uint4*>(o + f0) = pk;
        } else {
            *reinterpret_cast<float4*>(o + f0) = make_float4(acc[0], acc[1], acc[2], acc[3]);
            *reinterpret_cast<float4*>(o + f0 + 4) = make_float4(acc[4], acc[5], acc[6], acc[7]);
        }
    }
}

// Implicit-GEMM rows of a wide circular convolution: row m = (input, position
// r*16 + c), k = (u*KS + v)*128 + i -> act[input][(r+u-p) mod 16][(c+v-p) mod 16][i].
template <class P, int KS>
struct Conv2DRows {
    using T = typename P::T;
    const T* act;
    int rows;
    __device__ __forceinline__ int64_t at(int m, int k) const {
        constexpr int p = (KS - 1) / 2;
        const int inp = m >> 8, pos = m & 255;
        const int tap = k >> 7, i = k & 127;
        const int u = tap / KS, v = tap - u * KS;
        const int q = wrap16((pos >> 4) + u - p) * S + wrap16((pos & 15) + v - p);
        return ((int64_t)inp * NPOS + q) * 128 + i;
    }
    __device__ __forceinline__ bf16x8 frag8(int m, int k) const {
        if (m >= rows || k >= KS * KS * 128) return bf16x8{};
        return *reinterpret_cast<const bf16x8*>(reinterpret_cast<const uint16_t*>(act) + at(m, k));
    }
    __device__ __forceinline__ float frag1(int m, int k) const {
        if (m >= rows || k >= KS * KS * 128) return 0.0f;
        return P::to_f(act[at(m, k)]);
    }
};

// Epilogue of a wide convolution: bias added, each column's maximum over the
// 16 rows of an MFMA tile (the four lanes q of column r hold 4 rows each),
// then one 64-bit atomic max per (tile, column) into key[input][filter].
// Rows of a tile are 16 consecutive positions of one input (256 per input).
struct EpGmax {
    const float* bias;
    unsigned long long* key;   // [inputs][256]
    __device__ __forceinline__ void operator()(int m, int n, f32x4 a, int M, int N) const {
        const bool ok = m < M && n < N;
        uint64_t best = 0;
        if (ok) {
            const float bn = bias[n];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint64_t kq = pool_key(a[i] + bn, (m + i) & 255);
                best = kq > best ? kq : best;
            }
        }
        // the lanes 16 and 32 apart hold the other rows of the same column
        uint64_t o = __shfl_xor(best, 16);
        best = o > best ? o : best;
        o = __shfl_xor(best, 32);
        best = o > best ? o : best;
        if (ok && (threadIdx.x & 63) < 16)
            atomicMax(key + (int64_t)(m >> 8) * 256 + n, (unsigned long long)best);
    }
};

__global__ __launch_bounds__(256) void k_fill_u64(unsigned long long* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        p[i] = 0ull;
}

// Pooled values from the keys: g = max(0, max z) in the working precision,
// arg = the first position of the maximum, or -1 when it is not positive
// (ReLU then blocks every position).
template <class P>
__global__ __launch_bounds__(256) void k_gmax_finish(const unsigned long long* __restrict__ key,
                                                     int64_t n, typename P::T* __restrict__ g,
                                                     int32_t* __restrict__ arg) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const uint64_t k = key[i];
        const float z = ord_float((uint32_t)(k >> 32));
        const int pos = (int)(0xffffffffu - (uint32_t)k);
        const bool pos_ok = z > 0.0f;
        g[i] = P::from_f(pos_ok ? z : 0.0f);
        if (arg) arg[i] = pos_ok ? pos : -1;
    }
}

// Dense head, one block of 128 threads per input: h = ReLU(W5 g2 + b5),
// hd = h * keep (dropout; keep NULL at inference), logit = b6 + sum_j w6[j] hd[j]
// summed in index order. h is kept for the backward pass when h_out != NULL.
template <class P>
__global__ __launch_bounds__(128) void k_head(const typename P::T* __restrict__ g2,
                                              const float* __restrict__ w5,
                                              const float* __restrict__ b5,
                                              const float* __restrict__ w6, const float* __restrict__ b6,
                                              const float* __restrict__ keep,
                                              float* __restrict__ h_out, float* __restrict__ logits) {
    __shared__ float gs[F4];
    __shared__ float hd[H];
    const int j = threadIdx.x;
    const int64_t inp = blockIdx.x;
    for (int f = j; f < F4; f += 128) gs[f] = P::to_f(g2[inp * F4 + f]);
    __syncthreads();
    float a = b5[j];
    const float* wr = w5 + (int64_t)j * F4;
    for (int f = 0; f < F4; ++f) a += wr[f] * gs[f];
    const float h = fmaxf(a, 0.0f);
    if (h_out) h_out[inp * H + j] = h;
    hd[j] = keep ? h * keep[inp * H + j] : h;
    __syncthreads();
    if (j == 0) {
        float z = b6[0];
        for (int t = 0; t < H; ++t) z += w6[t] * hd[t];
        logits[inp] = z;
    }
}

// Fused pair for bf16 networks: one input per block of 8 waves. The
// one-channel convolution (KS1 x KS1, 128 filters, ReLU) writes the input's
// whole activation tile (256 positions x 128 channels bf16, 64 KB) into LDS,
// rows XOR-swizzled by 16-byte chunk (chunk ^ (position & 15)), optionally
// also to HBM for the backward pass; the wide convolution (KS2 x KS2, 256
// filters) then runs on the matrix cores with A fragments from that tile (the
// tap's circular shift applied to the position) and B fragments from k-chunks
// of 32 weights per filter staged in LDS (double-buffered, rows of 96 bytes:
// a 32 mod 64-byte stride keeps the fragment reads conflict-free), each chunk
// loaded while the previous one is multiplied. Waves: 2 (positions, 128 rows
// each) x 4 (filters, 64 columns each). The epilogue pools as the layer
// path's EpGmax does (same MFMA chains in the same k order, same keys), through
// 64-bit LDS atomic maxima, and writes the pooled values and positions: the
// result equals the layer path's bit for bit.
constexpr int kPairThreads = 512;
constexpr int kBRow = 48;   // staged weight row: 32 bf16 + 16 of padding (96 bytes)

template <int KS1, int KS2, bool kWrite>
__global__ __launch_bounds__(kPairThreads, 1) void k_pair_bf16(
    const void* __restrict__ x, int in_f32, const float* __restrict__ w1,
    const float* __restrict__ b1, const uint16_t* __restrict__ w2p, const float* __restrict__ b2,
    uint16_t* __restrict__ g, int32_t* __restrict__ arg, uint16_t* __restrict__ act) {
    constexpr int K = KS2 * KS2 * 128;
    constexpr int NK = K / 32;
    constexpr int p1 = (KS1 - 1) / 2, p2 = (KS2 - 1) / 2;
    __shared__ __attribute__((aligned(16))) uint16_t At[NPOS * 128];
    __shared__ __attribute__((aligned(16))) uint16_t Bt[2][256 * kBRow];
    __shared__ float img[NPOS];
    __shared__ float ws[128 * KS1 * KS1];
    __shared__ float bs[128];
    __shared__ unsigned long long keys[256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, q = lane >> 4;
    const int64_t inp = blockIdx.x;
    if (tid < NPOS) img[tid] = in_val<BF16>(x, in_f32, inp * NPOS + tid);
    for (int i = tid; i < 128 * KS1 * KS1; i += kPairThreads) ws[i] = w1[i];
    if (tid < 128) bs[tid] = b1[tid];
    if (tid < 256) keys[tid] = 0ull;
    // the first weight chunk into registers: thread t stages half (t & 1) of filter t >> 1
    const int bn = tid >> 1, bh = tid & 1;
    const uint4* bsrc = reinterpret_cast<const uint4*>(w2p + (int64_t)bn * K + 16 * bh);
    uint4 pf0 = bsrc[0], pf1 = bsrc[1];
    __syncthreads();
    // one-channel convolution + ReLU: thread t computes channels 64 (t & 1) .. + 63 at position t >> 1
    {
        const int pos = tid >> 1, h = tid & 1;
        const int rr = pos >> 4, cc = pos & 15;
        float v[KS1 * KS1];
#pragma unroll
        for (int u = 0; u < KS1; ++u)
#pragma unroll
            for (int w = 0; w < KS1; ++w) v[u * KS1 + w] = img[wrap16(rr + u - p1) * S + wrap16(cc + w - p1)];
        for (int f0 = 64 * h; f0 < 64 * h + 64; f0 += 8) {
            float a8[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                float a = bs[f0 + j];
#pragma unroll
                for (int t = 0; t < KS1 * KS1; ++t) a += ws[(f0 + j) * KS1 * KS1 + t] * v[t];
                a8[j] = fmaxf(a, 0.0f);
            }
            uint4 pk;
            pk.x = gcnn::f2bf2(a8[0], a8[1]);
            pk.y = gcnn::f2bf2(a8[2], a8[3]);
            pk.z = gcnn::f2bf2(a8[4], a8[5]);
            pk.w = gcnn::f2bf2(a8[6], a8[7]);
            const int chunk = f0 >> 3;
            *reinterpret_cast<uint4*>(At + pos * 128 + ((chunk ^ (pos & 15)) << 3)) = pk;
            if (kWrite) *reinterpret_cast<uint4*>(act + (inp * NPOS + pos) * 128 + f0) = pk;
        }
    }
    {
        uint4* d = reinterpret_cast<uint4*>(&Bt[0][bn * kBRow + 16 * bh]);
        d[0] = pf0;
        d[1] = pf1;
    }
    __syncthreads();
    const int wm = wave & 1, wn = wave >> 1;
    f32x4 acc[8][4];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    int cur = 0;
    for (int s = 0; s < NK; ++s) {
        if (s + 1 < NK) {
            pf0 = bsrc[4 * (s + 1)];
            pf1 = bsrc[4 * (s + 1) + 1];
        }
        const int tap = s >> 2;
        const int du = tap / KS2 - p2, dv = tap % KS2 - p2;
        const int chunk = ((s & 3) << 2) + q;
        bf16x8 bfr[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            bfr[j] = *reinterpret_cast<const bf16x8*>(&Bt[cur][(wn * 64 + j * 16 + r) * kBRow + q * 8]);
        const int qc = wrap16(r + dv);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int qpos = wrap16(wm * 8 + i + du) * S + qc;
            const bf16x8 afr =
                *reinterpret_cast<const bf16x8*>(At + qpos * 128 + ((chunk ^ (qpos & 15)) << 3));
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr, bfr[j], acc[i][j], 0, 0, 0);
        }
        if (s + 1 < NK) {
            uint4* d = reinterpret_cast<uint4*>(&Bt[cur ^ 1][bn * kBRow + 16 * bh]);
            d[0] = pf0;
            d[1] = pf1;
        }
        __syncthreads();
        cur ^= 1;
    }
    // pool: each column's first maximum over the block's 256 positions
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int n = wn * 64 + j * 16 + r;
        const float bb = b2[n];
        uint64_t best = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint64_t kq = pool_key(acc[i][j][e] + bb, wm * 128 + i * 16 + 4 * q + e);
                best = kq > best ? kq : best;
            }
        uint64_t o = __shfl_xor(best, 16);
        best = o > best ? o : best;
        o = __shfl_xor(best, 32);
        best = o > best ? o : best;
        if (q == 0) atomicMax(&keys[n], (unsigned long long)best);
    }
    __syncthreads();
    if (tid < 256) {
        const uint64_t k = keys[tid];
        const float z = ord_float((uint32_t)(k >> 32));
        const int pos = (int)(0xffffffffu - (uint32_t)k);
        const bool ok = z > 0.0f;
        g[inp * 256 + tid] = gcnn::f2bf(ok ? z : 0.0f);
        arg[inp * 256 + tid] = ok ? pos : -1;
    }
}

// ------------------------------------------------------------------ backward

// Output layer and dense layer, one block of 256 threads per input: the
// loss term, dz = (sigmoid(z) - y) / B, the per-input parts of the head's
// weight gradients (dz hd[j] for w6, dh[j] for b5, dz for b6), the hidden
// gradient dh and the pooled gradient dg2 = W5^T dh.
__global__ __launch_bounds__(256) void k_head_bwd(const float* __restrict__ logits,
                                                  const float* __restrict__ labels,
                                                  const float* __restrict__ h,
                                                  const float* __restrict__ keep,
                                                  const float* __restrict__ w5,
                                                  const float* __restrict__ w6, int64_t B,
                                                  float* __restrict__ loss_part,
                                                  float* __restrict__ dz_out,
                                                  float* __restrict__ dw6_part,
                                                  float* __restrict__ dh_out,
                                                  float* __restrict__ dg2) {
    __shared__ float dhs[H];
    const int t = threadIdx.x;
    const int64_t inp = blockIdx.x;
    const float z = logits[inp], y = labels[inp];
    const float dz = (1.0f / (1.0f + expf(-z)) - y) / (float)B;
    if (t == 0) {
        loss_part[inp] = fmaxf(z, 0.0f) - z * y + log1pf(expf(-fabsf(z)));
        dz_out[inp] = dz;
    }
    if (t < H) {
        const float hj = h[inp * H + t];
        const float kp = keep ? keep[inp * H + t] : 1.0f;
        dw6_part[inp * H + t] = dz * (hj * kp);
        const float d = hj > 0.0f ? dz * w6[t] * kp : 0.0f;
        dhs[t] = d;
        dh_out[inp * H + t] = d;
    }
    __syncthreads();
    float a = 0.0f;
    for (int j = 0; j < H; ++j) a += dhs[j] * w5[(int64_t)j * F4 + t];
    dg2[inp * F4 + t] = a;
}

// Column sums over the batch in input order: out[c] = sum_b part[b][c].
__global__ __launch_bounds__(256) void k_colsum(const float* __restrict__ part, int64_t B, int ncol,
                                                float* __restrict__ out, float scale) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= ncol) return;
    float a = 0.0f;
    for (int64_t b = 0; b < B; ++b) a += part[b * ncol + c];
    out[c] = a * scale;
}

// First stage of a column sum over many rows: rows cut into gridDim.y fixed
// chunks, each summed in order (the second stage, k_colsum over the chunks,
// adds them in chunk order: a fixed order, so the result is deterministic).
__global__ __launch_bounds__(256) void k_colsum_parts(const float* __restrict__ part, int64_t B, int ncol,
                                                      float* __restrict__ out) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= ncol) return;
    const int64_t per = (B + gridDim.y - 1) / gridDim.y;
    const int64_t b0 = (int64_t)blockIdx.y * per, b1 = b0 + per < B ? b0 + per : B;
    float a = 0.0f;
    for (int64_t b = b0; b < b1; ++b) a += part[b * ncol + c];
    out[(int64_t)blockIdx.y * ncol + c] = a;
}

// dW5[j][f] = sum_b dh[b][j] g2[b][f] over the batch chunk blockIdx.y (inputs
// in order), one thread per weight, into part y of dw5 ([gridDim.y][H F4]);
// the chunks are added in order afterwards.
template <class P>
__global__ __launch_bounds__(256) void k_w5_grad(const float* __restrict__ dh,
                                                 const typename P::T* __restrict__ g2, int64_t B,
                                                 float* __restrict__ dw5) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= H * F4) return;
    const int j = e / F4, f = e - j * F4;
    const int64_t per = (B + gridDim.y - 1) / gridDim.y;
    const int64_t b0 = (int64_t)blockIdx.y * per, b1 = b0 + per < B ? b0 + per : B;
    float a = 0.0f;
    for (int64_t b = b0; b < b1; ++b) a += dh[b * H + j] * P::to_f(g2[b * F4 + f]);
    dw5[(int64_t)blockIdx.y * (H * F4) + e] = a;
}

// Weight and bias gradients of a wide convolution from the routed pool
// gradient: for filter f (block x) and a chunk of the batch (block y),
// dW[f][i][u][v] = sum_b dg[b][f] act[b][arg[b][f] + (u-p, v-p)][i] over the
// chunk's inputs whose pooled value is positive, in input order; db[f] =
// sum_b dg[b][f] over the same inputs. Chunk y writes its part at
// dw + y (F NE + F) in the parameter layout (weights, then biases); the parts
// are added in chunk order afterwards. Threads take (u, v, i) with i fastest
// (coalesced channel rows).
template <class P, int KS>
__global__ __launch_bounds__(256) void k_wide_dw(const typename P::T* __restrict__ act,
                                                 const float* __restrict__ dg,
                                                 const int32_t* __restrict__ arg, int64_t B,
                                                 float* __restrict__ dw, float* __restrict__ db) {
    constexpr int p = (KS - 1) / 2;
    constexpr int NE = KS * KS * 128;
    constexpr int PER = (NE + 255) / 256;
    const int f = blockIdx.x;
    const int tid = threadIdx.x;
    // batch part blockIdx.y of gridDim.y (fixed chunks of inputs, each in order)
    const int64_t per_part = (B + gridDim.y - 1) / gridDim.y;
    const int64_t bb0 = (int64_t)blockIdx.y * per_part;
    const int64_t bb1 = bb0 + per_part < B ? bb0 + per_part : B;
    dw += (int64_t)blockIdx.y * ((int64_t)gridDim.x * NE + gridDim.x);
    db = dw + (int64_t)gridDim.x * NE;
    float acc[PER];
    int off[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        acc[j] = 0.0f;
        const int e = tid + 256 * j;
        const int tap = e >> 7;
        off[j] = tap;   // (u, v) index; -1 marks no element
        if (e >= NE) off[j] = -1;
    }
    float bsum = 0.0f;
    for (int64_t b = bb0; b < bb1; ++b) {
        const int a = arg[b * 256 + f];
        if (a < 0) continue;
        const float g = dg[b * 256 + f];
        bsum += g;
        const int ar = a >> 4, ac = a & 15;
        const typename P::T* base = act + (int64_t)b * NPOS * 128;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            if (off[j] < 0) continue;
            const int e = tid + 256 * j;
            const int u = off[j] / KS, v = off[j] - u * KS, i = e & 127;
            const int q = wrap16(ar + u - p) * S + wrap16(ac + v - p);
            acc[j] += g * P::to_f(base[q * 128 + i]);
        }
    }
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        if (off[j] < 0) continue;
        const int e = tid + 256 * j;
        const int u = off[j] / KS, v = off[j] - u * KS, i = e & 127;
        dw[(((int64_t)f * 128 + i) * KS + u) * KS + v] = acc[j];
    }
    if (tid == 0) db[f] = bsum;
}

// Per-input backward through both convolution pairs, one block of 1024
// threads per input, the data gradient held in LDS ([256 positions][128
// channels] FP32):
//  1. scatter the second wide convolution's routed gradient: for each filter
//     f in order, da3[arg2[f] + (u-2, v-2)][i] += dg2[f] w4[f][i][u][v];
//  2. mask by a3 > 0 (the ReLU), giving dz3;
//  3. the third convolution's per-input weight and bias gradient parts and
//     the gradient dg1 of its one-channel input image;
//  4. scatter the first wide convolution's routed gradient (dg1, arg1, w2)
//     the same way into da1, mask by a1 > 0;
//  5. the first convolution's per-input weight and bias gradient parts.
template <class P>
__global__ __launch_bounds__(1024) void k_conv_bwd(
    const void* __restrict__ x, int in_f32, const typename P::T* __restrict__ a1,
    const typename P::T* __restrict__ g1, const int32_t* __restrict__ arg1,
    const typename P::T* __restrict__ a3, const float* __restrict__ dg2,
    const int32_t* __restrict__ arg2, const typename P::T* __restrict__ w2p,
    const float* __restrict__ w3, const typename P::T* __restrict__ w4p,
    float* __restrict__ dg1_out, float* __restrict__ part3, float* __restrict__ part1) {
    __shared__ float da[NPOS * 128];
    __shared__ float img[NPOS];
    __shared__ float gsc[256];
    __shared__ int32_t asc[256];
    __shared__ float dg1s[256];
    __shared__ int32_t hoff[NPOS + 1];     // per position: its (filter, tap) list in ent
    __shared__ int32_t ent[256 * K2 * K2];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t inp = blockIdx.x;
    using T = typename P::T;

    // Scatter of a wide convolution's routed gradient into da: filter f adds
    // dg[f] w[f][i][u][v] at position arg[f] + (u - p, v - p). Each position
    // first lists, in filter order, the (filter, tap) pairs that reach it
    // (thread per position; a block scan turns the counts into offsets); then
    // a wave takes (position, 64 channels) and sums its list in registers, so
    // every da[q][i] is one sum over the filters in order and no two threads
    // write the same element.
    auto scatter = [&](const float* gsrc, const int32_t* asrc, const T* wp, int ks) {
        if (tid < 256) { gsc[tid] = gsrc[tid]; asc[tid] = asrc[tid]; }
        __syncthreads();
        const int p = (ks - 1) / 2, ne = ks * ks * 128;
        int cnt = 0;
        const int qr = tid >> 4, qc = tid & 15;
        if (tid < NPOS)
            for (int f = 0; f < 256; ++f) {
                const int a = asc[f];
                if (a < 0) continue;
                const int u = (qr - (a >> 4) + p) & 15, v = (qc - (a & 15) + p) & 15;
                cnt += (u < ks && v < ks);
            }
        // exclusive prefix of the 256 counts (waves 0-3), offsets in hoff
        int incl = cnt;
        for (int d = 1; d < 64; d <<= 1) {
            const int o = __shfl_up(incl, d, 64);
            if (lane >= d) incl += o;
        }
        if (tid < NPOS && lane == 63) hoff[wave] = incl;   // per-wave totals, briefly
        __syncthreads();
        int wbase = 0;
        for (int w = 0; w < wave && w < 4; ++w) wbase += hoff[w];
        __syncthreads();
        if (tid < NPOS) {
            int o = wbase + incl - cnt;
            hoff[tid] = o;
            if (tid == NPOS - 1) hoff[NPOS] = o + cnt;
            for (int f = 0; f < 256; ++f) {
                const int a = asc[f];
                if (a < 0) continue;
                const int u = (qr - (a >> 4) + p) & 15, v = (qc - (a & 15) + p) & 15;
                if (u < ks && v < ks) ent[o++] = (f << 8) | (u * ks + v);
            }
        }
        __syncthreads();
        for (int task = wave; task < 2 * NPOS; task += 16) {
            const int q = task >> 1, i = ((task & 1) << 6) + lane;
            float acc = 0.0f;
            int e = hoff[q];
            const int e1 = hoff[q + 1];
            // four entries' weights in flight at once, added in list order
            for (; e + 4 <= e1; e += 4) {
                float wv[4], gv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int en = ent[e + u];
                    gv[u] = gsc[en >> 8];
                    wv[u] = P::to_f(wp[(int64_t)(en >> 8) * ne + (en & 255) * 128 + i]);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) acc += gv[u] * wv[u];
            }
            for (; e < e1; ++e) {
                const int en = ent[e];
                acc += gsc[en >> 8] * P::to_f(wp[(int64_t)(en >> 8) * ne + (en & 255) * 128 + i]);
            }
            da[q * 128 + i] = acc;
        }
        __syncthreads();
    };

    // 1-2: second pair
    scatter(dg2 + inp * 256, arg2 + inp * 256, w4p, K2);
    for (int i = tid; i < NPOS * 128; i += 1024)
        if (!(P::to_f(a3[inp * NPOS * 128 + i]) > 0.0f)) da[i] = 0.0f;
    if (tid < 256) img[tid] = P::to_f(g1[inp * 256 + tid]);
    __syncthreads();
    // 3a: conv3 weight and bias parts: element (u, v, f) with f fastest
    {
        float* out = part3 + inp * (F3 * K2 * K2 + F3);
        for (int e = tid; e < K2 * K2 * F3; e += 1024) {
            const int tap = e >> 7, f = e & 127;
            const int u = tap / K2, v = tap - u * K2;
            float a = 0.0f;
            for (int pos = 0; pos < NPOS; ++pos) {
                const int q = wrap16((pos >> 4) + u - 2) * S + wrap16((pos & 15) + v - 2);
                a += da[pos * 128 + f] * img[q];
            }
            out[(f * K2 + u) * K2 + v] = a;
        }
        if (tid < F3) {
            float a = 0.0f;
            for (int pos = 0; pos < NPOS; ++pos) a += da[pos * 128 + tid];
            out[F3 * K2 * K2 + tid] = a;
        }
    }
    // 3b: dg1[q] = sum_f sum_{u,v} dz3[q - (u-2, v-2)][f] w3[f][u][v]; wave w
    // takes q = 16w .. 16w+15, lane l the filters l and l + 64, then a wave sum
    for (int qi = 0; qi < 16; ++qi) {
        const int q = wave * 16 + qi;
        const int qr = q >> 4, qc = q & 15;
        float a = 0.0f;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int f = lane + 64 * h;
            for (int u = 0; u < K2; ++u)
                for (int v = 0; v < K2; ++v) {
                    const int pos = wrap16(qr - u + 2) * S + wrap16(qc - v + 2);
                    a += da[pos * 128 + f] * w3[(f * K2 + u) * K2 + v];
                }
        }
        for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
        if (lane == 0) dg1s[q] = a;
    }
    __syncthreads();
    if (tid < 256) dg1_out[inp * 256 + tid] = dg1s[tid];
    // 4: first pair
    scatter(dg1s, arg1 + inp * 256, w2p, K1);
    for (int i = tid; i < NPOS * 128; i += 1024)
        if (!(P::to_f(a1[inp * NPOS * 128 + i]) > 0.0f)) da[i] = 0.0f;
    if (tid < 256) img[tid] = in_val<P>(x, in_f32, inp * NPOS + tid);
    __syncthreads();
    // 5: conv1 weight and bias parts
    {
        float* out = part1 + inp * (F1 * K1 * K1 + F1);
        for (int e = tid; e < K1 * K1 * F1; e += 1024) {
            const int tap = e >> 7, f = e & 127;
            const int u = tap / K1, v = tap - u * K1;
            float a = 0.0f;
            for (int pos = 0; pos < NPOS; ++pos) {
                const int q = wrap16((pos >> 4) + u - 1) * S + wrap16((pos & 15) + v - 1);
                a += da[pos * 128 + f] * img[q];
            }
            out[(f * K1 + u) * K1 + v] = a;
        }
        if (tid < F1) {
            float a = 0.0f;
            for (int pos = 0; pos < NPOS; ++pos) a += da[pos * 128 + tid];
            out[F1 * K1 * K1 + tid] = a;
        }
    }
}

// ------------------------------------------------------------------ weights

// Working copies from the FP32 masters: wide convolution weights packed
// [f][(u*KS + v)*128 + i] in the working type; every other weight as an FP32
// value rounded to the working precision, biases as they are.
template <class P>
__global__ __launch_bounds__(256) void k_pack_w(const float* __restrict__ m,
                                                typename P::T* __restrict__ w2p,
                                                typename P::T* __restrict__ w4p,
                                                float* __restrict__ rest) {
    const int64_t n2 = (int64_t)F2 * F1 * K1 * K1, n4 = (int64_t)F4 * F3 * K2 * K2;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n2 + n4 + NP;
         e += (int64_t)gridDim.x * 256) {
        if (e < n2) {
            const int f = (int)(e / (K1 * K1 * 128)), r = (int)(e % (K1 * K1 * 128));
            const int tap = r >> 7, i = r & 127, u = tap / K1, v = tap - u * K1;
            w2p[e] = P::from_f(m[W2 + (((int64_t)f * F1 + i) * K1 + u) * K1 + v]);
        } else if (e < n2 + n4) {
            const int64_t e4 = e - n2;
            const int f = (int)(e4 / (K2 * K2 * 128)), r = (int)(e4 % (K2 * K2 * 128));
            const int tap = r >> 7, i = r & 127, u = tap / K2, v = tap - u * K2;
            w4p[e4] = P::from_f(m[W4 + (((int64_t)f * F3 + i) * K2 + u) * K2 + v]);
        } else {
            // weights rounded to the working precision, biases kept FP32
            const int64_t j = e - n2 - n4;
            const bool bias = (j >= B1 && j < W2) || (j >= B2 && j < W3) || (j >= B3 && j < W4) ||
                              (j >= B4 && j < W5) || (j >= B5 && j < W6) || j >= B6;
            rest[j] = bias ? m[j] : P::to_f(P::from_f(m[j]));
        }
    }
}

// Adam on the FP32 masters (bias-corrected; the step's corrections come in).
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ w, float* __restrict__ m,
                                              float* __restrict__ v, const float* __restrict__ g,
                                              int64_t n, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

}  // namespace gpnet

// ------------------------------------------------------------------ host side

struct gpfc_pnet {
    int32_t device = 0;
    int32_t precision = GPFC_CNN_BF16;
    int64_t max_batch = 0;
    int64_t step = 0;
    void* mem = nullptr;          // one allocation for everything below
    float* master = nullptr;      // FP32 parameters
    float* grad = nullptr;
    float* adam_m = nullptr;
    float* adam_v = nullptr;
    float* rest = nullptr;        // FP32 working values of every parameter (flat order)
    void* w2p = nullptr;          // packed wide-convolution weights (working type)
    void* w4p = nullptr;
    void* a1 = nullptr;           // [B][256][128] working type
    void* a3 = nullptr;
    void* g1 = nullptr;           // [B][256] working type
    void* g2 = nullptr;
    int32_t* arg1 = nullptr;      // [B][256]
    int32_t* arg2 = nullptr;
    unsigned long long* key = nullptr;   // [B][256]
    float* h = nullptr;           // [B][128]
    float* dh = nullptr;
    float* dw6p = nullptr;        // [B][128]
    float* dg1 = nullptr;         // [B][256]
    float* dg2 = nullptr;
    float* dz = nullptr;          // [B]
    float* lossp = nullptr;       // [B]
    float* part1 = nullptr;       // [B][1280]
    float* part3 = nullptr;       // [B][3328]
    float* scalar = nullptr;      // the mean loss
    float* cparts = nullptr;      // [64][3328] chunk sums of the per-input gradient parts
    float* dwparts = nullptr;     // [64][F4 K2 K2 F3 + F4] batch-chunk parts of a weight gradient
    bool packed = false;
    bool fused = true;            // bf16: the fused pair kernels (false: layer by layer)
};

namespace {

thread_local char g_pnet_err[256] = "";

int32_t pnet_err(hipError_t e, const char* what) {
    snprintf(g_pnet_err, sizeof(g_pnet_err), "%s: %s", what, hipGetErrorString(e));
    return GPFC_EDEVICE;
}

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

constexpr int kColParts = 64;   // first-stage chunks of a column sum over the batch
constexpr int kDwParts = 64;    // batch chunks of a wide convolution's weight gradient

template <class P>
hipError_t pack(gpfc_pnet* n, hipStream_t s) {
    using T = typename P::T;
    hipLaunchKernelGGL(gpnet::k_pack_w<P>, dim3(2048), dim3(256), 0, s, n->master, (T*)n->w2p,
                       (T*)n->w4p, n->rest);
    return hipGetLastError();
}

hipError_t pack_any(gpfc_pnet* n, hipStream_t s) {
    return n->precision == GPFC_CNN_FP32 ? pack<gcnn::F32>(n, s) : pack<gcnn::BF16>(n, s);
}

// Forward of B inputs (B <= max_batch); keep: dropout mask or NULL;
// training keeps h for the backward pass.
template <class P>
hipError_t forward(gpfc_pnet* n, const void* x, int in_f32, int64_t B, const float* keep,
                   bool training, float* logits, hipStream_t s) {
    using namespace gpnet;
    using T = typename P::T;
    const float* r = n->rest;
    const unsigned nb = (unsigned)B;
    if constexpr (sizeof(T) == 2) {
        if (n->fused) {
            const uint16_t* w2 = (const uint16_t*)n->w2p;
            const uint16_t* w4 = (const uint16_t*)n->w4p;
            uint16_t* g1 = (uint16_t*)n->g1;
            uint16_t* g2 = (uint16_t*)n->g2;
            if (training) {
                hipLaunchKernelGGL((k_pair_bf16<K1, K1, true>), dim3(nb), dim3(kPairThreads), 0, s, x, in_f32,
                                   r + W1, r + B1, w2, r + B2, g1, n->arg1, (uint16_t*)n->a1);
                hipLaunchKernelGGL((k_pair_bf16<K2, K2, true>), dim3(nb), dim3(kPairThreads), 0, s,
                                   (const void*)g1, 0, r + W3, r + B3, w4, r + B4, g2, n->arg2,
                                   (uint16_t*)n->a3);
            } else {
                hipLaunchKernelGGL((k_pair_bf16<K1, K1, false>), dim3(nb), dim3(kPairThreads), 0, s, x, in_f32,
                                   r + W1, r + B1, w2, r + B2, g1, n->arg1, (uint16_t*)nullptr);
                hipLaunchKernelGGL((k_pair_bf16<K2, K2, false>), dim3(nb), dim3(kPairThreads), 0, s,
                                   (const void*)g1, 0, r + W3, r + B3, w4, r + B4, g2, n->arg2,
                                   (uint16_t*)nullptr);
            }
            hipLaunchKernelGGL(k_head<P>, dim3(nb), dim3(128), 0, s, (const T*)n->g2, r + W5, r + B5, r + W6,
                               r + B6, keep, training ? n->h : nullptr, logits);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_conv1ch<P, K1, F1>), dim3(nb), dim3(256), 0, s, x, in_f32, r + W1, r + B1,
                       (T*)n->a1);
    const int64_t nk = B * 256;
    const unsigned fb = (unsigned)std::min<int64_t>((nk + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_u64, dim3(fb), dim3(256), 0, s, n->key, nk);
    const int M = (int)(B * NPOS);
    {
        Conv2DRows<P, K1> la{(const T*)n->a1, M};
        gcnn::Rows<P> lb{(const T*)n->w2p, F2, K1 * K1 * 128, K1 * K1 * 128};
        EpGmax ep{r + B2, n->key};
        hipLaunchKernelGGL((gcnn::k_gemm<P, Conv2DRows<P, K1>, gcnn::Rows<P>, EpGmax>),
                           dim3((unsigned)(M / 64), F2 / 64, 1), dim3(256), 0, s, M, F2,
                           K1 * K1 * 128, K1 * K1 * 128, la, lb, ep);
    }
    hipLaunchKernelGGL(k_gmax_finish<P>, dim3(fb), dim3(256), 0, s, n->key, nk, (T*)n->g1, n->arg1);
    // the pooled values as a one-channel image
    hipLaunchKernelGGL((k_conv1ch<P, K2, F3>), dim3(nb), dim3(256), 0, s, (const void*)n->g1,
                       (int)(sizeof(T) == 4), r + W3, r + B3, (T*)n->a3);
    hipLaunchKernelGGL(k_fill_u64, dim3(fb), dim3(256), 0, s, n->key, nk);
    {
        Conv2DRows<P, K2> la{(const T*)n->a3, M};
        gcnn::Rows<P> lb{(const T*)n->w4p, F4, K2 * K2 * 128, K2 * K2 * 128};
        EpGmax ep{r + B4, n->key};
        hipLaunchKernelGGL((gcnn::k_gemm<P, Conv2DRows<P, K2>, gcnn::Rows<P>, EpGmax>),
                           dim3((unsigned)(M / 64), F4 / 64, 1), dim3(256), 0, s, M, F4,
                           K2 * K2 * 128, K2 * K2 * 128, la, lb, ep);
    }
    hipLaunchKernelGGL(k_gmax_finish<P>, dim3(fb), dim3(256), 0, s, n->key, nk, (T*)n->g2, n->arg2);
    hipLaunchKernelGGL(k_head<P>, dim3(nb), dim3(128), 0, s, (const T*)n->g2, r + W5, r + B5, r + W6,
                       r + B6, keep, training ? n->h : nullptr, logits);
    return hipGetLastError();
}

template <class P>
hipError_t backward(gpfc_pnet* n, const void* x, int in_f32, const float* labels, const float* keep,
                    int64_t B, float* logits_tmp, hipStream_t s) {
    using namespace gpnet;
    using T = typename P::T;
    hipError_t e = forward<P>(n, x, in_f32, B, keep, true, logits_tmp, s);
    if (e != hipSuccess) return e;
    const unsigned nb = (unsigned)B;
    const float* r = n->rest;
    float* g = n->grad;
    hipLaunchKernelGGL(k_head_bwd, dim3(nb), dim3(256), 0, s, logits_tmp, labels, n->h, keep, r + W5,
                       r + W6, B, n->lossp, n->dz, n->dw6p, n->dh, n->dg2);
    // column sums over the batch: fixed chunks summed in order, then the chunks in order
    const int np = (int)std::min<int64_t>(kColParts, B);
    auto colsum = [&](const float* part, int ncol, float* dst, float scale) {
        const unsigned cb = (unsigned)((ncol + 255) / 256);
        hipLaunchKernelGGL(k_colsum_parts, dim3(cb, (unsigned)np), dim3(256), 0, s, part, B, ncol, n->cparts);
        hipLaunchKernelGGL(k_colsum, dim3(cb), dim3(256), 0, s, (const float*)n->cparts, (int64_t)np, ncol,
                           dst, scale);
    };
    colsum(n->lossp, 1, n->scalar, 1.0f / (float)B);
    colsum(n->dw6p, H, g + W6, 1.0f);
    colsum(n->dh, H, g + B5, 1.0f);
    colsum(n->dz, 1, g + B6, 1.0f);
    hipLaunchKernelGGL(k_w5_grad<P>, dim3(H * F4 / 256, (unsigned)np), dim3(256), 0, s, n->dh,
                       (const T*)n->g2, B, n->dwparts);
    hipLaunchKernelGGL(k_colsum, dim3(H * F4 / 256), dim3(256), 0, s, (const float*)n->dwparts, (int64_t)np,
                       H * F4, g + W5, 1.0f);
    // wide convolutions' weight gradients: batch chunks in parallel, then the chunks in order
    const int nd = (int)std::min<int64_t>(kDwParts, B);
    const int n4 = F4 * F3 * K2 * K2 + F4, n2 = F2 * F1 * K1 * K1 + F2;
    hipLaunchKernelGGL((k_wide_dw<P, K2>), dim3(F4, (unsigned)nd), dim3(256), 0, s, (const T*)n->a3, n->dg2,
                       n->arg2, B, n->dwparts, (float*)nullptr);
    hipLaunchKernelGGL(k_colsum, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, s,
                       (const float*)n->dwparts, (int64_t)nd, n4, g + W4, 1.0f);
    hipLaunchKernelGGL(k_conv_bwd<P>, dim3(nb), dim3(1024), 0, s, x, in_f32, (const T*)n->a1,
                       (const T*)n->g1, n->arg1, (const T*)n->a3, n->dg2, n->arg2, (const T*)n->w2p,
                       r + W3, (const T*)n->w4p, n->dg1, n->part3, n->part1);
    hipLaunchKernelGGL((k_wide_dw<P, K1>), dim3(F2, (unsigned)nd), dim3(256), 0, s, (const T*)n->a1, n->dg1,
                       n->arg1, B, n->dwparts, (float*)nullptr);
    hipLaunchKernelGGL(k_colsum, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s,
                       (const float*)n->dwparts, (int64_t)nd, n2, g + W2, 1.0f);
    colsum(n->part3, F3 * K2 * K2 + F3, g + W3, 1.0f);
    colsum(n->part1, F1 * K1 * K1 + F1, g + W1, 1.0f);
    return hipGetLastError();
}

}  // namespace

extern "C" {

int32_t gpfc_pnet_nparams(void) { return (int32_t)gpnet::NP; }

const char* gpfc_pnet_last_error(void) { return g_pnet_err; }

int32_t gpfc_pnet_create(gpfc_pnet** out, int32_t device, int32_t precision, int64_t max_batch) {
    using namespace gpnet;
    if (!out) return GPFC_EINVAL;
    *out = nullptr;
    if (precision != GPFC_CNN_BF16 && precision != GPFC_CNN_FP32) return GPFC_EINVAL;
    if (max_batch < 1 || max_batch > (int64_t(1) << 22)) return GPFC_ERANGE;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return pnet_err(e, "hipGetDeviceCount");
    if (device < 0 || device >= count) return GPFC_EINVAL;
    e = hipSetDevice(device);
    if (e != hipSuccess) return pnet_err(e, "hipSetDevice");
    gpfc_pnet* n = new (std::nothrow) gpfc_pnet();
    if (!n) return GPFC_ENOMEM;
    n->device = device;
    n->precision = precision;
    n->max_batch = max_batch;
    const size_t ts = precision == GPFC_CNN_FP32 ? 4 : 2;
    const int64_t B = max_batch;
    const size_t sizes[] = {
        al256(NP * 4), al256(NP * 4), al256(NP * 4), al256(NP * 4), al256(NP * 4),   // master grad m v rest
        al256((size_t)F2 * F1 * K1 * K1 * ts), al256((size_t)F4 * F3 * K2 * K2 * ts),
        al256((size_t)B * NPOS * 128 * ts), al256((size_t)B * NPOS * 128 * ts),        // a1 a3
        al256((size_t)B * 256 * ts), al256((size_t)B * 256 * ts),                      // g1 g2
        al256((size_t)B * 256 * 4), al256((size_t)B * 256 * 4),                        // arg1 arg2
        al256((size_t)B * 256 * 8),                                                    // key
        al256((size_t)B * H * 4), al256((size_t)B * H * 4), al256((size_t)B * H * 4),  // h dh dw6p
        al256((size_t)B * 256 * 4), al256((size_t)B * 256 * 4),                        // dg1 dg2
        al256((size_t)B * 4), al256((size_t)B * 4),                                    // dz lossp
        al256((size_t)B * (F1 * K1 * K1 + F1) * 4), al256((size_t)B * (F3 * K2 * K2 + F3) * 4),
        256, al256((size_t)kColParts * (F3 * K2 * K2 + F3) * 4),
        al256((size_t)kDwParts * ((size_t)F4 * F3 * K2 * K2 + F4) * 4)};
    size_t total = 0;
    for (size_t z : sizes) total += z;
    e = hipMalloc(&n->mem, total);
    if (e != hipSuccess) {
        delete n;
        return e == hipErrorOutOfMemory ? GPFC_ENOMEM : pnet_err(e, "hipMalloc");
    }
    char* p = (char*)n->mem;
    int i = 0;
    auto take = [&]() { char* q = p; p += sizes[i++]; return (void*)q; };
    n->master = (float*)take();
    n->grad = (float*)take();
    n->adam_m = (float*)take();
    n->adam_v = (float*)take();
    n->rest = (float*)take();
    n->w2p = take();
    n->w4p = take();
    n->a1 = take();
    n->a3 = take();
    n->g1 = take();
    n->g2 = take();
    n->arg1 = (int32_t*)take();
    n->arg2 = (int32_t*)take();
    n->key = (unsigned long long*)take();
    n->h = (float*)take();
    n->dh = (float*)take();
    n->dw6p = (float*)take();
    n->dg1 = (float*)take();
    n->dg2 = (float*)take();
    n->dz = (float*)take();
    n->lossp = (float*)take();
    n->part1 = (float*)take();
    n->part3 = (float*)take();
    n->scalar = (float*)take();
    n->cparts = (float*)take();
    n->dwparts = (float*)take();
    e = hipMemset(n->mem, 0, total);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        (void)hipFree(n->mem);
        delete n;
        return pnet_err(e, "hipMemset");
    }
    *out = n;
    return GPFC_OK;
}

int32_t gpfc_pnet_set_fused(gpfc_pnet* n, int32_t on) {
    if (!n || on < 0 || on > 1) return GPFC_EINVAL;
    n->fused = on != 0;
    return GPFC_OK;
}

int32_t gpfc_pnet_destroy(gpfc_pnet* n) {
    if (!n) return GPFC_OK;
    (void)hipSetDevice(n->device);
    (void)hipDeviceSynchronize();
    if (n->mem) (void)hipFree(n->mem);
    delete n;
    return GPFC_OK;
}

int32_t gpfc_pnet_set_params(gpfc_pnet* n, const float* params, void* stream) {
    if (!n || !params) return GPFC_EINVAL;
    hipError_t e = hipSetDevice(n->device);
    hipStream_t s = (hipStream_t)stream;
    if (e == hipSuccess)
        e = hipMemcpyAsync(n->master, params, sizeof(float) * gpnet::NP, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(n->adam_m, 0, sizeof(float) * gpnet::NP, s);
    if (e == hipSuccess) e = hipMemsetAsync(n->adam_v, 0, sizeof(float) * gpnet::NP, s);
    if (e == hipSuccess) e = pack_any(n, s);
    if (e != hipSuccess) return pnet_err(e, "gpfc_pnet_set_params");
    n->step = 0;
    n->packed = true;
    return GPFC_OK;
}

int32_t gpfc_pnet_get_params(gpfc_pnet* n, float* params, void* stream) {
    if (!n || !params) return GPFC_EINVAL;
    hipError_t e = hipSetDevice(n->device);
    if (e == hipSuccess)
        e = hipMemcpyAsync(params, n->master, sizeof(float) * gpnet::NP, hipMemcpyDeviceToDevice,
                           (hipStream_t)stream);
    return e == hipSuccess ? GPFC_OK : pnet_err(e, "gpfc_pnet_get_params");
}

int32_t gpfc_pnet_get_grads(gpfc_pnet* n, float* grads, void* stream) {
    if (!n || !grads) return GPFC_EINVAL;
    hipError_t e = hipSetDevice(n->device);
    if (e == hipSuccess)
        e = hipMemcpyAsync(grads, n->grad, sizeof(float) * gpnet::NP, hipMemcpyDeviceToDevice,
                           (hipStream_t)stream);
    return e == hipSuccess ? GPFC_OK : pnet_err(e, "gpfc_pnet_get_grads");
}

int32_t gpfc_pnet_forward(gpfc_pnet* n, const void* x, int32_t x_f32, int64_t batch, float* logits,
                          void* stream) {
    if (!n || batch < 0 || (batch > 0 && (!x || !logits))) return GPFC_EINVAL;
    if (!n->packed) return GPFC_EINVAL;
    hipError_t e = hipSetDevice(n->device);
    if (e != hipSuccess) return pnet_err(e, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    for (int64_t b0 = 0; b0 < batch && e == hipSuccess; b0 += n->max_batch) {
        const int64_t B = std::min(n->max_batch, batch - b0);
        const void* xb = x_f32 ? (const void*)((const float*)x + b0 * gpnet::NPOS)
                               : (const void*)((const uint16_t*)x + b0 * gpnet::NPOS);
        e = n->precision == GPFC_CNN_FP32
                ? forward<gcnn::F32>(n, xb, x_f32, B, nullptr, false, logits + b0, s)
                : forward<gcnn::BF16>(n, xb, x_f32, B, nullptr, false, logits + b0, s);
    }
    return e == hipSuccess ? GPFC_OK : pnet_err(e, "gpfc_pnet_forward");
}

int32_t gpfc_pnet_backward(gpfc_pnet* n, const void* x, int32_t x_f32, const float* labels,
                           const float* keep, int64_t batch, float* logits, float* loss,
                           void* stream) {
    if (!n || !x || !labels || !logits || batch < 1) return GPFC_EINVAL;
    if (!n->packed) return GPFC_EINVAL;
    if (batch > n->max_batch) return GPFC_ERANGE;
    hipError_t e = hipSetDevice(n->device);
    if (e != hipSuccess) return pnet_err(e, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    e = n->precision == GPFC_CNN_FP32
            ? backward<gcnn::F32>(n, x, x_f32, labels, keep, batch, logits, s)
            : backward<gcnn::BF16>(n, x, x_f32, labels, keep, batch, logits, s);
    if (e == hipSuccess && loss)
        e = hipMemcpyAsync(loss, n->scalar, sizeof(float), hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? GPFC_OK : pnet_err(e, "gpfc_pnet_backward");
}

int32_t gpfc_pnet_adam(gpfc_pnet* n, float lr, float beta1, float beta2, float eps, void* stream) {
    if (!n || !(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps > 0.0f))
        return GPFC_EINVAL;
    hipError_t e = hipSetDevice(n->device);
    if (e != hipSuccess) return pnet_err(e, "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    n->step += 1;
    const float c1 = 1.0f - powf(beta1, (float)n->step), c2 = 1.0f - powf(beta2, (float)n->step);
    hipLaunchKernelGGL(gpnet::k_adam, dim3(2048), dim3(256), 0, s, n->master, n->adam_m, n->adam_v,
                       n->grad, (int64_t)gpnet::NP, lr, beta1, beta2, eps, c1, c2);
    e = hipGetLastError();
    if (e == hipSuccess) e = pack_any(n, s);
    return e == hipSuccess ? GPFC_OK : pnet_err(e, "gpfc_pnet_adam");
}

}  // extern "C"
