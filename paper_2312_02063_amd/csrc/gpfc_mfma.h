// Matrix-core building blocks shared by the networks on gfx950: bf16 and
// OCP FP8 E4M3 conversions, the element types of working copies (bf16, FP32,
// FP8), and a generic MFMA GEMM whose operands come from loader objects and
// whose tile results go to an epilogue object.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gcnn {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4v __attribute__((ext_vector_type(4)));

// A 16-byte load as a value. Assigning *reinterpret_cast<const uint4*>(p) to
// an array element copies the struct with a memcpy that keeps the array in
// scratch memory; loading a vector and rebuilding the uint4 does not.
__device__ __forceinline__ uint4 ld_u4(const void* p) {
    const u32x4v v = *reinterpret_cast<const u32x4v*>(p);
    return make_uint4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// Round to nearest even bfloat16, NaN kept NaN: gfx950's v_cvt_pk_bf16_f32,
// which gives the same bits as rounding the bit pattern (u + 0x7fff + lsb)
// for every finite value and sets the quiet bit of a NaN (checked against
// that rounding on 2^24 patterns: ties, denormals, overflow, NaNs).
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef float f32x2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
// Two values rounded as f2bf, lo in bits 0-15 and hi in bits 16-31 (one instruction).
__device__ __forceinline__ uint32_t f2bf2(float lo, float hi) {
    const f32x2v v = {lo, hi};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2v));
}

// Element types of the working copies and activations.
struct BF16 {
    using T = uint16_t;
    static constexpr int KSTEP = 32;   // K per MFMA
    static __device__ __forceinline__ float to_f(T v) { return bf2f(v); }
    static __device__ __forceinline__ T from_f(float v) { return f2bf(v); }
};
struct F32 {
    using T = float;
    static constexpr int KSTEP = 4;
    static __device__ __forceinline__ float to_f(T v) { return v; }
    static __device__ __forceinline__ T from_f(float v) { return v; }
};

// OCP FP8 E4M3 (bias 7, max 448, no infinities): round to nearest even,
// saturating at +-448; |f| < 2^-6 goes to the subnormals m * 2^-9.
__device__ __forceinline__ uint8_t f2e4m3(float f) {
    const uint32_t u = __float_as_uint(f);
    const uint8_t sign = (uint8_t)((u >> 24) & 0x80);
    const float a = fabsf(f);
    if (!(a < 448.0f)) return (uint8_t)(sign | 0x7E);   // saturate (NaN too)
    if (a < 0.015625f) return (uint8_t)(sign | (uint8_t)rintf(a * 512.0f));
    uint32_t v = __float_as_uint(a);
    v += 0x7FFFFu + ((v >> 20) & 1u);                     // RNE to 3 mantissa bits
    uint32_t code = (v >> 20) - ((127u - 7u) << 3);
    if (code > 0x7Eu) code = 0x7Eu;
    return (uint8_t)(sign | code);
}

// Inference with FP8 E4M3 operands: activations (kept as bf16) are scaled by
// a per-layer factor and rounded to E4M3 as they are loaded; weights are
// pre-rounded with one scale per output channel; the epilogue multiplies the
// FP32 accumulator back by both scales.
struct FP8 {
    using T = uint16_t;
    static constexpr int KSTEP = 32;
    static __device__ __forceinline__ float to_f(T v) { return bf2f(v); }
    static __device__ __forceinline__ T from_f(float v) { return f2bf(v); }
};

// ------------------------------------------------------------------ generic MFMA GEMM
//
// C[m][n] = sum_k A(m, k) * B(n, k); A and B are given by loaders that fill
// a lane's fragment: for bf16, 8 values at k .. k+7 of one row; for f32, one
// value. One wave computes a 32 x 32 tile (2 x 2 MFMA accumulators), four
// waves a 64 x 64 tile. The epilogue receives (m, n, acc) for every element
// of the tile inside [0, M) x [0, N).

template <class P, class LA, class LB, class EP>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, int kchunk, LA la, LB lb, EP ep) {
    // split K: block z sums k in [z * kchunk, min(K, (z + 1) * kchunk))
    const int kb = blockIdx.z * kchunk;
    const int ke = min(K, kb + kchunk);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int m0 = blockIdx.x * 64 + (wave & 1) * 32;
    const int n0 = blockIdx.y * 64 + (wave >> 1) * 32;
    const int r = lane & 15;
    const int q = lane >> 4;
    f32x4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = kb; k0 < ke; k0 += P::KSTEP) {
        if constexpr (__is_same(P, FP8)) {
            const int kk = k0 + q * 8;
            long a[2], b[2];
            for (int i = 0; i < 2; ++i) a[i] = la.frag8q(m0 + i * 16 + r, kk);
            for (int j = 0; j < 2; ++j) b[j] = lb.frag8q(n0 + j * 16 + r, kk);
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a[i], b[j], acc[i][j], 0, 0, 0);
        } else if constexpr (P::KSTEP == 32) {
            const int kk = k0 + q * 8;
            bf16x8 a[2], b[2];
            for (int i = 0; i < 2; ++i) a[i] = la.frag8(m0 + i * 16 + r, kk);
            for (int j = 0; j < 2; ++j) b[j] = lb.frag8(n0 + j * 16 + r, kk);
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        } else {
            const int kk = k0 + q;
            float a[2], b[2];
            for (int i = 0; i < 2; ++i) a[i] = la.frag1(m0 + i * 16 + r, kk);
            for (int j = 0; j < 2; ++j) b[j] = lb.frag1(n0 + j * 16 + r, kk);
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + j * 16 + r;
            const int mb = m0 + i * 16 + q * 4;
            ep(mb, n, acc[i][j], M, N);
        }
}

// Loader helpers: a row of `ld` elements of type T at p, k-range checked.
template <class P>
struct Rows {
    using T = typename P::T;
    const T* p;
    int rows, ld, K;
    __device__ __forceinline__ bf16x8 frag8(int m, int k) const {
        bf16x8 v;
        if (m < rows && k + 8 <= K) {
            v = *reinterpret_cast<const bf16x8*>(reinterpret_cast<const uint16_t*>(p) + (int64_t)m * ld + k);
        } else {
            for (int j = 0; j < 8; ++j) {
                uint16_t h = (m < rows && k + j < K) ? reinterpret_cast<const uint16_t*>(p)[(int64_t)m * ld + k + j] : 0;
                v[j] = __builtin_bit_cast(__bf16, h);
            }
        }
        return v;
    }
    __device__ __forceinline__ float frag1(int m, int k) const {
        return (m < rows && k < K) ? P::to_f(p[(int64_t)m * ld + k]) : 0.0f;
    }
};

// Strided operand: element (m, k) at p[k * ld + m] (k-major storage).
template <class P>
struct Cols {
    using T = typename P::T;
    const T* p;
    int rows, ld, K;
    __device__ __forceinline__ bf16x8 frag8(int m, int k) const {
        const uint16_t* q = reinterpret_cast<const uint16_t*>(p) + (int64_t)k * ld + m;
        u16x8 h;
        if (m < rows && k + 8 <= K) {
            for (int j = 0; j < 8; ++j) h[j] = q[(int64_t)j * ld];
        } else {
            for (int j = 0; j < 8; ++j) h[j] = (m < rows && k + j < K) ? q[(int64_t)j * ld] : (uint16_t)0;
        }
        return __builtin_bit_cast(bf16x8, h);
    }
    __device__ __forceinline__ float frag1(int m, int k) const {
        return (m < rows && k < K) ? P::to_f(p[(int64_t)k * ld + m]) : 0.0f;
    }
};

}  // namespace gcnn
