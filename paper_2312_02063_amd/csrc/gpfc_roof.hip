// Micro-benchmarks that measure the roofline denominators of the fold on the
// running GPU: conflict-free LDS integer atomics (the fold's one operation
// per sample-period update), float LDS atomics (the FP32 precision-study
// fold), dependent-free FP64 FMAs (the phase product) and an HBM copy. They
// are the measured counterpart of the runtime breakdown the paper tabulates
// for its own GPU (Sec. 2.4, Table 1).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gpfc.h"

namespace {

constexpr int kThreads = 1024;
constexpr int kSlots = 16384;          // 128 KB of 64-bit slots (the fold's histogram size)

// Every lane adds to its own slot in the fold's layout: rows of 32 lanes x
// 8 bytes, two halves of 64 KB, so the 16 lanes of one 64-bit pass touch 32
// distinct banks. Rows advance each step; 8 independent atomics per step.
template <typename T>
__global__ __launch_bounds__(kThreads, 1) void k_roof_lds(int iters, T* __restrict__ out) {
    __shared__ __attribute__((aligned(16))) uint64_t h64[kSlots];
    T* h = reinterpret_cast<T*>(h64);
    constexpr int rowlen = 256 / (int)sizeof(T);      // slots of a 256-byte row
    constexpr int half = kSlots * 8 / 2 / (int)sizeof(T);
    for (int i = threadIdx.x; i < kSlots * 8 / (int)sizeof(T); i += kThreads) h[i] = T(0);
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int laneoff = sizeof(T) == 8 ? (lane & 31) + (lane >> 5) * half : lane;
    const int rows = sizeof(T) == 8 ? 256 : kSlots * 8 / 256;
    int r = wave * 16;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int row = (r + j) & (rows - 1);
            __hip_atomic_fetch_add(h + row * rowlen + laneoff, T(1), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        r += 8;
    }
    __syncthreads();
    out[(int64_t)blockIdx.x * kThreads + threadIdx.x] = h[threadIdx.x];
}

// 8 independent FMA chains per lane (x <- x * a + b with a, b near 1 and 0).
__global__ __launch_bounds__(256) void k_roof_fp64(int iters, double a, double b,
                                                   double* __restrict__ out) {
    double x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = 1.0 + 1e-3 * (threadIdx.x + j);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 8; ++j) x[j] = __builtin_fma(x[j], a, b);
    }
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += x[j];
    out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

// Streaming copy with 16-byte loads and stores.
__global__ __launch_bounds__(256) void k_roof_copy(const uint4* __restrict__ src,
                                                   uint4* __restrict__ dst, int64_t n16) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n16;
         i += (int64_t)gridDim.x * 256)
        dst[i] = src[i];
}

template <class F>
hipError_t time_ms(hipStream_t s, int reps, F launch, float* ms) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) { launch(); e = hipGetLastError(); }   // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) { launch(); e = hipGetLastError(); }
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    if (e == hipSuccess) *ms /= (float)reps;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return e;
}

}  // namespace

extern "C" int32_t gpfc_roof_probe(int32_t device, int32_t kind, double* rate_out, double* ms_out,
                                   void* stream) {
    if (!rate_out || kind < GPFC_ROOF_LDS_U64 || kind > GPFC_ROOF_HBM_COPY) return GPFC_EINVAL;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return GPFC_EDEVICE;
    if (device < 0 || device >= count) return GPFC_EINVAL;
    e = hipSetDevice(device);
    if (e != hipSuccess) return GPFC_EDEVICE;
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return GPFC_EDEVICE;
    const int cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 1;
    hipStream_t s = (hipStream_t)stream;
    float ms = 0.0f;
    double work = 0.0;
    void* buf = nullptr;
    void* buf2 = nullptr;
    if (kind == GPFC_ROOF_LDS_U64 || kind == GPFC_ROOF_LDS_U32 || kind == GPFC_ROOF_LDS_F32) {
        const int blocks = 4 * cus;
        const int iters = kind == GPFC_ROOF_LDS_F32 ? 256 : 4096;
        e = hipMalloc(&buf, (size_t)blocks * kThreads * 8);
        if (e == hipSuccess) {
            if (kind == GPFC_ROOF_LDS_U64)
                e = time_ms(s, 5, [&] { hipLaunchKernelGGL(k_roof_lds<unsigned long long>, dim3(blocks),
                                                           dim3(kThreads), 0, s, iters,
                                                           (unsigned long long*)buf); }, &ms);
            else if (kind == GPFC_ROOF_LDS_U32)
                e = time_ms(s, 5, [&] { hipLaunchKernelGGL(k_roof_lds<uint32_t>, dim3(blocks),
                                                           dim3(kThreads), 0, s, iters,
                                                           (uint32_t*)buf); }, &ms);
            else
                e = time_ms(s, 5, [&] { hipLaunchKernelGGL(k_roof_lds<float>, dim3(blocks),
                                                           dim3(kThreads), 0, s, iters,
                                                           (float*)buf); }, &ms);
        }
        work = (double)blocks * kThreads * iters * 8;          // lane-atomics
    } else if (kind == GPFC_ROOF_FP64_FMA) {
        const int blocks = 64 * cus, iters = 4096;
        e = hipMalloc(&buf, (size_t)blocks * 256 * 8);
        if (e == hipSuccess)
            e = time_ms(s, 5, [&] { hipLaunchKernelGGL(k_roof_fp64, dim3(blocks), dim3(256), 0, s,
                                                       iters, 0.9999999, 1e-7, (double*)buf); }, &ms);
        work = (double)blocks * 256 * iters * 8 * 2;           // flops
    } else {
        const int64_t bytes = int64_t(1) << 30;
        e = hipMalloc(&buf, (size_t)bytes);
        if (e == hipSuccess) e = hipMalloc(&buf2, (size_t)bytes);
        if (e == hipSuccess) e = hipMemsetAsync(buf, 0, (size_t)bytes, s);
        if (e == hipSuccess)
            e = time_ms(s, 5, [&] { hipLaunchKernelGGL(k_roof_copy, dim3(16 * cus), dim3(256), 0, s,
                                                       (const uint4*)buf, (uint4*)buf2, bytes / 16); },
                        &ms);
        work = 2.0 * (double)bytes;                            // bytes read + written
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (buf) (void)hipFree(buf);
    if (buf2) (void)hipFree(buf2);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? GPFC_ENOMEM : GPFC_EDEVICE;
    *rate_out = work / ((double)ms * 1e-3);
    if (ms_out) *ms_out = ms;
    return GPFC_OK;
}
