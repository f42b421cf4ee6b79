// LDS atomic-add microbenchmark (include/sindi_probe.h): the rate at which
// gfx950 applies workgroup-local atomic adds, for lane address patterns from
// conflict-free to the random scatter of postings into a score tile (the
// accumulate step of Alg. 2, Sec. 3.2).  Measurement only.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "sindi_probe.h"

namespace {

constexpr uint32_t kWords = 12288;  // 48 KB: three workgroups per compute unit
constexpr uint32_t kMask = 8191;    // addresses stay in the first 8192 words
constexpr int kThreads = 512;
constexpr int kSlots = 8;           // independent adds in flight per thread

// A fixed integer hash (the finalizer of MurmurHash3, Appleby), for the
// random pattern's addresses.
__device__ __forceinline__ uint32_t mix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

template <int OP>
__global__ __launch_bounds__(kThreads) void k_lds_add(int32_t stride, int32_t iters, uint32_t *sink)
{
    __shared__ uint32_t a[kWords];
    for (uint32_t i = threadIdx.x; i < kWords; i += kThreads) a[i] = 0u;
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    uint32_t addr[kSlots];
#pragma unroll
    for (int j = 0; j < kSlots; ++j) {
        if (stride == 0)
            addr[j] = mix32((blockIdx.x * kThreads + threadIdx.x) * kSlots + j) & kMask;
        else
            addr[j] = (lane * (uint32_t)stride + (wave * kSlots + j) * 64u * (uint32_t)stride) & kMask;
    }
    for (int32_t it = 0; it < iters; ++it) {
        const uint32_t off = (uint32_t)it * 97u;  // moves every lane alike: bank sharing is kept
#pragma unroll
        for (int j = 0; j < kSlots; ++j) {
            const uint32_t w = (addr[j] + off) & kMask;
            if (OP == 0)
                __hip_atomic_fetch_add(&a[w], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            else
                __hip_atomic_fetch_add(reinterpret_cast<float *>(&a[w]), 1.0f, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    __syncthreads();
    if (a[threadIdx.x] == 0x7FFFFFFFu) *sink = 1u;  // keeps the adds observable
}

}  // namespace

extern "C" int sindi_probe_lds_add(int32_t op, int32_t stride, int32_t n_workgroups, int32_t iters,
                                   void *stream, double *ms, double *updates)
{
    if ((op != 0 && op != 1) || stride < 0 || stride > 4096 || n_workgroups < 1 ||
        n_workgroups > (1 << 20) || iters < 1 || iters > 1000000 || !ms || !updates)
        return (int)hipErrorInvalidValue;
    hipStream_t s = (hipStream_t)stream;
    uint32_t *sink = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipMalloc(&sink, sizeof(uint32_t));
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = hipEventRecord(a, s);
    if (e == hipSuccess) {
        if (op == 0)
            hipLaunchKernelGGL(k_lds_add<0>, dim3((unsigned)n_workgroups), dim3(kThreads), 0, s,
                               stride, iters, sink);
        else
            hipLaunchKernelGGL(k_lds_add<1>, dim3((unsigned)n_workgroups), dim3(kThreads), 0, s,
                               stride, iters, sink);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    if (e == hipSuccess) {
        *ms = t;
        *updates = (double)n_workgroups * kThreads * (double)iters * kSlots;
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (sink) (void)hipFree(sink);
    return (int)e;
}
