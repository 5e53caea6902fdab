// Measurement kernel for the benchmark: a plain device-to-device copy with
// 128-bit loads and stores, the ceiling the dump kernel's HBM rate is
// compared with. Not part of the checkpoint path; built into its own
// library (libmkcopy.so).
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef unsigned int v4u __attribute__((ext_vector_type(4)));

// Copy of n16 16-byte blocks in tiles of U * blockDim blocks: work-group b
// copies tiles b, b + grid, ...; within a tile, load u of thread t takes
// block u * blockDim + t, so every load instruction of a wave is one
// contiguous 1 KiB and a tile is one contiguous stretch of HBM. U loads are
// in flight per thread before the stores.
template <int U, bool NT>
__global__ void k_copy(v4u* __restrict__ dst, const v4u* __restrict__ src, uint64_t n16) {
    const uint64_t tile = (uint64_t)U * blockDim.x;
    const uint64_t full = n16 / tile;
    for (uint64_t b = blockIdx.x; b < full; b += gridDim.x) {
        const uint64_t base = b * tile + threadIdx.x;
        v4u x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) x[u] = src[base + (uint64_t)u * blockDim.x];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (NT) __builtin_nontemporal_store(x[u], &dst[base + (uint64_t)u * blockDim.x]);
            else dst[base + (uint64_t)u * blockDim.x] = x[u];
        }
    }
    // the blocks past the last whole tile
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = full * tile + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        dst[i] = src[i];
}

}  // namespace

// Copies n bytes (a multiple of 16, both pointers 16-byte aligned) reps
// times with the given launch shape; *best_ms = the fastest copy, timed by
// HIP events on a stream of its own. nt: bit 0 non-temporal stores, bit 1
// eight loads in flight per thread instead of four. Returns a hipError_t.
extern "C" int mkcopy_run(void* dst, const void* src, uint64_t n, int blocks, int threads, int nt, int reps,
                          float* best_ms) {
    if (!dst || !src || (n & 15) || blocks <= 0 || threads <= 0 || threads > 1024 || reps <= 0 || !best_ms)
        return (int)hipErrorInvalidValue;
    hipStream_t s;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) return (int)e;
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    float best = 1e30f;
    for (int r = 0; r < reps + 1 && e == hipSuccess; ++r) {
        (void)hipEventRecord(a, s);
        v4u* d = static_cast<v4u*>(dst);
        const v4u* q = static_cast<const v4u*>(src);
        switch (nt) {   // bit 0: non-temporal stores; bit 1: 8 loads in flight per thread (else 4)
            case 0: hipLaunchKernelGGL((k_copy<4, false>), dim3(blocks), dim3(threads), 0, s, d, q, n / 16); break;
            case 1: hipLaunchKernelGGL((k_copy<4, true>), dim3(blocks), dim3(threads), 0, s, d, q, n / 16); break;
            case 2: hipLaunchKernelGGL((k_copy<8, false>), dim3(blocks), dim3(threads), 0, s, d, q, n / 16); break;
            default: hipLaunchKernelGGL((k_copy<8, true>), dim3(blocks), dim3(threads), 0, s, d, q, n / 16); break;
        }
        e = hipGetLastError();
        (void)hipEventRecord(b, s);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0;
        if (e == hipSuccess && r > 0 && hipEventElapsedTime(&ms, a, b) == hipSuccess && ms < best) best = ms;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipStreamDestroy(s);
    *best_ms = best;
    return (int)e;
}
