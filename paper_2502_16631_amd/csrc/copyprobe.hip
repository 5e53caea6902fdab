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

// Copy of 64 KiB chunks by persistent work-groups of 512 threads that take
// chunk tickets from a counter: per chunk, eight rows of 8 KiB, each one
// 128-bit load per thread, then eight stores.
template <bool NT>
__global__ void __launch_bounds__(512) k_copy_chunks(v4u* __restrict__ dst, const v4u* __restrict__ src,
                                                     uint32_t n_chunks, uint32_t* ticket) {
    constexpr uint32_t T = 512, K = 8;
    __shared__ uint32_t s_t;
    for (;;) {
        if (threadIdx.x == 0) s_t = atomicAdd(ticket, 1u);
        __syncthreads();
        const uint32_t c = s_t;
        __syncthreads();
        if (c >= n_chunks) break;
        const uint64_t base = (uint64_t)c * (T * K) + threadIdx.x;
        v4u x[K];
#pragma unroll
        for (uint32_t r = 0; r < K; ++r) x[r] = src[base + r * T];
#pragma unroll
        for (uint32_t r = 0; r < K; ++r) {
            if (NT) __builtin_nontemporal_store(x[r], &dst[base + r * T]);
            else dst[base + r * T] = x[r];
        }
    }
}

}  // namespace

// Copies n bytes (a multiple of 16, both pointers 16-byte aligned) reps
// times with the given launch shape; *best_ms = the fastest copy, timed by
// HIP events on a stream of its own. nt: bit 0 non-temporal stores, bit 1
// eight loads in flight per thread instead of four, bit 2 the ticketed
// 64 KiB-chunk copy (threads must be 512 and n a multiple of 64 KiB).
// Returns a hipError_t.
extern "C" int mkcopy_run(void* dst, const void* src, uint64_t n, int blocks, int threads, int nt, int reps,
                          float* best_ms) {
    if (!dst || !src || (n & 15) || blocks <= 0 || threads <= 0 || threads > 1024 || reps <= 0 || !best_ms)
        return (int)hipErrorInvalidValue;
    const bool chunks = (nt & 4) != 0;
    if (chunks && (threads != 512 || (n & 65535) || n / 65536 > 0xFFFFFFFFull)) return (int)hipErrorInvalidValue;
    uint32_t* ticket = nullptr;
    hipStream_t s;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) return (int)e;
    if (chunks && (e = hipMalloc(&ticket, sizeof(uint32_t))) != hipSuccess) {
        (void)hipStreamDestroy(s);
        return (int)e;
    }
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    float best = 1e30f;
    for (int r = 0; r < reps + 1 && e == hipSuccess; ++r) {
        v4u* d = static_cast<v4u*>(dst);
        const v4u* q = static_cast<const v4u*>(src);
        if (chunks) {
            e = hipMemsetAsync(ticket, 0, sizeof(uint32_t), s);
            if (e != hipSuccess) break;
            (void)hipEventRecord(a, s);
            if (nt & 1) hipLaunchKernelGGL((k_copy_chunks<true>), dim3(blocks), dim3(512), 0, s, d, q, (uint32_t)(n / 65536), ticket);
            else hipLaunchKernelGGL((k_copy_chunks<false>), dim3(blocks), dim3(512), 0, s, d, q, (uint32_t)(n / 65536), ticket);
        } else {
            (void)hipEventRecord(a, s);
            switch (nt & 3) {   // bit 0: non-temporal stores; bit 1: 8 loads in flight per thread (else 4)
                case 0: hipLaunchKernelGGL((k_copy<4, false>), dim3(blocks), dim3(threads), 0, s, d, q, n / 16); break;
                case 1: hipLaunchKernelGGL((k_copy<4, true>), dim3(blocks), dim3(threads), 0, s, d, q, n / 16); break;
                case 2: hipLaunchKernelGGL((k_copy<8, false>), dim3(blocks), dim3(threads), 0, s, d, q, n / 16); break;
                default: hipLaunchKernelGGL((k_copy<8, true>), dim3(blocks), dim3(threads), 0, s, d, q, n / 16); break;
            }
        }
        e = hipGetLastError();
        (void)hipEventRecord(b, s);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0;
        if (e == hipSuccess && r > 0 && hipEventElapsedTime(&ms, a, b) == hipSuccess && ms < best) best = ms;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipStreamSynchronize(s);
    if (ticket) (void)hipFree(ticket);
    (void)hipStreamDestroy(s);
    *best_ms = best;
    return (int)e;
}
