// DATA chunks to their payload records (see gather.h).
#include <hip/hip_runtime.h>

#include "gather.h"

namespace mk {
namespace {

constexpr int NT = 256;

__global__ void __launch_bounds__(NT) k_gather(GatherJob j) {
    const int tid = threadIdx.x;
    const uint32_t C = j.C;
    for (uint64_t g = j.g0 + blockIdx.x; g < j.g1; g += gridDim.x) {
        if (j.kind[g] != kData) continue;   // the same on every lane
        const AllocDesc ad = j.allocs[j.amap[g]];
        const uint64_t k = g - ad.first;
        const uint64_t nk = (ad.size + C - 1) / C;
        const uint32_t len = (k + 1 == nk) ? ad.tail_len : C;
        const uint4* src = reinterpret_cast<const uint4*>(ad.ptr + k * C);
        uint4* dst = reinterpret_cast<uint4*>(j.slot + (j.off[g] - j.slot_base));
        const uint32_t full = len / 16, rem = len % 16;
#pragma unroll 4
        for (uint32_t i = tid; i < full; i += NT) dst[i] = src[i];
        if (rem && tid == 0) {
            const uint8_t* sb = reinterpret_cast<const uint8_t*>(src + full);
            uint32_t w[4] = {0, 0, 0, 0};
            for (uint32_t b = 0; b < rem; ++b) w[b >> 2] |= (uint32_t)sb[b] << (8 * (b & 3));
            dst[full] = make_uint4(w[0], w[1], w[2], w[3]);
        }
    }
}

}  // namespace

hipError_t launch_gather(const GatherJob& j, int grid, hipStream_t s) {
    if (!j.amap || grid < 1) return hipErrorInvalidValue;
    if (j.g1 <= j.g0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3(grid), dim3(NT), 0, s, j);
    return hipGetLastError();
}

}  // namespace mk
