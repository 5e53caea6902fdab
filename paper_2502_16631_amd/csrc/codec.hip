// Byte-plane codec kernels (see codec.h for the record layout).
#include <hip/hip_runtime.h>

#include "codec.h"
#include "hostmath.h"

namespace mk {
namespace {

constexpr int NT = kCodecThreads;
constexpr int NW = NT / 64;

__host__ __device__ inline uint32_t r16(uint32_t n) { return (n + 15u) & ~15u; }

__host__ __device__ inline uint32_t section_len(uint32_t L, uint32_t mode, uint32_t esc) {
    return mode == kPlaneConst ? 16u : mode == kPlaneDict ? 16u + r16(L / 2) + r16(esc) : r16(L);
}

// byte j (0..15) of a 16-byte row
__device__ inline uint32_t byte_of(const uint4& v, int j) {
    const uint32_t w = j < 4 ? v.x : j < 8 ? v.y : j < 12 ? v.z : v.w;
    return (w >> (8 * (j & 3))) & 255u;
}

__device__ inline uint32_t wave_max(uint32_t v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = max(v, (uint32_t)__shfl_xor(v, m));
    return v;
}

// Exclusive block scan of two u64 values (each holds four 16-bit counters
// that never carry into each other); ta / tb are the block totals.
__device__ inline void block_scan2(uint64_t& a, uint64_t& b, unsigned long long* s_w, uint64_t& ta, uint64_t& tb) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    unsigned long long ia = a, ib = b;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned long long xa = __shfl_up(ia, d), xb = __shfl_up(ib, d);
        if (lane >= d) {
            ia += xa;
            ib += xb;
        }
    }
    if (lane == 63) {
        s_w[2 * w] = ia;
        s_w[2 * w + 1] = ib;
    }
    __syncthreads();
    uint64_t pa = 0, pb = 0;
    ta = 0;
    tb = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        const uint64_t wa = s_w[2 * i], wb = s_w[2 * i + 1];
        if (i < w) {
            pa += wa;
            pb += wb;
        }
        ta += wa;
        tb += wb;
    }
    a = pa + ia - a;
    b = pb + ib - b;
}

__device__ inline uint32_t field16(uint64_t a, uint64_t b, int p) {
    return (uint32_t)(((p < 4 ? a : b) >> (16 * (p & 3))) & 0xFFFFu);
}

// Size pass (ENCODE false): the record length of every full DATA chunk; the
// chunk becomes PACKED when it is shorter than C. Encode pass: the record of
// every PACKED chunk, built in LDS and copied to its payload offset.
template <int K, bool ENCODE>
__global__ void __launch_bounds__(NT) k_pack(PackJob j) {
    __shared__ uint32_t s_hist[8 * 256];
    __shared__ uint8_t s_code[8 * 256];
    __shared__ uint8_t s_dict[8 * 16];
    __shared__ uint32_t s_mode[8], s_esc[8], s_nused[8], s_sec[9];
    __shared__ unsigned long long s_w[2 * NW];
    __shared__ uint4 s_rec[ENCODE ? kCodecMaxChunk / 16 : 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t C = j.C, L = C / 8;
    for (uint64_t g = j.g0 + blockIdx.x; g < j.g1; g += gridDim.x) {
        __syncthreads();   // the previous chunk's LDS is no longer read
        const uint8_t kd = j.kind[g];
        const AllocDesc ad = j.allocs[j.amap[g]];
        const uint64_t k = g - ad.first;
        const uint64_t nk = (ad.size + C - 1) / C;
        const uint32_t len = (k + 1 == nk) ? ad.tail_len : C;
        if constexpr (!ENCODE) {
            if (kd != kData || len != C) {
                if (tid == 0) j.rlen[g] = kd == kData ? r16(len) : 0u;
                continue;
            }
        } else {
            if (kd != kPacked) continue;
        }
        const uint4* src = reinterpret_cast<const uint4*>(ad.ptr + k * C) + (uint32_t)tid * K;
        uint4 v[K];
#pragma unroll
        for (int r = 0; r < K; ++r) v[r] = src[r];
        for (int i = tid; i < 8 * 256; i += NT) s_hist[i] = 0;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < K; ++r)
#pragma unroll
            for (int b = 0; b < 16; ++b) atomicAdd(&s_hist[(b & 7) * 256 + byte_of(v[r], b)], 1u);
        __syncthreads();
        // dictionaries: wave w selects for planes w and w + 4, one value per
        // round (largest count, then smallest value: key = count << 8 | 255 - v)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int p = wave + 4 * h;
            uint32_t key[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t val = (uint32_t)lane + 64u * q;
                key[q] = (s_hist[p * 256 + val] << 8) | (255u - val);
            }
            uint32_t covered = 0, n = 0, first = 0;
            for (int i = 0; i < 15; ++i) {
                const uint32_t m = wave_max(max(max(key[0], key[1]), max(key[2], key[3])));
                if ((m >> 8) == 0) break;
                const uint32_t val = 255u - (m & 255u), cnt = m >> 8;
                if (i == 0) first = cnt;
                covered += cnt;
                ++n;
                if (lane == 0) s_dict[p * 16 + i] = (uint8_t)val;
                if (lane == (int)(val & 63u)) {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (q == (int)(val >> 6)) key[q] = 0;
                }
            }
            if (lane == 0) {
                for (uint32_t i = n; i < 16; ++i) s_dict[p * 16 + i] = 0;
                uint32_t mode = kPlaneRaw, esc = 0;
                if (n == 1 && first == L) {
                    mode = kPlaneConst;
                } else if (section_len(L, kPlaneDict, L - covered) < section_len(L, kPlaneRaw, 0)) {
                    mode = kPlaneDict;
                    esc = L - covered;
                }
                s_mode[p] = mode;
                s_esc[p] = esc;
                s_nused[p] = n;
            }
        }
        __syncthreads();
        if constexpr (!ENCODE) {
            if (tid == 0) {
                uint32_t at = kRecordHead;
                for (int p = 0; p < 8; ++p) at += section_len(L, s_mode[p], s_esc[p]);
                if (at < C) {
                    j.kind[g] = kPacked;
                    j.rlen[g] = at;
                } else {
                    j.rlen[g] = C;
                }
            }
        } else {
            if (tid == 0) {
                uint32_t at = kRecordHead;
                for (int p = 0; p < 8; ++p) {
                    s_sec[p] = at;
                    at += section_len(L, s_mode[p], s_esc[p]);
                }
                s_sec[8] = at;
            }
            for (int i = tid; i < 8 * 256; i += NT) s_code[i] = 15;
            __syncthreads();
            const uint32_t rl = s_sec[8];
            const bool ok = rl < C && rl == j.rlen[g];
            if (tid < 8 * 16) {
                const int p = tid >> 4, i = tid & 15;
                if (i < (int)s_nused[p]) s_code[p * 256 + s_dict[p * 16 + i]] = (uint8_t)i;
            }
            if (ok)
                for (uint32_t i = tid; i < rl / 16; i += NT) s_rec[i] = make_uint4(0, 0, 0, 0);
            __syncthreads();
            if (!ok) {
                if (tid == 0) atomicOr(j.err, 1u);
                continue;
            }
            uint8_t* rec8 = reinterpret_cast<uint8_t*>(s_rec);
            // head, constant values and dictionaries
            if (tid < 8) {
                rec8[tid] = (uint8_t)s_mode[tid];
                reinterpret_cast<uint32_t*>(rec8 + 8)[tid] = s_esc[tid];
                if (s_mode[tid] == kPlaneConst) rec8[s_sec[tid]] = s_dict[tid * 16];
            }
            if (tid < 8 * 16) {
                const int p = tid >> 4, i = tid & 15;
                if (s_mode[p] == kPlaneDict) rec8[s_sec[p] + i] = s_dict[p * 16 + i];
            }
            uint32_t mode[8], base[8];
#pragma unroll
            for (int p = 0; p < 8; ++p) {
                mode[p] = s_mode[p];
                base[p] = s_sec[p];
            }
            // escape positions: per-lane counts, then a block scan
            uint64_t ca = 0, cb = 0;
#pragma unroll
            for (int r = 0; r < K; ++r)
#pragma unroll
                for (int p = 0; p < 8; ++p)
                    if (mode[p] == kPlaneDict) {
                        const uint32_t n15 = (s_code[p * 256 + byte_of(v[r], p)] == 15) +
                                             (s_code[p * 256 + byte_of(v[r], p + 8)] == 15);
                        if (p < 4) ca += (uint64_t)n15 << (16 * p);
                        else cb += (uint64_t)n15 << (16 * (p - 4));
                    }
            uint64_t ta, tb;
            block_scan2(ca, cb, s_w, ta, tb);
            uint32_t pre[8];
#pragma unroll
            for (int p = 0; p < 8; ++p) pre[p] = field16(ca, cb, p);
            const uint32_t esc_at = 16 + r16(L / 2);
#pragma unroll
            for (int r = 0; r < K; ++r) {
                const uint32_t row = (uint32_t)tid * K + r;
#pragma unroll
                for (int p = 0; p < 8; ++p) {
                    const uint32_t b0 = byte_of(v[r], p), b1 = byte_of(v[r], p + 8);
                    if (mode[p] == kPlaneRaw) {
                        *reinterpret_cast<uint16_t*>(rec8 + base[p] + 2 * row) = (uint16_t)(b0 | (b1 << 8));
                    } else if (mode[p] == kPlaneDict) {
                        const uint32_t c0 = s_code[p * 256 + b0], c1 = s_code[p * 256 + b1];
                        rec8[base[p] + 16 + row] = (uint8_t)(c0 | (c1 << 4));
                        if (c0 == 15) rec8[base[p] + esc_at + pre[p]++] = (uint8_t)b0;
                        if (c1 == 15) rec8[base[p] + esc_at + pre[p]++] = (uint8_t)b1;
                    }
                }
            }
            __syncthreads();
            uint4* dst = reinterpret_cast<uint4*>(j.slot + j.off[g]);
            for (uint32_t i = tid; i < rl / 16; i += NT) dst[i] = s_rec[i];
        }
    }
}

// Decode of PACKED chunks: record to LDS, head checked, escape positions by a
// block scan (their count checked against the head), rows decoded, stored to
// the allocation and digested per lane (one table lookup per byte); the lane
// digests are combined into the chunk's CRC and compared with the image's.
template <int K>
__global__ void __launch_bounds__(NT) k_unpack(JobList jl, const uint32_t* rlen, const CodecConsts* cc) {
    __shared__ uint4 s_rec[kCodecMaxChunk / 16];
    __shared__ uint32_t s_tab[256];
    __shared__ uint32_t s_mode[8], s_esc[8], s_sec[9];
    __shared__ uint32_t s_ok;
    __shared__ unsigned long long s_w[2 * NW];
    __shared__ uint32_t s_red[NW];
    const int tid = threadIdx.x;
    for (int i = tid; i < 256; i += NT) s_tab[i] = cc->table[i];
    const uint32_t lanec = cc->lane[tid], full_init = cc->full_init;
    const uint32_t C = jl.job[0].C, L = C / 8;
    const uint64_t total = jl.prefix[jl.n_jobs];
    for (uint64_t tk = blockIdx.x; tk < total; tk += gridDim.x) {
        __syncthreads();   // the previous chunk's LDS is no longer read
        uint32_t jj = 0;
        while (jj + 1 < jl.n_jobs && jl.prefix[jj + 1] <= tk) ++jj;
        const ChunkJob& job = jl.job[jj];
        const uint64_t g = job.g0 + (tk - jl.prefix[jj]);
        if (job.kind_in[g] != kPacked) continue;
        const AllocDesc ad = job.allocs[job.amap[g]];
        const uint64_t k = g - ad.first;
        const uint64_t nk = (ad.size + C - 1) / C;
        const uint32_t len = (k + 1 == nk) ? ad.tail_len : C;
        const uint32_t rl = rlen[g];
        if (len != C || rl < kRecordHead + 8 * 16 || rl >= C || (rl & 15u)) {
            if (tid == 0) atomicMin(job.bad, (unsigned long long)g);
            continue;
        }
        const uint4* src = reinterpret_cast<const uint4*>(job.slot + (job.off[g] - job.slot_base));
        for (uint32_t i = tid; i < rl / 16; i += NT) s_rec[i] = src[i];
        __syncthreads();
        const uint8_t* rec8 = reinterpret_cast<const uint8_t*>(s_rec);
        if (tid == 0) {
            const uint32_t* h32 = reinterpret_cast<const uint32_t*>(rec8);
            bool ok = h32[10] == 0 && h32[11] == 0;
            uint32_t at = kRecordHead;
            for (int p = 0; p < 8; ++p) {
                const uint32_t mode = rec8[p], esc = h32[2 + p];
                ok = ok && mode <= kPlaneDict && (mode == kPlaneDict || esc == 0) && esc <= L;
                s_mode[p] = mode;
                s_esc[p] = esc;
                s_sec[p] = at;
                if (ok) at += section_len(L, mode, esc);
            }
            s_sec[8] = at;
            s_ok = ok && at == rl;
        }
        __syncthreads();
        if (!s_ok) {
            if (tid == 0) atomicMin(job.bad, (unsigned long long)g);
            continue;
        }
        uint32_t mode[8], base[8];
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            mode[p] = s_mode[p];
            base[p] = s_sec[p];
        }
        const uint32_t row0 = (uint32_t)tid * K;
        uint64_t ca = 0, cb = 0;
#pragma unroll
        for (int p = 0; p < 8; ++p)
            if (mode[p] == kPlaneDict) {
                uint32_t n15 = 0;
#pragma unroll
                for (int r = 0; r < K; ++r) {
                    const uint32_t byte = rec8[base[p] + 16 + row0 + r];
                    n15 += ((byte & 15u) == 15u) + ((byte >> 4) == 15u);
                }
                if (p < 4) ca += (uint64_t)n15 << (16 * p);
                else cb += (uint64_t)n15 << (16 * (p - 4));
            }
        uint64_t ta, tb;
        block_scan2(ca, cb, s_w, ta, tb);
        bool good = true;
#pragma unroll
        for (int p = 0; p < 8; ++p)
            if (mode[p] == kPlaneDict && field16(ta, tb, p) != s_esc[p]) good = false;
        if (!good) {   // the same on every lane: totals are block-wide
            if (tid == 0) atomicMin(job.bad, (unsigned long long)g);
            continue;
        }
        uint32_t pre[8];
#pragma unroll
        for (int p = 0; p < 8; ++p) pre[p] = field16(ca, cb, p);
        const uint32_t esc_at = 16 + r16(L / 2);
        uint4* dst = reinterpret_cast<uint4*>(ad.ptr + k * C);
        uint32_t crc = 0;
#pragma unroll
        for (int r = 0; r < K; ++r) {
            const uint32_t row = row0 + r;
            uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
            for (int p = 0; p < 8; ++p) {
                uint32_t b0, b1;
                if (mode[p] == kPlaneRaw) {
                    b0 = rec8[base[p] + 2 * row];
                    b1 = rec8[base[p] + 2 * row + 1];
                } else if (mode[p] == kPlaneConst) {
                    b0 = b1 = rec8[base[p]];
                } else {
                    const uint32_t byte = rec8[base[p] + 16 + row];
                    const uint32_t c0 = byte & 15u, c1 = byte >> 4;
                    b0 = c0 < 15 ? rec8[base[p] + c0] : rec8[base[p] + esc_at + pre[p]++];
                    b1 = c1 < 15 ? rec8[base[p] + c1] : rec8[base[p] + esc_at + pre[p]++];
                }
                w[p >> 2] |= b0 << (8 * (p & 3));
                w[2 + (p >> 2)] |= b1 << (8 * (p & 3));
            }
            dst[row] = make_uint4(w[0], w[1], w[2], w[3]);
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int b = 0; b < 4; ++b) crc = (crc >> 8) ^ s_tab[(crc ^ (w[q] >> (8 * b))) & 255u];
        }
        // r(chunk) = xor over lanes of r(segment t) * x^(8 * bytes after it)
        uint32_t x = gf_mul(crc, lanec);
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) x ^= __shfl_xor(x, m);
        if ((tid & 63) == 0) s_red[tid >> 6] = x;
        __syncthreads();
        if (tid == 0) {
            uint32_t raw = 0;
            for (int i = 0; i < NW; ++i) raw ^= s_red[i];
            if (~(raw ^ full_init) != job.ref_crc[g]) atomicMin(job.bad, (unsigned long long)g);
        }
    }
}

template <int K>
hipError_t pack_k(const PackJob& j, bool encode, int grid, hipStream_t s) {
    if (encode) hipLaunchKernelGGL((k_pack<K, true>), dim3(grid), dim3(NT), 0, s, j);
    else hipLaunchKernelGGL((k_pack<K, false>), dim3(grid), dim3(NT), 0, s, j);
    return hipGetLastError();
}

template <int K>
hipError_t unpack_k(const JobList& jl, const uint32_t* rlen, const CodecConsts* cc, int grid, hipStream_t s) {
    hipLaunchKernelGGL((k_unpack<K>), dim3(grid), dim3(NT), 0, s, jl, rlen, cc);
    return hipGetLastError();
}

}  // namespace

void build_codec_consts(CodecConsts* cc, uint32_t C) {
    for (uint32_t b = 0; b < 256; ++b) {
        uint32_t r = b;
        for (int i = 0; i < 8; ++i) r = (r >> 1) ^ ((r & 1u) ? kPoly : 0u);
        cc->table[b] = r;
    }
    const uint64_t seg = C / kCodecThreads;   // bytes per lane
    for (int t = 0; t < kCodecThreads; ++t) cc->lane[t] = xpow8(seg * (uint64_t)(kCodecThreads - 1 - t));
    cc->full_init = gf_mul(0xFFFFFFFFu, xpow8(C));
    for (uint32_t& x : cc->pad) x = 0;
}

hipError_t launch_pack(const PackJob& j, bool encode, int grid, hipStream_t s) {
    if (!codec_chunk_supported(j.C) || !j.amap || grid < 1) return hipErrorInvalidValue;
    if (j.g1 <= j.g0) return hipSuccess;
    switch (j.C / kCodecMinChunk) {
        case 1: return pack_k<1>(j, encode, grid, s);
        case 2: return pack_k<2>(j, encode, grid, s);
        case 4: return pack_k<4>(j, encode, grid, s);
        case 8: return pack_k<8>(j, encode, grid, s);
        case 16: return pack_k<16>(j, encode, grid, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_unpack(const JobList& jl, const uint32_t* rlen, const CodecConsts* cc, int grid, hipStream_t s) {
    if (jl.n_jobs == 0 || jl.n_jobs > (uint32_t)kMaxJobs || grid < 1 || !rlen || !cc) return hipErrorInvalidValue;
    const uint32_t C = jl.job[0].C;
    for (uint32_t i = 0; i < jl.n_jobs; ++i)
        if (jl.job[i].C != C || !jl.job[i].amap) return hipErrorInvalidValue;
    if (!codec_chunk_supported(C)) return hipErrorInvalidValue;
    if (jl.prefix[jl.n_jobs] == 0) return hipSuccess;
    switch (C / kCodecMinChunk) {
        case 1: return unpack_k<1>(jl, rlen, cc, grid, s);
        case 2: return unpack_k<2>(jl, rlen, cc, grid, s);
        case 4: return unpack_k<4>(jl, rlen, cc, grid, s);
        case 8: return unpack_k<8>(jl, rlen, cc, grid, s);
        case 16: return unpack_k<16>(jl, rlen, cc, grid, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mk
