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

// NB bytes held in little-endian words w[] to p (global memory, aligned to
// min(NB, 16)).
template <int NB>
__device__ inline void store_bytes(uint8_t* p, const uint32_t* w) {
    if constexpr (NB == 1) {
        *p = (uint8_t)w[0];
    } else if constexpr (NB == 2) {
        *reinterpret_cast<uint16_t*>(p) = (uint16_t)w[0];
    } else if constexpr (NB == 4) {
        *reinterpret_cast<uint32_t*>(p) = w[0];
    } else if constexpr (NB == 8) {
        *reinterpret_cast<uint2*>(p) = make_uint2(w[0], w[1]);
    } else {
#pragma unroll
        for (int i = 0; i < NB / 16; ++i)
            reinterpret_cast<uint4*>(p)[i] = make_uint4(w[4 * i], w[4 * i + 1], w[4 * i + 2], w[4 * i + 3]);
    }
}

template <int NB>
__device__ inline void load_bytes(const uint8_t* p, uint32_t* w) {
    if constexpr (NB == 1) {
        w[0] = *p;
    } else if constexpr (NB == 2) {
        w[0] = *reinterpret_cast<const uint16_t*>(p);
    } else if constexpr (NB == 4) {
        w[0] = *reinterpret_cast<const uint32_t*>(p);
    } else if constexpr (NB == 8) {
        const uint2 x = *reinterpret_cast<const uint2*>(p);
        w[0] = x.x;
        w[1] = x.y;
    } else {
#pragma unroll
        for (int i = 0; i < NB / 16; ++i) {
            const uint4 x = reinterpret_cast<const uint4*>(p)[i];
            w[4 * i] = x.x;
            w[4 * i + 1] = x.y;
            w[4 * i + 2] = x.z;
            w[4 * i + 3] = x.w;
        }
    }
}

__device__ inline uint32_t byte_in(const uint32_t* w, int i) { return (w[i >> 2] >> (8 * (i & 3))) & 255u; }

// Entry c (0..14, run-time) of a 16-byte dictionary held in four registers:
// two byte permutes (v_perm_b32; selector 0x0C gives a zero byte) and a
// select, where byte_in would need a compare-and-select chain over the four
// registers.
__device__ inline uint32_t dict_byte(const uint32_t (&d)[4], uint32_t c) {
    const uint32_t sel = (c & 7u) | 0x0C0C0C00u;
    const uint32_t lo = __builtin_amdgcn_perm(d[1], d[0], sel);
    const uint32_t hi = __builtin_amdgcn_perm(d[3], d[2], sel);
    return (c & 8u) ? hi : lo;
}

// Size pass (ENCODE false): the record length of every full DATA chunk; the
// chunk becomes PACKED when it is shorter than C. Encode pass: the record of
// every PACKED chunk, written to its payload offset (every byte of the
// record exactly once, padding included).
// Byte counts go to kHistCopies histograms, lane l to copy l % kHistCopies:
// the sign / exponent planes of floating-point data hold few distinct bytes,
// and the lanes of a wave adding to the same counter are served one at a
// time. The copies are kHistStride words apart, one bank off each other.
constexpr int kHistCopies = 4;
constexpr int kHistStride = 8 * 256 + 1;

template <int K, bool ENCODE>
__global__ void __launch_bounds__(NT) k_pack(PackJob j) {
    __shared__ uint32_t s_hist[ENCODE ? 1 : kHistCopies * kHistStride];
    __shared__ uint8_t s_code[8 * 256];
    __shared__ __align__(16) uint8_t s_dict[8 * 16];
    __shared__ __align__(16) uint8_t s_meta[ENCODE ? kPackMeta : 16];
    __shared__ uint32_t s_mode[8], s_esc[8], s_nused[8];
    __shared__ unsigned long long s_w[2 * NW];
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
        const uint4* src = reinterpret_cast<const uint4*>(ad.ptr + k * C);
        uint4 v[K];
        // the size pass only counts bytes: rows interleaved across lanes
        // (coalesced); the encode pass needs each lane's rows consecutive
#pragma unroll
        for (int r = 0; r < K; ++r) v[r] = ENCODE ? src[tid * K + r] : src[r * NT + tid];
        if constexpr (ENCODE) {
            // modes, escape counts and dictionaries as the size pass chose them
            for (int i = tid; i < 8 * 256; i += NT) s_code[i] = 15;
            if (tid < (int)(kPackMeta / 16))
                reinterpret_cast<uint4*>(s_meta)[tid] = reinterpret_cast<const uint4*>(j.meta + g * kPackMeta)[tid];
            __syncthreads();
            if (tid < 8) {
                s_mode[tid] = s_meta[tid];
                s_esc[tid] = (uint32_t)s_meta[8 + 4 * tid] | ((uint32_t)s_meta[9 + 4 * tid] << 8) |
                             ((uint32_t)s_meta[10 + 4 * tid] << 16) | ((uint32_t)s_meta[11 + 4 * tid] << 24);
                s_nused[tid] = s_meta[176 + tid];
            }
            if (tid < 8 * 16) s_dict[tid] = s_meta[48 + tid];
            __syncthreads();
        } else {
            for (int i = tid; i < kHistCopies * kHistStride; i += NT) s_hist[i] = 0;
            __syncthreads();
            uint32_t* hist = s_hist + (tid % kHistCopies) * kHistStride;
#pragma unroll
            for (int r = 0; r < K; ++r)
#pragma unroll
                for (int b = 0; b < 16; ++b) {
                    // the wave's lanes holding the first lane's value are
                    // counted with one atomic (the sign / exponent planes
                    // repeat a few values, and an LDS atomic serializes the
                    // lanes it finds on one address)
                    const uint32_t val = byte_of(v[r], b);
                    const uint32_t v0 = __builtin_amdgcn_readfirstlane(val);
                    const uint64_t m = __ballot(val == v0);
                    if (val != v0) atomicAdd(&hist[(b & 7) * 256 + val], 1u);
                    else if ((tid & 63) == __ffsll((unsigned long long)m) - 1)   // the lane v0 came from
                        atomicAdd(&hist[(b & 7) * 256 + v0], (uint32_t)__popcll(m));
                }
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
                    uint32_t cnt = 0;
#pragma unroll
                    for (int cp = 0; cp < kHistCopies; ++cp) cnt += s_hist[cp * kHistStride + p * 256 + val];
                    key[q] = (cnt << 8) | (255u - val);
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
        }
        uint32_t mode[8], esc[8], base[8];
        uint32_t rl = kRecordHead;
#pragma unroll
        for (int p = 0; p < 8; ++p) {   // work-group-uniform: kept in scalar registers
            mode[p] = __builtin_amdgcn_readfirstlane(s_mode[p]);
            esc[p] = __builtin_amdgcn_readfirstlane(s_esc[p]);
            base[p] = rl;
            rl += section_len(L, mode[p], esc[p]);
        }
        if constexpr (!ENCODE) {
            if (tid == 0) {
                if (rl < C) {
                    j.kind[g] = kPacked;
                    j.rlen[g] = rl;
                } else {
                    j.rlen[g] = C;
                }
            }
            if (rl < C && tid < (int)(kPackMeta / 16)) {
                // for the encode: head, dictionaries, used entries
                uint32_t w[4] = {0, 0, 0, 0};
                if (tid == 0) {
                    w[0] = mode[0] | (mode[1] << 8) | (mode[2] << 16) | (mode[3] << 24);
                    w[1] = mode[4] | (mode[5] << 8) | (mode[6] << 16) | (mode[7] << 24);
                    w[2] = esc[0];
                    w[3] = esc[1];
                } else if (tid == 1) {
                    w[0] = esc[2];
                    w[1] = esc[3];
                    w[2] = esc[4];
                    w[3] = esc[5];
                } else if (tid == 2) {
                    w[0] = esc[6];
                    w[1] = esc[7];
                } else if (tid < 11) {
                    const uint4 d = *reinterpret_cast<const uint4*>(&s_dict[(tid - 3) * 16]);
                    w[0] = d.x;
                    w[1] = d.y;
                    w[2] = d.z;
                    w[3] = d.w;
                } else {
                    w[0] = s_nused[0] | (s_nused[1] << 8) | (s_nused[2] << 16) | (s_nused[3] << 24);
                    w[1] = s_nused[4] | (s_nused[5] << 8) | (s_nused[6] << 16) | (s_nused[7] << 24);
                }
                reinterpret_cast<uint4*>(j.meta + g * kPackMeta)[tid] = make_uint4(w[0], w[1], w[2], w[3]);
            }
        } else {
            if (tid < 8 * 16) {
                const int p = tid >> 4, i = tid & 15;
                if (i < (int)s_nused[p]) s_code[p * 256 + s_dict[p * 16 + i]] = (uint8_t)i;
            }
            if (!(rl < C && rl == j.rlen[g])) {   // the same on every lane
                if (tid == 0) atomicOr(j.err, 1u);
                continue;
            }
            uint8_t* dst = j.slot + (j.off[g] - j.slot_base);
            const uint32_t esc_at = 16 + r16(L / 2);
            // head (48 bytes), constant values, dictionaries, escape padding
            if (tid < 3) {
                uint32_t hw[4];
                if (tid == 0) {
                    hw[0] = mode[0] | (mode[1] << 8) | (mode[2] << 16) | (mode[3] << 24);
                    hw[1] = mode[4] | (mode[5] << 8) | (mode[6] << 16) | (mode[7] << 24);
                    hw[2] = esc[0];
                    hw[3] = esc[1];
                } else if (tid == 1) {
                    hw[0] = esc[2];
                    hw[1] = esc[3];
                    hw[2] = esc[4];
                    hw[3] = esc[5];
                } else {
                    hw[0] = esc[6];
                    hw[1] = esc[7];
                    hw[2] = 0;
                    hw[3] = 0;
                }
                store_bytes<16>(dst + 16 * tid, hw);
            }
#pragma unroll
            for (int p = 0; p < 8; ++p) {
                if (tid == 8 + p && mode[p] == kPlaneConst) {
                    const uint32_t w[4] = {s_dict[p * 16], 0, 0, 0};
                    store_bytes<16>(dst + base[p], w);
                }
                if (tid == 16 + p && mode[p] == kPlaneDict) {
                    const uint4 d = *reinterpret_cast<const uint4*>(&s_dict[p * 16]);
                    const uint32_t w[4] = {d.x, d.y, d.z, d.w};
                    store_bytes<16>(dst + base[p], w);
                }
                if (tid == 24 + p && mode[p] == kPlaneDict)
                    for (uint32_t b = esc[p]; b < r16(esc[p]); ++b) dst[base[p] + esc_at + b] = 0;
            }
            __syncthreads();   // s_code complete
            // escape positions: per-lane counts, then a block scan
            uint64_t ca = 0, cb = 0;
#pragma unroll
            for (int p = 0; p < 8; ++p)
                if (mode[p] == kPlaneDict) {
                    uint32_t n15 = 0;
#pragma unroll
                    for (int r = 0; r < K; ++r)
                        n15 += (s_code[p * 256 + byte_of(v[r], p)] == 15) + (s_code[p * 256 + byte_of(v[r], p + 8)] == 15);
                    if (p < 4) ca += (uint64_t)n15 << (16 * p);
                    else cb += (uint64_t)n15 << (16 * (p - 4));
                }
            uint64_t ta, tb;
            block_scan2(ca, cb, s_w, ta, tb);
            const uint32_t row0 = (uint32_t)tid * K;
#pragma unroll
            for (int p = 0; p < 8; ++p) {
                if (mode[p] == kPlaneRaw) {
                    // the lane's 2K plane bytes: element 2r, 2r+1 of each row
                    uint32_t w[(2 * K + 3) / 4];
#pragma unroll
                    for (int i = 0; i < (2 * K + 3) / 4; ++i) w[i] = 0;
#pragma unroll
                    for (int r = 0; r < K; ++r)
                        w[r >> 1] |= (byte_of(v[r], p) | (byte_of(v[r], p + 8) << 8)) << (16 * (r & 1));
                    store_bytes<2 * K>(dst + base[p] + 2 * row0, w);
                } else if (mode[p] == kPlaneDict) {
                    uint32_t pre = field16(ca, cb, p);
                    uint32_t w[(K + 3) / 4];
#pragma unroll
                    for (int i = 0; i < (K + 3) / 4; ++i) w[i] = 0;
#pragma unroll
                    for (int r = 0; r < K; ++r) {
                        const uint32_t b0 = byte_of(v[r], p), b1 = byte_of(v[r], p + 8);
                        const uint32_t c0 = s_code[p * 256 + b0], c1 = s_code[p * 256 + b1];
                        w[r >> 2] |= (c0 | (c1 << 4)) << (8 * (r & 3));
                        if (c0 == 15) dst[base[p] + esc_at + pre++] = (uint8_t)b0;
                        if (c1 == 15) dst[base[p] + esc_at + pre++] = (uint8_t)b1;
                    }
                    store_bytes<K>(dst + base[p] + 16 + row0, w);
                }
                // one plane at a time: keeps the compiler from hoisting every
                // plane's table lookups (hundreds of live registers)
                asm volatile("" ::: "memory");
            }
        }
    }
}

// Decode of PACKED chunks from the staging window: head checked, escape
// positions by a block scan (their count checked against the head), rows
// decoded, stored to the allocation and digested per lane, 16 bytes per
// step; the lane digests are combined into the chunk's CRC and compared
// with the image's.
template <int K>
__global__ void __launch_bounds__(NT) k_unpack(JobList jl, const uint32_t* rlen, const CodecConsts* cc) {
    __shared__ uint32_t s_tab[16 * 256];
    __shared__ unsigned long long s_w[2 * NW];
    __shared__ uint32_t s_red[NW];
    const int tid = threadIdx.x;
    for (int i = tid; i < 16 * 256; i += NT) s_tab[i] = cc->tab[i];
    const uint32_t lanec = cc->lane[tid], full_init = cc->full_init;
    const uint32_t C = jl.job[0].C, L = C / 8;
    const uint64_t total = jl.prefix[jl.n_jobs];
    const uint32_t row0 = (uint32_t)tid * K;
    for (uint64_t tk = blockIdx.x; tk < total; tk += gridDim.x) {
        __syncthreads();   // s_tab loaded; s_w / s_red of the previous chunk read
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
        const uint8_t* rec = job.slot + (job.off[g] - job.slot_base);
        uint32_t h[12];
        load_bytes<16>(rec, h);
        load_bytes<16>(rec + 16, h + 4);
        load_bytes<16>(rec + 32, h + 8);
#pragma unroll
        for (int i = 0; i < 12; ++i) h[i] = __builtin_amdgcn_readfirstlane(h[i]);   // the same on every lane
        uint32_t mode[8], esc[8], base[8];
        bool ok = h[10] == 0 && h[11] == 0;
        uint32_t at = kRecordHead;
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            mode[p] = byte_in(h, p);
            esc[p] = h[2 + p];
            ok = ok && mode[p] <= kPlaneDict && (mode[p] == kPlaneDict || esc[p] == 0) && esc[p] <= L;
            base[p] = at;
            if (ok) at += section_len(L, mode[p], esc[p]);
        }
        if (!(ok && at == rl)) {   // the same on every lane
            if (tid == 0) atomicMin(job.bad, (unsigned long long)g);
            continue;
        }
        // escape counts of the lane's codes (the codes are read again, plane
        // by plane, when decoded: keeping all 8 planes' codes live across the
        // scan costs a wave per SIMD)
        uint64_t ca = 0, cb = 0;
#pragma unroll
        for (int p = 0; p < 8; ++p)
            if (mode[p] == kPlaneDict) {
                uint32_t cw[(K + 3) / 4];
                load_bytes<K>(rec + base[p] + 16 + row0, cw);
                uint32_t n15 = 0;
#pragma unroll
                for (int r = 0; r < K; ++r) {
                    const uint32_t byte = byte_in(cw, r);
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
            if (mode[p] == kPlaneDict && field16(ta, tb, p) != esc[p]) good = false;
        if (!good) {   // the same on every lane: totals are block-wide
            if (tid == 0) atomicMin(job.bad, (unsigned long long)g);
            continue;
        }
        const uint32_t esc_at = 16 + r16(L / 2);
        // the lane's rows in parts of KH (at most 8 rows live at once; the
        // escape positions of each plane carry over from part to part)
        constexpr int KH = K < 8 ? K : 8;
        uint32_t pre[8];
#pragma unroll
        for (int p = 0; p < 8; ++p) pre[p] = field16(ca, cb, p);
        uint32_t crc = 0;
#pragma unroll 1
        for (int part = 0; part < K / KH; ++part) {
            const uint32_t r0 = row0 + (uint32_t)part * KH;
            uint32_t out[KH][4];
#pragma unroll
            for (int r = 0; r < KH; ++r) out[r][0] = out[r][1] = out[r][2] = out[r][3] = 0;
#pragma unroll
            for (int p = 0; p < 8; ++p) {
                const int wl = p >> 2, sh = 8 * (p & 3);
                if (mode[p] == kPlaneRaw) {
                    uint32_t w[(2 * KH + 3) / 4];
                    load_bytes<2 * KH>(rec + base[p] + 2 * r0, w);
#pragma unroll
                    for (int r = 0; r < KH; ++r) {
                        out[r][wl] |= byte_in(w, 2 * r) << sh;
                        out[r][2 + wl] |= byte_in(w, 2 * r + 1) << sh;
                    }
                } else if (mode[p] == kPlaneConst) {
                    const uint32_t b = rec[base[p]];
#pragma unroll
                    for (int r = 0; r < KH; ++r) {
                        out[r][wl] |= b << sh;
                        out[r][2 + wl] |= b << sh;
                    }
                } else {
                    uint32_t d[4], cw[(KH + 3) / 4];
                    load_bytes<16>(rec + base[p], d);
                    load_bytes<KH>(rec + base[p] + 16 + r0, cw);
                    const uint8_t* escs = rec + base[p] + esc_at;
                    uint32_t q = pre[p];
#pragma unroll
                    for (int r = 0; r < KH; ++r) {
                        const uint32_t byte = byte_in(cw, r);
                        const uint32_t c0 = byte & 15u, c1 = byte >> 4;
                        const uint32_t b0 = c0 < 15 ? dict_byte(d, c0) : escs[q++];
                        const uint32_t b1 = c1 < 15 ? dict_byte(d, c1) : escs[q++];
                        out[r][wl] |= b0 << sh;
                        out[r][2 + wl] |= b1 << sh;
                    }
                    pre[p] = q;
                }
                asm volatile("" ::: "memory");   // one plane at a time (register pressure)
            }
            uint4* dst = reinterpret_cast<uint4*>(ad.ptr + k * C) + r0;
#pragma unroll
            for (int r = 0; r < KH; ++r) {
                dst[r] = make_uint4(out[r][0], out[r][1], out[r][2], out[r][3]);
                const uint32_t x[4] = {out[r][0] ^ crc, out[r][1], out[r][2], out[r][3]};
                uint32_t c = 0;
#pragma unroll
                for (int i = 0; i < 16; ++i) c ^= s_tab[i * 256 + byte_in(x, i)];
                crc = c;
            }
        }
        // r(chunk) = xor over lanes of r(segment t) * x^(8 * bytes after it)
        uint32_t xr = gf_mul(crc, lanec);
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) xr ^= __shfl_xor(xr, m);
        if ((tid & 63) == 0) s_red[tid >> 6] = xr;
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
