// Chunk kernels for gfx950 (CDNA4, wave64).
//
// One persistent kernel family processes the chunk grid of an allocation
// table: each work-group takes chunk tickets in increasing order from an
// atomic counter, so every chunk below its ticket has already been taken by
// a running work-group (this is what makes the decoupled look-back safe).
//
// Per chunk, the T threads of a work-group read the chunk as K rows of
// 16 T bytes: thread t owns the 16-byte block at offset r*16T + 16t of each
// row r, so every row is one fully coalesced 128-bit load per thread. The
// CRC-32C of the chunk is computed without moving the data between lanes:
// lane t keeps the raw CRC of its own interleaved stream (its blocks, with
// the other lanes' bytes read as zeros). Per row the running value is xored
// into the first four bytes of the lane's block and the block is reduced
// with sixteen lookups in tables (dt, in LDS) that also carry the shift over
// the rest of the row, so advancing over a row costs no extra lookup. At the
// end lane t's value is moved to its place in the chunk (multiplied by
// x^(-8*16t)) and the lanes' values are xor-reduced.
// Modes:
//   dump    - digest + zero test + unchanged test against the previous
//             digest table, then the chunk's payload offset from a decoupled
//             look-back over the chunks before it, then the chunk is stored
//             from registers into the staging window (single pass: the data
//             is read from HBM once);
//   digest  - digest only (used for the image's table digests);
//   verify  - digest of UNCHANGED chunks compared with the image (delta
//             restore checks that the target holds the base), or of every
//             chunk (kJobVerifyAll: the strict re-read after a restore);
//   restore - DATA chunks read from the staging window, stored to their
//             allocation and verified on the data in registers; ZERO chunks
//             zero-filled (PACKED chunks are left to the codec's decode).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace mk {
namespace {

constexpr uint32_t kMaxSpins = 1u << 24;

typedef __attribute__((address_space(1))) uint64_t gu64;
__device__ inline void st_relaxed(uint64_t* p, uint64_t v) {
    __hip_atomic_store((gu64*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t ld_relaxed(uint64_t* p) {
    return __hip_atomic_load((gu64*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

__device__ inline uint32_t wave_xor(uint32_t v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v ^= __shfl_xor(v, m);
    return v;
}

// Decoupled look-back (single-pass prefix scan). lb_publish stores the
// aggregate `agg` of position idx (at position 0 it is the inclusive
// prefix); lb_walk then sums the aggregates of the predecessors back to the
// nearest published inclusive prefix, publishes the inclusive prefix of idx
// and returns the exclusive one (all 64 lanes of one wave call it).
__device__ inline void lb_publish(uint64_t* status, uint64_t idx, uint64_t agg, uint32_t epoch) {
    const uint64_t tag = (uint64_t)(epoch & kEpochMask) << 40;
    st_relaxed(&status[idx], (idx == 0 ? kStInc : kStAgg) | tag | agg);
}

__device__ inline bool lb_valid(uint64_t w, uint32_t epoch) {
    return (w >> 62) != 0 && ((w >> 40) & kEpochMask) == (epoch & kEpochMask);
}

// The walk reads one status word per lane per step (64 predecessors). Four
// words per lane (256 per step) made the streamed dump kernel spill two
// registers at its 128-VGPR budget and ran 14 % slower (12.3 against
// 10.8 ms on the training state); two words, without a spill, 4 % slower.
__device__ uint64_t lb_walk(uint64_t* status, uint64_t idx, uint64_t agg, uint32_t epoch, uint32_t* err) {
    const int lane = threadIdx.x & 63;
    const uint64_t tag = (uint64_t)(epoch & kEpochMask) << 40;
    if (idx == 0) return 0;
    uint64_t excl = 0;
    int64_t base = (int64_t)idx - 1;
    for (;;) {
        const int64_t j = base - lane;
        uint64_t w = kStInc | tag;          // before the start: inclusive 0
        if (j >= 0) {
            uint32_t spins = 0;
            for (;;) {
                w = ld_relaxed(&status[j]);
                if (lb_valid(w, epoch)) break;
                if (++spins > kMaxSpins) {   // bounded wait: report, never hang
                    atomicOr(err, 1u);
                    w = kStInc | tag;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        const bool inc = (w >> 62) == 2;
        const uint64_t val = w & kStValueMask;
        const uint64_t incmask = __ballot(inc);
        if (incmask) {
            // lanes up to the nearest inclusive prefix
            const int first = __ffsll((unsigned long long)incmask) - 1;
            excl += wave_sum_u64(lane <= first ? val : 0);
            break;
        }
        excl += wave_sum_u64(val);
        base -= 64;
    }
    if (lane == 0) st_relaxed(&status[idx], kStInc | tag | (excl + agg));
    return excl;
}

__device__ inline uint64_t lookback(uint64_t* status, uint64_t idx, uint64_t agg, uint32_t epoch, uint32_t* err) {
    if ((threadIdx.x & 63) == 0) lb_publish(status, idx, agg, epoch);
    return lb_walk(status, idx, agg, epoch, err);
}

// last allocation whose first chunk is <= g (empty allocations share their
// successor's first chunk and are therefore never selected)
__device__ inline uint32_t find_alloc(const AllocDesc* a, uint32_t n, uint64_t g) {
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (*(const __attribute__((address_space(4))) uint64_t*)(&a[mid].first) <= g) lo = mid; else hi = mid;
    }
    return lo;
}

// 128-bit data type. Accesses go through address-space-1 (global) pointers:
// the chunk pointers come from descriptors (integers), and without an
// explicit address space the compiler emits flat accesses.
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const v4u gcv4;
typedef __attribute__((address_space(1))) v4u gv4;
typedef __attribute__((address_space(1))) const uint8_t gcu8;
typedef __attribute__((address_space(1))) uint8_t gu8;
__device__ inline v4u gload(const uint8_t* p) { return *(gcv4*)(p); }
__device__ inline void gstore(uint8_t* p, v4u v) { *(gv4*)(p) = v; }
__device__ inline v4u vzero() { return (v4u){0u, 0u, 0u, 0u}; }

__device__ inline v4u load_partial(const uint8_t* p, uint32_t n) {   // 0 < n < 16
    uint64_t lo = 0, hi = 0;
    for (uint32_t i = 0; i < n; ++i) {
        const uint64_t b = ((gcu8*)p)[i];
        if (i < 8) lo |= b << (8 * i); else hi |= b << (8 * (i - 8));
    }
    return (v4u){(uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32)};
}

__device__ inline void store_partial(uint8_t* p, v4u v, uint32_t n) {   // 0 < n < 16
    const uint64_t lo = (uint64_t)v.x | ((uint64_t)v.y << 32);
    const uint64_t hi = (uint64_t)v.z | ((uint64_t)v.w << 32);
    for (uint32_t i = 0; i < n; ++i) ((gu8*)p)[i] = (uint8_t)((i < 8 ? lo >> (8 * i) : hi >> (8 * (i - 8))) & 0xFF);
}

// keep the low n bytes of v (0 < n < 16); *dropped |= the other bytes
__device__ inline v4u keep_low(v4u v, uint32_t n, uint32_t* dropped) {
    v4u out;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int nb = (int)n - 4 * i;   // bytes of word i to keep
        const uint32_t m = nb >= 4 ? 0xFFFFFFFFu : nb <= 0 ? 0u : ((1u << (8 * nb)) - 1u);
        out[i] = v[i] & m;
        *dropped |= v[i] & ~m;
    }
    return out;
}

__device__ inline uint32_t or4(v4u v) { return v.x | v.y | v.z | v.w; }

// The digest's arithmetic is VALU-bound, so two of its steps are written as
// the gfx950 instructions that do them in the fewest operations (measured on
// the dump kernel: -3.7 % kernel time against the compiler's own sequences):
// a three-input XOR is one v_bitop3_b32 (truth table 0x96; gfx9 has no
// v_xor3_b32), and the GF(2) multiply below takes five instructions per bit.
__device__ inline uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// a * b mod P, bit-serial over the coefficients of a (x^0 first), as
// gf_mul: per bit, the coefficient as a mask (v_bfe_i32), p ^= b & mask
// (v_bitop3_b32, table 0x78 = s0 ^ (s1 & s2)), then b * x: the low bit as a
// mask, b >> 1, and (b >> 1) ^ (P & mask).
__device__ inline uint32_t gf_mul_v(uint32_t a, uint32_t b) {
    uint32_t p = 0;
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        uint32_t m;
        asm("v_bfe_i32 %0, %1, %2, 1" : "=v"(m) : "v"(a), "i"(31 - i));
        asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x78" : "=v"(p) : "v"(p), "v"(b), "v"(m));
        if (i < 31) {
            uint32_t s, t;
            asm("v_bfe_i32 %0, %1, 0, 1" : "=v"(s) : "v"(b));
            asm("v_lshrrev_b32 %0, 1, %1" : "=v"(t) : "v"(b));
            asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x78" : "=v"(b) : "v"(t), "s"(kPoly), "v"(s));
        }
    }
    return p;
}

__device__ inline uint32_t blk16(v4u v, const uint32_t* dt) {
    const uint32_t l0 = dt[0 * 256 + (v.x & 255)], l1 = dt[1 * 256 + ((v.x >> 8) & 255)];
    const uint32_t l2 = dt[2 * 256 + ((v.x >> 16) & 255)], l3 = dt[3 * 256 + (v.x >> 24)];
    const uint32_t l4 = dt[4 * 256 + (v.y & 255)], l5 = dt[5 * 256 + ((v.y >> 8) & 255)];
    const uint32_t l6 = dt[6 * 256 + ((v.y >> 16) & 255)], l7 = dt[7 * 256 + (v.y >> 24)];
    const uint32_t l8 = dt[8 * 256 + (v.z & 255)], l9 = dt[9 * 256 + ((v.z >> 8) & 255)];
    const uint32_t l10 = dt[10 * 256 + ((v.z >> 16) & 255)], l11 = dt[11 * 256 + (v.z >> 24)];
    const uint32_t l12 = dt[12 * 256 + (v.w & 255)], l13 = dt[13 * 256 + ((v.w >> 8) & 255)];
    const uint32_t l14 = dt[14 * 256 + ((v.w >> 16) & 255)], l15 = dt[15 * 256 + (v.w >> 24)];
    uint32_t a = xor3(l0, l1, l2);
    a = xor3(a, l3, l4);
    a = xor3(a, l5, l6);
    a = xor3(a, l7, l8);
    a = xor3(a, l9, l10);
    a = xor3(a, l11, l12);
    a = xor3(a, l13, l14);
    return a ^ l15;
}

template <int K>
__device__ inline uint32_t crc_rows(const v4u (&v)[K], uint32_t acc, const uint32_t* dt) {
#pragma unroll
    for (int r = 0; r < K; ++r) {
        v4u b = v[r];
        b.x ^= acc;
        acc = blk16(b, dt);
        // one row of lookups in flight at a time: keeps the register
        // footprint near the data itself (other waves hide the latency)
        __builtin_amdgcn_sched_barrier(0);
    }
    return acc;
}

// Load one pass (K rows) of a chunk, zero-extending beyond `len` valid bytes.
template <int T, int K>
__device__ inline void load_rows(v4u (&v)[K], const uint8_t* base, uint64_t len, uint32_t tid, bool active) {
    constexpr uint32_t R = 16u * T;
    if (!active) {
#pragma unroll
        for (int r = 0; r < K; ++r) v[r] = vzero();
        return;
    }
    if (len >= (uint64_t)R * K) {
#pragma unroll
        for (int r = 0; r < K; ++r) v[r] = gload(base + r * R + 16u * tid);
    } else {
#pragma unroll
        for (int r = 0; r < K; ++r) {
            const uint32_t o = r * R + 16u * tid;
            if (o + 16 <= len) v[r] = gload(base + o);
            else if (o < len) v[r] = load_partial(base + o, (uint32_t)(len - o));
            else v[r] = vzero();
        }
    }
}

// Load one pass of a payload record from staging: whole 16-byte blocks up to
// round16(len) exist; bytes beyond len are padding that must be zero.
template <int T, int K>
__device__ inline void load_rows_staged(v4u (&v)[K], const uint8_t* base, uint64_t len, uint32_t tid, bool active,
                                        uint32_t* padbad) {
    constexpr uint32_t R = 16u * T;
#pragma unroll
    for (int r = 0; r < K; ++r) {
        const uint32_t o = r * R + 16u * tid;
        if (!active || o >= len) {
            v[r] = vzero();
        } else {
            v[r] = gload(base + o);
            if (o + 16 > len) v[r] = keep_low(v[r], (uint32_t)(len - o), padbad);
        }
    }
}

// Store the valid bytes of one pass (len valid bytes from base) into an
// allocation being restored. Whole blocks go out as non-temporal stores: the
// restore does not read them back, and streaming them past the caches cut
// the restore kernel's time by 2-3 % on the training state.
template <int T, int K>
__device__ inline void store_rows_exact(const v4u (&v)[K], uint8_t* base, uint64_t len, uint32_t tid, bool active) {
    constexpr uint32_t R = 16u * T;
    if (!active) return;
#pragma unroll
    for (int r = 0; r < K; ++r) {
        const uint32_t o = r * R + 16u * tid;
        if (o + 16 <= len) __builtin_nontemporal_store(v[r], (gv4*)(base + o));
        else if (o < len) store_partial(base + o, v[r], (uint32_t)(len - o));
    }
}

// Store whole 16-byte blocks of one pass up to len16 bytes (payload records);
// NT: as non-temporal stores (the staging window is read next by the copy
// engines, not by a kernel).
template <int T, int K, bool NT = false>
__device__ inline void store_rows_padded(const v4u (&v)[K], uint8_t* base, uint64_t len16, uint32_t tid, bool active) {
    constexpr uint32_t R = 16u * T;
    if (!active) return;
#pragma unroll
    for (int r = 0; r < K; ++r) {
        const uint32_t o = r * R + 16u * tid;
        if (o < len16) {
            if constexpr (NT) __builtin_nontemporal_store(v[r], (gv4*)(base + o));
            else gstore(base + o, v[r]);
        }
    }
}

// Work-group barrier for LDS traffic only. __syncthreads also waits for
// every outstanding global load and store of the wave (its release fence);
// this one lets them run on, which keeps streamed rows in flight across it.
// Only LDS data is exchanged between the waves of a work-group across it.
__device__ inline void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Is p true in any thread of the work-group? (s_any: one word per wave)
template <int NW>
__device__ inline uint32_t wg_any_lds(bool p, uint32_t* s_any) {
    const uint64_t b = __ballot(p);
    if ((threadIdx.x & 63) == 0) s_any[threadIdx.x >> 6] = b != 0;
    lds_barrier();
    uint32_t r = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) r |= s_any[w];
    return r;
}

template <int NW>
__device__ inline uint32_t wg_xor_lds(uint32_t x, uint32_t* s_red) {
    x = wave_xor(x);
    if constexpr (NW > 1) {
        if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = x;
        lds_barrier();
        x = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) x ^= s_red[w];
    }
    return x;
}

template <int NW>
__device__ inline uint32_t wg_xor(uint32_t x, uint32_t* s_red) {
    x = wave_xor(x);
    if constexpr (NW > 1) {
        if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = x;
        __syncthreads();
        x = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) x ^= s_red[w];
    }
    return x;
}

// Register cap: 128 VGPRs (4 waves per SIMD) for every shape; the 8-row
// shapes hold 32 VGPRs of chunk data between load and store.
template <int T, int K, int MODE>
__global__ void __launch_bounds__(T < 64 ? 64 : T) __attribute__((amdgpu_waves_per_eu(4)))
k_chunks(JobList jl) {
    constexpr int NT = T < 64 ? 64 : T;
    constexpr int NW = NT / 64;
    constexpr uint32_t TILE = 16u * T * K;
    __shared__ uint32_t s_dt[16 * 256];
    __shared__ uint32_t s_red[NW];
    __shared__ uint32_t s_any[NW];
    __shared__ uint32_t s_tk[2];
    __shared__ uint64_t s_off;

    const int tid = threadIdx.x;
    const bool active = T >= 64 || tid < T;
    // a restore that its graph's validation rejected writes nothing
    if constexpr (MODE == kModeRestore || MODE == kModeVerify)
        if (jl.job[0].gate && *jl.job[0].gate == 0) return;
    const EngineConsts* ec = jl.job[0].ec;
    for (int i = tid; i < 16 * 256; i += NT) s_dt[i] = ec->dt[i];
    const uint32_t lanec = active ? ec->lane[tid] : 0u;
    const uint32_t full_init = ec->full_init;
    const uint32_t C = jl.job[0].C;
    const uint64_t total = jl.prefix[jl.n_jobs];
    const uint32_t log2c = 31 - __builtin_clz(C);
    const uint32_t P = C / TILE;        // passes per chunk (C is a multiple of TILE)
    __syncthreads();

    // The next ticket is fetched while the current chunk is processed, so
    // the atomic's latency is hidden. A work-group holds at most two
    // tickets, its current one and the next; the chunks before its current
    // one are held by running work-groups, so every look-back wait ends.
    // The dump mode's look-back needs chunks taken in ticket order, and the
    // restore mode keeps it (concurrently processed chunks stay adjacent in
    // HBM: 5.2-5.8 TB/s against 4.7 TB/s grid-stride on the training state);
    // the verify, digest and classify modes take chunks grid-stride,
    // so a chunk they skip costs no atomic and no barrier (a barrier follows
    // each chunk they process, for the LDS reductions).
    constexpr bool kTickets = MODE == kModeDump || MODE == kModeRestore;
    if (kTickets && tid == 0) s_tk[0] = atomicAdd(jl.ticket, 1u);
    bool dirty = false;
    for (uint32_t it = 0;; ++it) {
        uint64_t tk;
        if constexpr (kTickets) {
            lds_barrier();
            tk = (uint32_t)__builtin_amdgcn_readfirstlane(s_tk[it & 1]);
            if (tk >= total) break;
            if (tid == 0) s_tk[(it + 1) & 1] = atomicAdd(jl.ticket, 1u);
        } else {
            if (dirty) lds_barrier();   // the previous chunk's reductions are read
            dirty = false;
            tk = (uint64_t)blockIdx.x + (uint64_t)it * gridDim.x;
            if (tk >= total) break;
        }
        uint32_t jj = 0;
        while (jj + 1 < jl.n_jobs && jl.prefix[jj + 1] <= tk) ++jj;
        const ChunkJob& job = jl.job[jj];
        const uint64_t g = job.g0 + (tk - jl.prefix[jj]);
        // Opaque per-chunk copies of per-lane values: without them the
        // compiler hoists 32 multiples of the lane constant and one address
        // per row out of the loop, which costs ~50 VGPRs per lane.
        uint32_t lc = lanec;
        uint32_t ltid = (uint32_t)tid;
        asm volatile("" : "+v"(lc), "+v"(ltid));

        uint8_t kd_in = kData;
        if constexpr (MODE == kModeVerify || MODE == kModeRestore) {
            kd_in = job.kind_in[g];
            if (MODE == kModeVerify && kd_in != kUnchanged && !(job.flags & kJobVerifyAll)) continue;
            // UNCHANGED: nothing to write; PACKED: the codec's decode kernel
            if (MODE == kModeRestore && (kd_in == kUnchanged || kd_in == kPacked)) continue;
        }
        dirty = true;
        const uint32_t a = job.amap ? job.amap[g] : find_alloc(job.allocs, job.n_allocs, g);
        const AllocDesc ad = job.allocs[a];
        const uint64_t k = g - ad.first;
        const uint64_t nk = (ad.size + C - 1) >> log2c;
        const uint32_t len = (k + 1 == nk) ? ad.tail_len : C;
        const bool full = len == C;
        const uint32_t init = full ? full_init : ad.tail_init;
        uint8_t* const aptr = reinterpret_cast<uint8_t*>(ad.ptr) + (k << log2c);

        if constexpr (MODE == kModeRestore) {
            if (kd_in == kZero) {
                const v4u z = vzero();
                v4u zv[K];
#pragma unroll
                for (int r = 0; r < K; ++r) zv[r] = z;
                for (uint32_t p = 0; p < P; ++p) {
                    const uint64_t lp = (uint64_t)p * TILE;
                    if (lp >= len) break;
                    store_rows_exact<T, K>(zv, aptr + lp, len - lp, ltid, active);
                }
                if (tid == 0 && job.ref_crc[g] != ~init) atomicMin(job.bad, (unsigned long long)g);
                continue;
            }
            const uint8_t* src = job.slot + (job.off[g] - job.slot_base);
            uint32_t acc = 0, padbad = 0;
            if (P == 1 && full && T >= 64) {
                // a whole one-tile chunk (uniform): no per-row bounds or padding
                constexpr uint32_t R = 16u * NT;
                v4u v[K];
#pragma unroll
                for (int r = 0; r < K; ++r) v[r] = gload(src + r * R + 16u * ltid);
#pragma unroll
                for (int r = 0; r < K; ++r) __builtin_nontemporal_store(v[r], (gv4*)(aptr + r * R + 16u * ltid));
                acc = crc_rows<K>(v, 0, s_dt);
            } else {
                for (uint32_t p = 0; p < P; ++p) {
                    const uint64_t lp = (uint64_t)p * TILE;
                    v4u v[K];
                    const uint64_t rem = len > lp ? len - lp : 0;
                    load_rows_staged<T, K>(v, src + lp, rem, ltid, active, &padbad);
                    if (rem) store_rows_exact<T, K>(v, aptr + lp, rem, ltid, active);
                    acc = crc_rows<K>(v, acc, s_dt);
                }
            }
            uint32_t raw = wg_xor_lds<NW>(gf_mul_v(acc, lc), s_red);
            const uint32_t pb = wg_any_lds<NW>(padbad != 0, s_any);
            if (!full) raw = gf_mul_v(raw, ad.tail_unshift);
            const uint32_t crc = ~(raw ^ init);
            if (tid == 0 && (crc != job.ref_crc[g] || pb)) atomicMin(job.bad, (unsigned long long)g);
            continue;
        } else {
            v4u v[K];
            uint32_t acc = 0, orw = 0;
            int any;
            // When the kind does not depend on the digest (a zero chunk, or no
            // previous digest for the allocation) the payload length follows
            // from the zero test alone: the aggregate is then published before
            // the digest is computed, so the successors' look-backs rarely wait
            // on this chunk.
            const uint64_t len16 = (len + 15u) & ~15u;
            bool early = MODE == kModeDump && (job.prev_crc == nullptr || ad.prev_first == ~0ull);
            if (P == 1) {
                load_rows<T, K>(v, aptr, len, ltid, active);
                if constexpr (MODE == kModeDump || MODE == kModeClassify) {
#pragma unroll
                    for (int r = 0; r < K; ++r) orw |= or4(v[r]);
                    any = wg_any_lds<NW>(orw != 0, s_any);
                    if constexpr (MODE == kModeDump) {
                        early = early || !any;
                        if (early && tid == 0) lb_publish(job.status, g - job.g0, any ? len16 : 0, job.epoch);
                    }
                    if (any) acc = crc_rows<K>(v, 0, s_dt);
                } else {
                    any = 1;
                    acc = crc_rows<K>(v, 0, s_dt);
                }
            } else {
                for (uint32_t p = 0; p < P; ++p) {
                    const uint64_t lp = (uint64_t)p * TILE;
                    load_rows<T, K>(v, aptr + lp, len > lp ? len - lp : 0, ltid, active);
#pragma unroll
                    for (int r = 0; r < K; ++r) orw |= or4(v[r]);
                    acc = crc_rows<K>(v, acc, s_dt);
                }
                any = (MODE == kModeDump || MODE == kModeClassify) ? wg_any_lds<NW>(orw != 0, s_any) : 1;
                early = early || (MODE == kModeDump && !any);
                if (early && tid == 0) lb_publish(job.status, g - job.g0, any ? len16 : 0, job.epoch);
            }
            uint32_t crc = ~init;
            if (any) {
                uint32_t raw = wg_xor_lds<NW>(gf_mul_v(acc, lc), s_red);
                if (!full) raw = gf_mul_v(raw, ad.tail_unshift);
                crc = ~(raw ^ init);
            }
            if constexpr (MODE == kModeDigest) {
                if (tid == 0) job.crc_out[g] = crc;
                continue;
            }
            if constexpr (MODE == kModeClassify) {
                // digest and kind only; offsets and payload come from later passes
                uint8_t kd = kData;
                if (!any) kd = kZero;
                else if (job.prev_crc != nullptr && ad.prev_first != ~0ull && job.prev_crc[ad.prev_first + k] == crc)
                    kd = kUnchanged;
                if (tid == 0) {
                    job.crc_out[g] = crc;
                    job.kind_out[g] = kd;
                }
                continue;
            }
            if constexpr (MODE == kModeVerify) {
                if (tid == 0 && crc != job.ref_crc[g]) atomicMin(job.bad, (unsigned long long)g);
                continue;
            }
            if constexpr (MODE == kModeDump) {
                uint8_t kd = kData;
                if (!any) kd = kZero;
                else if (job.prev_crc != nullptr && ad.prev_first != ~0ull && job.prev_crc[ad.prev_first + k] == crc)
                    kd = kUnchanged;
                if (tid == 0) {
                    job.crc_out[g] = crc;
                    job.kind_out[g] = kd;
                }
                const uint64_t plen = kd == kData ? len16 : 0;
                if (tid < 64) {
                    __builtin_amdgcn_s_setprio(3);   // as in k_dump_stream
                    const uint64_t e = early ? lb_walk(job.status, g - job.g0, plen, job.epoch, job.err)
                                             : lookback(job.status, g - job.g0, plen, job.epoch, job.err);
                    if (tid == 0) s_off = e;
                    __builtin_amdgcn_s_setprio(0);
                }
                lds_barrier();
                const uint64_t excl = s_off;
                if (kd == kData) {
                    uint8_t* dst = job.slot + excl;
                    if (P == 1) {
                        store_rows_padded<T, K>(v, dst, len16, ltid, active);
                    } else {
                        for (uint32_t p = 0; p < P; ++p) {
                            const uint64_t lp = (uint64_t)p * TILE;
                            if (lp >= len16) break;
                            load_rows<T, K>(v, aptr + lp, len - lp, ltid, active);
                            store_rows_padded<T, K>(v, dst + lp, len16 - lp, ltid, active);
                        }
                    }
                }
                if (g + 1 == job.g1 && tid == 0) *job.wtotal = excl + plen;
            }
        }
    }
}

// Loads through the scalar cache, for tables that no work-group writes
// while the kernel runs (descriptors, the chunk map, the previous digest
// table); the dispatch invalidates the scalar cache, so what earlier
// kernels wrote is seen. They stay off the vector memory counter, so
// waiting for them never waits for the streamed rows.
template <typename V>
__device__ inline V ld_const(const V* p) {
    return *(const __attribute__((address_space(4))) V*)(p);
}

// Where the ticket tk falls: its job, global chunk, allocation and chunk
// geometry. Every value is uniform across the work-group.
struct ChunkAt {
    uint32_t jj;            // job
    uint32_t len;           // valid bytes
    uint64_t g;             // global chunk of the job
    uint64_t k;             // chunk within its allocation
    uint64_t prev_first;    // first chunk of the allocation in the previous table, or ~0
    uint32_t tail_init;
    uint32_t tail_unshift;
    const uint8_t* ptr;     // first byte of the chunk
};

template <uint32_t C>
__device__ inline ChunkAt chunk_at(const JobList& jl, uint64_t tk) {
    ChunkAt c;
    uint32_t jj = 0;
    while (jj + 1 < jl.n_jobs && jl.prefix[jj + 1] <= tk) ++jj;
    const ChunkJob& job = jl.job[jj];
    c.jj = jj;
    c.g = job.g0 + (tk - jl.prefix[jj]);
    const uint32_t a = job.amap ? ld_const(job.amap + c.g) : find_alloc(job.allocs, job.n_allocs, c.g);
    const AllocDesc* ad = job.allocs + a;
    const uint64_t first = ld_const(&ad->first), size = ld_const(&ad->size);
    c.k = c.g - first;
    const uint64_t nk = (size + C - 1) / C;
    c.len = (c.k + 1 == nk) ? ld_const(&ad->tail_len) : C;
    c.prev_first = ld_const(&ad->prev_first);
    c.tail_init = ld_const(&ad->tail_init);
    c.tail_unshift = ld_const(&ad->tail_unshift);
    c.ptr = reinterpret_cast<const uint8_t*>(ld_const(&ad->ptr)) + c.k * C;
    return c;
}

typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) void glb_void;

// Dump mode for chunks of exactly one tile (C = 16 T K), streamed: while a
// work-group digests, scans and stores its current chunk from registers,
// the rows of its next chunk are already on their way -- the first K-1
// rows straight into LDS (global_load_lds_dwordx4: lane i of a wave lands
// at the wave's LDS base + 16 i, so every lane later reads back exactly the
// 16 bytes it requested and no barrier is needed between the waves), the
// last row into registers. HBM reads therefore stay in flight during the
// work-group's LDS lookups, barriers and look-back. In the last, partial
// chunk of an allocation only whole 16-byte blocks below its end are
// streamed; the block that straddles the end is read byte by byte and the
// blocks past it are zeros. Tickets: a work-group holds its current ticket,
// the next one (being streamed) and the one after (a value only); every
// ticket below its current one is held by a running work-group, so
// look-back waits end.
//
// With CLASSIFY the kernel is the first pass of a two-pass dump: digest and
// kind of every chunk, no look-back and no payload.
template <int T, int K, bool CLASSIFY>
__global__ void __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(4)))
k_dump_stream(JobList jl) {
    static_assert(T >= 64 && T % 64 == 0, "whole waves");
    constexpr int NW = T / 64;
    constexpr uint32_t R = 16u * T;       // bytes per row
    constexpr uint32_t C = R * K;         // the chunk is one tile
    constexpr uint32_t BUF = K > 1 ? (K - 1) * R : 16;
    // The tables at the start of LDS: every lookup's table offset then fits
    // the 16-bit offset field of the LDS read, and a lookup's address takes
    // one instruction (byte select and scale). The streamed rows follow.
    __shared__ struct __attribute__((aligned(16))) {
        uint32_t dt[16 * 256];
        uint8_t buf[BUF];
    } s_lds;
    uint32_t* const s_dt = s_lds.dt;
    uint8_t* const s_buf = s_lds.buf;
    __shared__ uint32_t s_red[NW];
    __shared__ uint32_t s_any[NW];
    __shared__ uint32_t s_tk[2];
    __shared__ uint64_t s_off;

    const int tid = threadIdx.x;
    const uint32_t wave = __builtin_amdgcn_readfirstlane((uint32_t)tid >> 6);
    const EngineConsts* ec = jl.job[0].ec;
    for (int i = tid; i < 16 * 256; i += T) s_dt[i] = ec->dt[i];
    const uint32_t lanec = ec->lane[tid];
    const uint32_t full_init = ec->full_init;
    const uint64_t total = jl.prefix[jl.n_jobs];
    if (tid == 0) {
        s_tk[0] = atomicAdd(jl.ticket, 1u);
        s_tk[1] = atomicAdd(jl.ticket, 1u);
    }
    __syncthreads();

    // start the whole 16-byte blocks of a chunk on their way (K-1 rows to
    // LDS, the last row to registers)
    auto stream = [&](const ChunkAt& c, v4u& last) {
        // this wave's reads of the buffer must be complete before it is refilled
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        const uint32_t o = (K - 1) * R + 16u * tid;
        if (c.len == C) {   // a whole chunk (uniform): no per-row bounds
#pragma unroll
            for (int r = 0; r < K - 1; ++r)
                __builtin_amdgcn_global_load_lds((glb_void*)(c.ptr + r * R + 16u * tid),
                                                 (lds_void*)(s_buf + r * R + wave * 1024u), 16, 0, 0);
            last = gload(c.ptr + o);
        } else {
#pragma unroll
            for (int r = 0; r < K - 1; ++r)
                if (r * R + 16u * tid + 16u <= c.len)
                    __builtin_amdgcn_global_load_lds((glb_void*)(c.ptr + r * R + 16u * tid),
                                                     (lds_void*)(s_buf + r * R + wave * 1024u), 16, 0, 0);
            last = o + 16u <= c.len ? gload(c.ptr + o) : vzero();
        }
    };

    uint64_t tk = (uint32_t)__builtin_amdgcn_readfirstlane(s_tk[0]);
    ChunkAt cur{};
    v4u last = vzero();
    if (tk < total) {
        cur = chunk_at<C>(jl, tk);
        stream(cur, last);
    }
    // zero test of the current chunk already taken (and its aggregate
    // published) in the previous iteration
    bool known = false;
    uint32_t any_known = 0;
    for (uint32_t it = 0;; ++it) {
        if (tk >= total) break;
        // the current chunk into registers (its streamed blocks have landed
        // once the vector memory counter drains)
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        v4u v[K];
        uint32_t orw = 0;
        if (cur.len == C) {
#pragma unroll
            for (int r = 0; r < K; ++r) {
                v[r] = r < K - 1 ? *reinterpret_cast<const v4u*>(s_buf + r * R + 16u * tid) : last;
                orw |= or4(v[r]);
            }
        } else {
#pragma unroll
            for (int r = 0; r < K; ++r) {
                const uint32_t o = r * R + 16u * tid;
                v4u x = r < K - 1 ? *reinterpret_cast<const v4u*>(s_buf + r * R + 16u * tid) : last;
                if (o + 16u > cur.len) x = o < cur.len ? load_partial(cur.ptr + o, cur.len - o) : vzero();
                v[r] = x;
                orw |= or4(x);
            }
        }
        // the ticket after next; its value is needed only at the end of the
        // iteration
        uint32_t tk2 = 0;
        if (tid == 0) tk2 = atomicAdd(jl.ticket, 1u);
        const uint64_t tk_next = (uint32_t)__builtin_amdgcn_readfirstlane(s_tk[(it + 1) & 1]);

        const ChunkJob& job = jl.job[cur.jj];
        const uint64_t g = cur.g;
        const uint32_t len = cur.len;
        const bool full = len == C;
        const uint32_t init = full ? full_init : cur.tail_init;
        const uint64_t len16 = (len + 15u) & ~15u;
        uint32_t lc = lanec;
        uint32_t ltid = (uint32_t)tid;
        asm volatile("" : "+v"(lc), "+v"(ltid));

        // (LDS-only barriers from here on: streamed blocks stay in flight)
        const uint32_t any = known ? any_known : wg_any_lds<NW>(orw != 0, s_any);
        // When the kind does not depend on the digest -- a zero chunk, or no
        // previous digest for the allocation -- the payload length follows
        // from the zero test: its aggregate is published now, before the
        // digest, so the successors' look-backs can pass this chunk while it
        // is still being digested. (The look-back's own walk comes after the
        // digest: its status loads wait on the vector memory counter, which
        // by then the next chunk's loads have cleared.)
        const bool early = !any || job.prev_crc == nullptr || cur.prev_first == ~0ull;
        if (!CLASSIFY && early && !known && tid == 0) lb_publish(job.status, g - job.g0, any ? len16 : 0, job.epoch);
        ChunkAt nxt{};
        if (tk_next < total) {
            nxt = chunk_at<C>(jl, tk_next);
            stream(nxt, last);
        }
        uint32_t acc = 0;
        if (any) acc = crc_rows<K>(v, 0, s_dt);
        if (tid == 0) s_tk[it & 1] = tk2;
        uint32_t raw = wg_xor_lds<NW>(gf_mul_v(acc, lc), s_red);
        if (!full) raw = gf_mul_v(raw, cur.tail_unshift);
        const uint32_t crc = ~(raw ^ init);
        uint8_t kd = kData;
        if (!any) kd = kZero;
        else if (!early && ld_const(job.prev_crc + cur.prev_first + cur.k) == crc) kd = kUnchanged;
        if (tid == 0) {
            job.crc_out[g] = crc;
            job.kind_out[g] = kd;
        }
        known = false;
        if constexpr (!CLASSIFY) {
            // the next chunk's blocks have had the digest's time to land: its
            // zero test now, and its aggregate published before this chunk's
            // look-back, so successors' look-backs pass it an iteration sooner
            if (tk_next < total) {
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                uint32_t orn = 0;
                if (nxt.len == C) {
#pragma unroll
                    for (int r = 0; r < K; ++r)
                        orn |= or4(r < K - 1 ? *reinterpret_cast<const v4u*>(s_buf + r * R + 16u * tid) : last);
                } else {
#pragma unroll
                    for (int r = 0; r < K; ++r) {
                        const uint32_t o = r * R + 16u * tid;
                        v4u x = r < K - 1 ? *reinterpret_cast<const v4u*>(s_buf + r * R + 16u * tid) : last;
                        if (o + 16u > nxt.len) x = o < nxt.len ? load_partial(nxt.ptr + o, nxt.len - o) : vzero();
                        orn |= or4(x);
                    }
                }
                any_known = wg_any_lds<NW>(orn != 0, s_any);
                known = true;
                const ChunkJob& jn = jl.job[nxt.jj];
                const bool early_n = !any_known || jn.prev_crc == nullptr || nxt.prev_first == ~0ull;
                if (early_n && tid == 0)
                    lb_publish(jn.status, nxt.g - jn.g0, any_known ? ((nxt.len + 15u) & ~15u) : 0, jn.epoch);
            }
            const uint64_t plen = kd == kData ? len16 : 0;
            if (tid < 64) {
                // the look-back wave at the highest priority: the work-group's
                // other waves wait for its result, while the CU's other
                // work-group keeps its memory streams going (-2 % kernel time)
                __builtin_amdgcn_s_setprio(3);
                const uint64_t e = early ? lb_walk(job.status, g - job.g0, plen, job.epoch, job.err)
                                         : lookback(job.status, g - job.g0, plen, job.epoch, job.err);
                if (tid == 0) s_off = e;
                __builtin_amdgcn_s_setprio(0);
            }
            lds_barrier();
            const uint64_t excl = s_off;
            if (kd == kData) {
                if (full) store_rows_padded<T, K, true>(v, job.slot + excl, C, ltid, true);
                else store_rows_padded<T, K, true>(v, job.slot + excl, len16, ltid, true);
            }
            if (g + 1 == job.g1 && tid == 0) *job.wtotal = excl + plen;
        }
        tk = tk_next;
        cur = nxt;
    }
}

__global__ void __launch_bounds__(256) k_offsets(OffJob job) {
    __shared__ uint32_t s_tk[2];
    __shared__ uint64_t s_wsum[4];
    __shared__ uint64_t s_off;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (uint32_t it = 0;; ++it) {
        if (tid == 0) s_tk[it & 1] = atomicAdd(job.ticket, 1u);
        __syncthreads();
        const uint64_t tile = __builtin_amdgcn_readfirstlane(s_tk[it & 1]);
        const uint64_t g0 = tile * 256;
        if (g0 >= job.n_chunks) break;
        const uint64_t g = g0 + tid;
        uint64_t plen = 0;
        uint32_t cz = 0, cd = 0, cu = 0, ci = 0;
        const uint64_t gg = job.g_base + g;   // global chunk
        if (g < job.n_chunks) {
            const uint8_t kd = job.kind[gg];
            const uint32_t a = job.amap ? job.amap[gg] : find_alloc(job.allocs, job.n_allocs, gg);
            const uint64_t first = job.allocs[a].first, size = job.allocs[a].size;
            const uint64_t nk = (size + job.C - 1) / job.C;
            const uint64_t len = (gg - first + 1 == nk) ? job.allocs[a].tail_len : job.C;
            if (kd == kData) { plen = (len + 15) & ~15ull; cd = 1; }
            else if (kd == kZero) cz = 1;
            else if (kd == kUnchanged) cu = 1;
            else ci = 1;
        }
        // block scan of plen
        uint64_t x = plen;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint64_t y = __shfl_up(x, d);
            if (lane >= d) x += y;
        }
        if (lane == 63) s_wsum[wave] = x;
        // kind counts
        const uint64_t bz = __ballot(cz), bd = __ballot(cd), bu = __ballot(cu), bi = __ballot(ci);
        if (lane == 0) {
            if (bz) atomicAdd(&job.counts[0], (unsigned long long)__popcll(bz));
            if (bd) atomicAdd(&job.counts[1], (unsigned long long)__popcll(bd));
            if (bu) atomicAdd(&job.counts[2], (unsigned long long)__popcll(bu));
            if (bi) atomicAdd(&job.counts[3], (unsigned long long)__popcll(bi));
        }
        __syncthreads();
        uint64_t before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            before += w < wave ? s_wsum[w] : 0;
            total += s_wsum[w];
        }
        const uint64_t local = before + x - plen;
        if (tid < 64) {
            const uint64_t e = lookback(job.status, tile, total, job.epoch, job.err);
            if (tid == 0) s_off = e;
        }
        __syncthreads();
        const uint64_t o = s_off + local;
        if (g < job.n_chunks) {
            job.off[gg] = o;
            if (g % job.per_window == 0) job.wb[g / job.per_window] = o;
            if (g + 1 == job.n_chunks) job.wb[job.n_windows] = o + plen;
        }
    }
}

__global__ void k_gate(GateJob j) {
    if (threadIdx.x != 0) return;
    const uint32_t tcrc = gf_mul_v(j.dig[0], j.xlen) ^ j.dig[1];
    const bool ok = tcrc == (uint32_t)j.expect[0] && j.counts[3] == 0 && j.counts[2] == 0 &&
                    j.counts[0] + j.counts[1] == j.n_chunks && *j.total == j.expect[1];
    *j.gate = ok ? 1u : 0u;
}

__device__ inline uint32_t xpow8(uint64_t n, const uint32_t* x2n) {   // x^(8n)
    uint32_t r = kOne;
    for (int b = 3; n; n >>= 1, ++b)
        if (n & 1) r = gf_mul_v(r, x2n[b]);
    return r;
}

__global__ void __launch_bounds__(256) k_combine(CombineJob job) {
    __shared__ uint32_t s_red[4];
    __shared__ uint32_t s_x2n[64];
    const int tid = threadIdx.x;
    if (tid < 64) s_x2n[tid] = job.ec->x2n[tid];
    __syncthreads();
    const uint32_t a = blockIdx.x;
    const AllocDesc ad = job.allocs[a];
    const uint64_t C = job.C;
    const uint64_t nk = (ad.size + C - 1) / C;
    const uint64_t m = (nk + 255) / 256;
    const uint64_t k0 = (uint64_t)tid * m, k1 = k0 + m < nk ? k0 + m : nk;
    uint32_t contrib = 0;
    if (k0 < k1) {
        const uint32_t full_x = job.ec->full_x;
        uint32_t acc = 0;
        for (uint64_t k = k0; k < k1; ++k) {
            const uint32_t xk = (k + 1 == nk) ? ad.tail_x : full_x;
            acc = gf_mul_v(acc, xk) ^ job.crc[ad.first + k];
        }
        const uint64_t end = k1 == nk ? ad.size : k1 * C;
        contrib = gf_mul_v(acc, xpow8(ad.size - end, s_x2n));
    }
    const uint32_t crc = wg_xor<4>(contrib, s_red);
    if (tid == 0) {
        if (job.mode == kCombineWrite) {
            uint8_t* rec = job.recs + 32ull * a;
            reinterpret_cast<uint64_t*>(rec)[0] = ad.id;
            reinterpret_cast<uint64_t*>(rec)[1] = ad.size;
            reinterpret_cast<uint64_t*>(rec)[2] = ad.first;
            reinterpret_cast<uint32_t*>(rec)[6] = crc;
            reinterpret_cast<uint32_t*>(rec)[7] = 0;
        } else if (job.mode == kCombineCheck) {
            const uint32_t want = reinterpret_cast<const uint32_t*>(job.recs + 32ull * a)[6];
            if (want != crc) atomicMin(job.bad, (unsigned long long)ad.first);
        } else {
            job.out[a] = crc;
        }
    }
}

// Chunk -> allocation map: work-group a writes a over its chunk range.
__global__ void __launch_bounds__(256) k_chunk_map(const AllocDesc* allocs, uint32_t n, uint32_t C, uint32_t* map) {
    for (uint32_t a = blockIdx.x; a < n; a += gridDim.x) {
        const uint64_t first = allocs[a].first, nk = (allocs[a].size + C - 1) / C;
        for (uint64_t k = threadIdx.x; k < nk; k += blockDim.x) map[first + k] = a;
    }
}

// Two descriptors passed by value (kernel arguments are captured at launch,
// so the host copy may go away at once, also inside a captured graph).
__global__ void k_store_descs(AllocDesc* dst, AllocDesc a, AllocDesc b) {
    if (threadIdx.x == 0) {
        dst[0] = a;
        dst[1] = b;
    }
}

__global__ void k_fill64(uint64_t* p, uint64_t v, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill32(uint32_t* p, uint32_t v, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <int T, int K>
hipError_t launch_tk(int mode, const JobList& jl, int grid, hipStream_t s) {
    constexpr int NT = T < 64 ? 64 : T;
    switch (mode) {
        case kModeDump:
            if constexpr (T >= 64) {
                if (jl.job[0].C == 16u * T * K) {
                    hipLaunchKernelGGL((k_dump_stream<T, K, false>), dim3(grid), dim3(T), 0, s, jl);
                    break;
                }
            }
            hipLaunchKernelGGL((k_chunks<T, K, kModeDump>), dim3(grid), dim3(NT), 0, s, jl);
            break;
        case kModeClassify:
            if constexpr (T >= 64) {
                if (jl.job[0].C == 16u * T * K) {
                    hipLaunchKernelGGL((k_dump_stream<T, K, true>), dim3(grid), dim3(T), 0, s, jl);
                    break;
                }
            }
            hipLaunchKernelGGL((k_chunks<T, K, kModeClassify>), dim3(grid), dim3(NT), 0, s, jl);
            break;
        case kModeDigest: hipLaunchKernelGGL((k_chunks<T, K, kModeDigest>), dim3(grid), dim3(NT), 0, s, jl); break;
        case kModeVerify: hipLaunchKernelGGL((k_chunks<T, K, kModeVerify>), dim3(grid), dim3(NT), 0, s, jl); break;
        case kModeRestore: hipLaunchKernelGGL((k_chunks<T, K, kModeRestore>), dim3(grid), dim3(NT), 0, s, jl); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int T, int K>
hipError_t occ_tk(int mode, int* n) {
    constexpr int NT = T < 64 ? 64 : T;
    switch (mode) {
        case kModeDump: {
            // the smaller of the two dump kernels' residencies (which one
            // runs depends on the chunk size)
            hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(n, k_chunks<T, K, kModeDump>, NT, 0);
            if constexpr (T >= 64) {
                int m = 0;
                if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&m, k_dump_stream<T, K, false>, T, 0);
                if (e == hipSuccess && m < *n) *n = m;
            }
            return e;
        }
        case kModeClassify: {
            hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(n, k_chunks<T, K, kModeClassify>, NT, 0);
            if constexpr (T >= 64) {
                int m = 0;
                if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&m, k_dump_stream<T, K, true>, T, 0);
                if (e == hipSuccess && m < *n) *n = m;
            }
            return e;
        }
        case kModeDigest: return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, k_chunks<T, K, kModeDigest>, NT, 0);
        case kModeVerify: return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, k_chunks<T, K, kModeVerify>, NT, 0);
        case kModeRestore: return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, k_chunks<T, K, kModeRestore>, NT, 0);
        default: return hipErrorInvalidValue;
    }
}

// the work-group shapes that are compiled
#define MK_TILES(X) \
    X(1, 1) X(2, 1) X(4, 1) X(8, 1) X(16, 1) X(32, 1) \
    X(64, 1) X(64, 4) X(256, 1) X(256, 4) X(256, 8) X(512, 4) X(512, 8) X(1024, 4) X(1024, 8)

}  // namespace

bool tile_supported(int T, int K) {
#define MK_TEST(t, k) if (T == t && K == k) return true;
    MK_TILES(MK_TEST)
#undef MK_TEST
    return false;
}

hipError_t launch_chunks(int T, int K, int mode, const JobList& jl, int grid, hipStream_t s) {
    if (jl.n_jobs < 1 || jl.n_jobs > (uint32_t)kMaxJobs) return hipErrorInvalidValue;
#define MK_LAUNCH(t, k) if (T == t && K == k) return launch_tk<t, k>(mode, jl, grid, s);
    MK_TILES(MK_LAUNCH)
#undef MK_LAUNCH
    return hipErrorInvalidValue;
}

hipError_t chunks_occupancy(int T, int K, int mode, int* n) {
#define MK_OCC(t, k) if (T == t && K == k) return occ_tk<t, k>(mode, n);
    MK_TILES(MK_OCC)
#undef MK_OCC
    return hipErrorInvalidValue;
}

hipError_t launch_offsets(const OffJob& job, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_offsets, dim3(grid), dim3(256), 0, s, job);
    return hipGetLastError();
}

hipError_t launch_gate(const GateJob& job, hipStream_t s) {
    hipLaunchKernelGGL(k_gate, dim3(1), dim3(64), 0, s, job);
    return hipGetLastError();
}

hipError_t launch_combine(const CombineJob& job, hipStream_t s) {
    if (job.n_allocs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_combine, dim3(job.n_allocs), dim3(256), 0, s, job);
    return hipGetLastError();
}

hipError_t launch_chunk_map(const AllocDesc* allocs, uint32_t n_allocs, uint32_t C, uint32_t* map, hipStream_t s) {
    if (n_allocs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_chunk_map, dim3(n_allocs < 4096 ? n_allocs : 4096), dim3(256), 0, s, allocs, n_allocs, C, map);
    return hipGetLastError();
}

hipError_t launch_store_descs(AllocDesc* dst, const AllocDesc& a, const AllocDesc& b, hipStream_t s) {
    hipLaunchKernelGGL(k_store_descs, dim3(1), dim3(64), 0, s, dst, a, b);
    return hipGetLastError();
}

hipError_t launch_fill64(uint64_t* p, uint64_t v, uint64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill64, dim3(blocks < 1024 ? (unsigned)blocks : 1024u), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill32, dim3(blocks < 1024 ? (unsigned)blocks : 1024u), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

}  // namespace mk
