// Shared definitions of the GPU library: GF(2) arithmetic modulo the CRC-32C
// polynomial, the device descriptors and the engine constant block.
//
// CRC-32C here is the reflected Castagnoli CRC (polynomial 0x1EDC6F41, bit
// reversed 0x82F63B78, register preset to all ones, final complement). In the
// reflected representation bit 31 of a word is the coefficient of x^0 and
// bit 0 the coefficient of x^31.
//
// Notation used throughout:
//   r(M)        raw CRC: the register after feeding M into a register that
//               starts at 0, with no final complement (linear in M);
//   CRC(M)      = ~( (~0) * x^(8|M|)  xor  r(M) )    (preset, complement);
//   r(A || B)   = r(A) * x^(8|B|)  xor  r(B);
//   r(0^z || M) = r(M)                   (leading zeros change nothing);
//   r(M || 0^z) = r(M) * x^(8z);
//   CRC(A || B) = CRC(A) * x^(8|B|)  xor  CRC(B)     (the combine identity:
//               the preset terms cancel because CRC is affine).
// Products are polynomial products modulo P over GF(2).
#pragma once
#include <stdint.h>

#ifndef __HIPCC__
#define __host__
#define __device__
#endif

namespace mk {

constexpr uint32_t kPoly = 0x82F63B78u;   // P without the x^32 term, reflected
constexpr uint32_t kOne = 0x80000000u;    // the polynomial 1
constexpr uint32_t kX1 = 0x40000000u;     // the polynomial x

enum : uint8_t { kZero = 0, kData = 1, kUnchanged = 2, kPacked = 3 };   // kPacked: byte-plane record

// b * x mod P
__host__ __device__ inline uint32_t gf_xtimes(uint32_t b) {
    return (b >> 1) ^ ((b & 1u) ? kPoly : 0u);
}

// a * b mod P, bit-serial over the coefficients of a (x^0 first).
__host__ __device__ inline uint32_t gf_mul(uint32_t a, uint32_t b) {
    uint32_t p = 0;
#ifdef __HIP_DEVICE_COMPILE__
#pragma unroll
#endif
    for (int i = 0; i < 32; ++i) {
        p ^= ((a >> (31 - i)) & 1u) ? b : 0u;
        b = gf_xtimes(b);
    }
    return p;
}

// Per-allocation descriptor used by every chunk kernel (64 bytes).
// Chunk k of the allocation covers [k*C, min((k+1)*C, size)); the last
// ("tail") chunk may be short. Its CRC is computed over the chunk zero-
// extended to C bytes and corrected by multiplying with tail_unshift.
struct AllocDesc {
    uint64_t ptr;          // device address (16-byte aligned)
    uint64_t size;         // bytes
    uint64_t first;        // global index of the allocation's first chunk
    uint64_t prev_first;   // first chunk of the matching allocation in the
                           // previous digest table, or ~0 if none
    uint64_t id;           // caller id
    uint32_t tail_len;     // bytes of the last chunk (0 if size == 0)
    uint32_t tail_unshift; // x^(-8 (C - tail_len))
    uint32_t tail_init;    // (~0) * x^(8 tail_len): the preset's term
    uint32_t tail_x;       // x^(8 tail_len): shift of the combine over the tail
    uint32_t pad[2];
};
static_assert(sizeof(AllocDesc) == 64, "descriptor layout");

// Engine constants for one (work-group width T, chunk size C) pair. The
// chunk kernels copy the tables into LDS once per persistent work-group.
//   dt[j][x]  = r(byte x followed by 15-j zero bytes) * x^(8G), G = 16 (T-1):
//               the digest of a 16-byte block followed by the G bytes that
//               separate it from the lane's next block (the other lanes'
//               share of the row, read as zeros) is the xor of dt[j][byte j]
//               over its 16 bytes. A lane's running digest is folded into
//               the first four bytes of its next block before the lookups
//               (r(M || B) = r((r(M) as 4 bytes xor B[0..3]) || B[4..15]), so
//               no separate step advances it over a row;
//   lane[t]   = x^(-8 * 16 t): lane t's stream then ends G bytes past the
//               end of the tile; this moves it back to its own position.
struct EngineConsts {
    uint32_t dt[16 * 256];
    uint32_t lane[1024];
    uint32_t full_init;    // (~0) * x^(8C)
    uint32_t full_x;       // x^(8C)
    uint32_t pad0[2];
    uint32_t x2n[64];      // x^(2^i)
    uint32_t pad1[60];
};

// Look-back status word: flag (2 bits) | epoch (22 bits) | value (40 bits).
constexpr uint64_t kStAgg = 1ull << 62;
constexpr uint64_t kStInc = 2ull << 62;
constexpr uint64_t kStValueMask = (1ull << 40) - 1;
constexpr uint32_t kEpochMask = (1u << 22) - 1;

}  // namespace mk
