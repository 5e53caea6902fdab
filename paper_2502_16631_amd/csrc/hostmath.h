// Host-side arithmetic of the library: CRC-32C of host bytes (SSE4.2
// instruction), powers of x modulo the CRC polynomial, and the engine
// constant block for a (work-group width, chunk size) pair.
#pragma once
#include <stdint.h>

#include "common.h"

namespace mk {

// CRC-32C of host memory (preset and final complement), continuing from a
// previous CRC value `prev` of the bytes before (0 for a fresh message).
uint32_t host_crc32c(const void* p, uint64_t n, uint32_t prev = 0);

// CRC(A || B) from CRC(A), CRC(B) and |B|.
uint32_t crc_combine(uint32_t crc_a, uint32_t crc_b, uint64_t len_b);

// x^(8n) and x^(-8n) modulo P (reflected representation).
uint32_t xpow8(uint64_t n);
uint32_t xinvpow8(uint64_t n);

// Fill the constant block for work-group width T (threads per chunk) and
// chunk size C.
void build_engine_consts(EngineConsts* ec, int T, uint32_t C);

}  // namespace mk
