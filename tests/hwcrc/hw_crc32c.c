/* Cross-check only: CRC-32C from the x86 SSE4.2 crc32 instruction, an
 * implementation in hardware that shares nothing with the oracle's table
 * code. Used by the CPU tests to pin the oracle; never linked into it. */
#include <nmmintrin.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

uint32_t hw_crc32c(const uint8_t* p, uint64_t n) {
    uint64_t c = 0xFFFFFFFFu;
    while (n >= 8) { uint64_t v; memcpy(&v, p, 8); c = _mm_crc32_u64(c, v); p += 8; n -= 8; }
    uint32_t c32 = (uint32_t)c;
    while (n--) c32 = _mm_crc32_u8(c32, *p++);
    return ~c32;
}
