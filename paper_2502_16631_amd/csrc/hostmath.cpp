// Host arithmetic: see hostmath.h.
#include "hostmath.h"
#include "codec_consts.h"

#include <nmmintrin.h>
#include <string.h>

namespace mk {

__attribute__((target("sse4.2"))) uint32_t host_crc32c(const void* p, uint64_t n, uint32_t prev) {
    const uint8_t* b = static_cast<const uint8_t*>(p);
    uint64_t c = ~prev & 0xFFFFFFFFu;
    // three interleaved streams would be faster; tables and headers are small
    while (n >= 8) {
        uint64_t v;
        memcpy(&v, b, 8);
        c = _mm_crc32_u64(c, v);
        b += 8;
        n -= 8;
    }
    uint32_t c32 = static_cast<uint32_t>(c);
    while (n--) c32 = _mm_crc32_u8(c32, *b++);
    return ~c32;
}

namespace {

struct PowTables {
    // pw[i][j] = x^(8 * j * 256^i), i = 0..7 covers every 64-bit n
    uint32_t pw[8][256];
    uint32_t ipw[8][256];   // the inverses
    PowTables() {
        // x^8 and x^-8
        uint32_t x8 = kOne;
        for (int i = 0; i < 8; ++i) x8 = gf_xtimes(x8);
        // x^-1: the unique y with y * x = 1 (undo one shift step)
        const uint32_t c = kOne ^ kPoly;                 // top bit of c is 0
        const uint32_t xinv = (c << 1) | 1u;
        uint32_t xinv8 = kOne;
        for (int i = 0; i < 8; ++i) xinv8 = gf_mul(xinv8, xinv);
        uint32_t base = x8, ibase = xinv8;               // x^(8 * 256^i)
        for (int i = 0; i < 8; ++i) {
            pw[i][0] = kOne;
            ipw[i][0] = kOne;
            for (int j = 1; j < 256; ++j) {
                pw[i][j] = gf_mul(pw[i][j - 1], base);
                ipw[i][j] = gf_mul(ipw[i][j - 1], ibase);
            }
            base = gf_mul(pw[i][255], base);             // ^256
            ibase = gf_mul(ipw[i][255], ibase);
        }
    }
};

const PowTables& tables() {
    static const PowTables t;
    return t;
}

}  // namespace

uint32_t xpow8(uint64_t n) {
    const PowTables& t = tables();
    uint32_t r = kOne;
    for (int i = 0; n; ++i, n >>= 8)
        if (n & 255) r = gf_mul(r, t.pw[i][n & 255]);
    return r;
}

uint32_t xinvpow8(uint64_t n) {
    const PowTables& t = tables();
    uint32_t r = kOne;
    for (int i = 0; n; ++i, n >>= 8)
        if (n & 255) r = gf_mul(r, t.ipw[i][n & 255]);
    return r;
}

uint32_t crc_combine(uint32_t crc_a, uint32_t crc_b, uint64_t len_b) {
    return gf_mul(crc_a, xpow8(len_b)) ^ crc_b;
}

void build_engine_consts(EngineConsts* ec, int T, uint32_t C) {
    memset(ec, 0, sizeof(*ec));
    // raw CRC of one byte followed by (15 - j) zero bytes and by the gap of
    // 16 (T - 1) bytes to the lane's next block
    const uint32_t gap = xpow8(16ull * (uint64_t)(T - 1));
    for (uint32_t x = 0; x < 256; ++x) {
        uint32_t r = x;
        for (int i = 0; i < 8; ++i) r = gf_xtimes(r);   // r(x) = x * x^8 ... in register form
        for (int j = 15; j >= 0; --j) {
            ec->dt[j * 256 + x] = gf_mul(r, gap);
            r = gf_mul(r, xpow8(1));
        }
    }
    for (int t = 0; t < 1024; ++t) ec->lane[t] = t < T ? xinvpow8(16ull * (uint64_t)t) : 0u;
    ec->full_x = xpow8(C);
    ec->full_init = gf_mul(0xFFFFFFFFu, ec->full_x);
    uint32_t p = kX1;
    for (int i = 0; i < 64; ++i) {
        ec->x2n[i] = p;
        p = gf_mul(p, p);
    }
}

void build_codec_consts(CodecConsts* cc, uint32_t C) {
    for (uint32_t b = 0; b < 256; ++b) {
        uint32_t r = b;   // r(byte b): the register after one byte from 0
        for (int i = 0; i < 8; ++i) r = (r >> 1) ^ ((r & 1u) ? kPoly : 0u);
        for (int i = 0; i < 16; ++i) cc->tab[i * 256 + b] = gf_mul(r, xpow8(15 - i));
    }
    const uint64_t seg = C / 256;   // bytes per lane
    for (int t = 0; t < 256; ++t) cc->lane[t] = xpow8(seg * (uint64_t)(255 - t));
    cc->full_init = gf_mul(0xFFFFFFFFu, xpow8(C));
    for (uint32_t& x : cc->pad) x = 0;
}

}  // namespace mk
