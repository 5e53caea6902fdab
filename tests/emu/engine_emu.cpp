// CPU emulation of the GPU chunk engine's CRC decomposition (and of the
// codec decode kernel's), for testing the constants on a machine without a
// GPU. It reproduces the
// per-lane interleaved streams, the fold of the running digest into the
// next block, the lane alignment, the tail
// correction and the per-allocation combine exactly as the kernels do, using
// the library's own constant builder; the tests compare its results with
// the SSE4.2 hardware CRC-32C.
#include <string.h>
#include <vector>

#include "codec_consts.h"
#include "common.h"
#include "hostmath.h"

using namespace mk;

static uint32_t blk16(const uint8_t* b, const EngineConsts& ec) {
    uint32_t h = 0;
    for (int j = 0; j < 16; ++j) h ^= ec.dt[j * 256 + b[j]];
    return h;
}

extern "C" uint32_t emu_chunk_crc(const uint8_t* p, uint32_t len, uint32_t C, int T, int K) {
    static EngineConsts ec;
    build_engine_consts(&ec, T, C);
    const uint32_t R = 16u * T, TILE = R * K, P = C / TILE;
    uint32_t raw = 0;
    for (int t = 0; t < T; ++t) {
        uint32_t acc = 0;
        for (uint32_t pp = 0; pp < P; ++pp)
            for (int r = 0; r < K; ++r) {
                uint8_t blk[16];
                const uint32_t o = pp * TILE + r * R + 16u * t;
                for (int j = 0; j < 16; ++j) blk[j] = (o + j < len) ? p[o + j] : 0;
                for (int j = 0; j < 4; ++j) blk[j] ^= (uint8_t)(acc >> (8 * j));   // fold the running digest
                acc = blk16(blk, ec);
            }
        raw ^= gf_mul(acc, ec.lane[t]);
    }
    uint32_t init = ec.full_init;
    if (len != C) {
        raw = gf_mul(raw, xinvpow8(C - len));
        init = gf_mul(0xFFFFFFFFu, xpow8(len));
    }
    return ~(raw ^ init);
}

// per-allocation CRC from chunk CRCs, as the combine kernel does it with
// `threads` lanes
extern "C" uint32_t emu_alloc_crc(const uint32_t* crcs, uint64_t size, uint32_t C, int threads) {
    const uint64_t nk = (size + C - 1) / C;
    if (!nk) return 0;
    const uint32_t tail = (uint32_t)(size - (nk - 1) * C);
    const uint64_t m = (nk + threads - 1) / threads;
    uint32_t out = 0;
    for (int t = 0; t < threads; ++t) {
        const uint64_t k0 = t * m, k1 = k0 + m < nk ? k0 + m : nk;
        if (k0 >= k1) continue;
        uint32_t acc = 0;
        for (uint64_t k = k0; k < k1; ++k) acc = gf_mul(acc, k + 1 == nk ? xpow8(tail) : xpow8(C)) ^ crcs[k];
        const uint64_t end = k1 == nk ? size : k1 * C;
        out ^= gf_mul(acc, xpow8(size - end));
    }
    return out;
}

extern "C" uint32_t emu_combine(uint32_t a, uint32_t b, uint64_t len_b) { return crc_combine(a, b, len_b); }

// the codec decode kernel's digest of a full chunk of C bytes: 256 lanes,
// lane t over its C/256 consecutive bytes 16 at a time (running value folded
// into the next row), lane digests moved into place and xored, preset term
extern "C" uint32_t emu_codec_crc(const uint8_t* p, uint32_t C) {
    static CodecConsts cc;
    build_codec_consts(&cc, C);
    const uint32_t seg = C / 256;
    uint32_t raw = 0;
    for (int t = 0; t < 256; ++t) {
        uint32_t crc = 0;
        for (uint32_t r = 0; r < seg / 16; ++r) {
            uint8_t b[16];
            memcpy(b, p + (uint64_t)t * seg + 16u * r, 16);
            for (int j = 0; j < 4; ++j) b[j] ^= (uint8_t)(crc >> (8 * j));
            uint32_t c = 0;
            for (int i = 0; i < 16; ++i) c ^= cc.tab[i * 256 + b[i]];
            crc = c;
        }
        raw ^= gf_mul(crc, cc.lane[t]);
    }
    return ~(raw ^ cc.full_init);
}
