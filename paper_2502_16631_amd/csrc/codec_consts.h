// Constant block of the codec's decode digest (host and device).
#pragma once
#include <stdint.h>

namespace mk {

// For one chunk size C. A lane digests its consecutive rows 16 bytes at a
// time: the running value is xored into the first four bytes of the next
// row, whose raw CRC is the xor of tab[i][byte i] over its 16 bytes.
struct CodecConsts {
    uint32_t tab[16 * 256];   // tab[i][x] = r(byte x followed by 15 - i zero bytes)
    uint32_t lane[256];       // x^(8 (C/256) (255 - t)): moves lane t's segment digest
                              // to its place in the chunk
    uint32_t full_init;       // (~0) * x^(8C): the preset's term
    uint32_t pad[63];
};

// Fill the block for chunk size C (256 lanes of C/256 bytes each).
void build_codec_consts(CodecConsts* cc, uint32_t C);

}  // namespace mk
