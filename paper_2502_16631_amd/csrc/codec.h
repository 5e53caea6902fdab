// Byte-plane codec of full-length DATA chunks (kind kPacked), gfx950.
//
// The paper names data compression among the techniques that could speed up
// checkpoint and restore of large models (section 5.2) and among the
// optimisations its method can take on (section 7); it defines no codec.
// This one targets what a device's memory holds in training and HPC jobs:
// arrays of 2-, 4- and 8-byte numbers whose high (sign / exponent) bytes take
// few values. A chunk of C bytes is read as 8 byte planes (plane p = bytes
// p, p+8, p+16, ...; element e of plane p is byte 8e+p); each plane is stored
//   CONST  one value (16-byte section),
//   DICT   a 15-entry dictionary of its most frequent bytes (count
//          descending, value ascending), 4-bit codes (15 = escape, low
//          nibble first) and the escaped bytes in element order,
//   RAW    its bytes,
// in 16-byte-aligned sections after a 48-byte head (u8 mode[8], u32 esc[8],
// 8 zero bytes). DICT is chosen when its section is shorter than RAW; the
// record replaces the chunk only when it is shorter than C. The image then
// carries a u32 record-length table after the digest table.
//
// Work-group shape: 256 threads. In the encode and decode kernels lane t owns
// the C/4096 consecutive 16-byte rows starting at row t*C/4096, so its
// elements of every plane are consecutive: its codes and raw bytes are one
// aligned piece of each section (written or read with whole 16-byte accesses
// where they are that long) and one block scan gives every lane its escape
// positions. Records are written and read in global memory directly.
#pragma once
#include <hip/hip_runtime.h>

#include "codec_consts.h"
#include "kernels.h"

namespace mk {

constexpr uint32_t kCodecMinChunk = 4096;    // one 16-byte row per lane
constexpr uint32_t kCodecMaxChunk = 65536;   // records are staged in LDS
constexpr int kCodecThreads = 256;
constexpr uint64_t kCodecPieces = 8;         // a codec dump's encode / copy-out pipeline depth
constexpr uint32_t kRecordHead = 48;
// What the size pass keeps of a PACKED chunk for its encode: the record head
// (48 bytes), the 8 planes' 16-byte dictionaries and their used entries
// (8 bytes), padded to 192 bytes.
constexpr uint32_t kPackMeta = 192;
enum : uint32_t { kPlaneRaw = 0, kPlaneConst = 1, kPlaneDict = 2 };

inline bool codec_chunk_supported(uint32_t C) { return C >= kCodecMinChunk && C <= kCodecMaxChunk; }

// Constants of the decode kernel's digest: CodecConsts (codec_consts.h).

// Size and encode passes over the chunks [g0, g1) of one table.
struct PackJob {
    const AllocDesc* allocs;
    const uint32_t* amap;    // allocation of chunk g (required)
    uint64_t g0, g1;
    uint32_t C;
    uint32_t pad;
    uint8_t* kind;           // size: DATA becomes PACKED where the record is shorter
    uint32_t* rlen;          // size: record length of every chunk (written); encode: read
    const uint64_t* off;     // encode: payload offset of chunk g in slot
    uint8_t* slot;           // encode: staging holding the payload from offset slot_base
    uint64_t slot_base;
    uint32_t* err;           // encode: set when a record's length differs from the size pass
    uint8_t* meta;           // kPackMeta bytes per chunk (global index): size: written for PACKED
                             // chunks; encode: read, in place of a second histogram
};

// encode = false: size pass; true: encode pass (PACKED chunks to slot + off[g]).
hipError_t launch_pack(const PackJob& j, bool encode, int grid, hipStream_t s);
// Decode, store and verify the PACKED chunks of the jobs' ranges (restore):
// uses allocs, amap, g0/g1, kind_in, ref_crc, slot, off, slot_base and bad of
// each job; rlen is the image's record-length table (global chunk index).
hipError_t launch_unpack(const JobList& jl, const uint32_t* rlen, const CodecConsts* cc, int grid, hipStream_t s);

}  // namespace mk
