// Gather of DATA chunks to their payload records (gfx950): the last pass of
// the three-pass delta dump and of the codec dump, after the payload offsets
// are known.
#pragma once
#include <hip/hip_runtime.h>

#include "common.h"

namespace mk {

struct GatherJob {
    const AllocDesc* allocs;
    const uint32_t* amap;    // allocation of chunk g (required)
    uint64_t g0, g1;         // chunks [g0, g1)
    uint32_t C;
    uint32_t pad;
    const uint8_t* kind;     // only DATA chunks are copied
    const uint64_t* off;     // payload offset of chunk g
    uint8_t* slot;           // payload buffer holding offsets from slot_base
    uint64_t slot_base;
};

// Grid-stride over the chunks: a chunk that is not DATA costs one uniform
// byte load, a DATA chunk is copied in 16-byte blocks, its last partial block
// byte by byte and zero-padded to 16 bytes.
hipError_t launch_gather(const GatherJob& j, int grid, hipStream_t s);

}  // namespace mk
