// Launch interface of the chunk kernels (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include "common.h"

namespace mk {

// classify: digest and kind of every chunk, nothing else (first pass of a
// two-pass dump; its last pass, the gather, is k_gather in gather.hip).
enum Mode : int { kModeDump = 0, kModeDigest = 1, kModeVerify = 2, kModeRestore = 3, kModeClassify = 4 };

// One launch of the chunk engine over global chunks [g0, g1).
struct ChunkJob {
    const AllocDesc* allocs;
    uint32_t n_allocs;
    uint32_t C;                  // chunk size
    const uint32_t* amap;        // allocation of chunk g at [g], or nullptr (binary search)
    uint64_t g0, g1;
    const EngineConsts* ec;      // tables for (T, C)
    uint32_t* crc_out;           // dump / digest / classify: digest of chunk g at [g]
    uint8_t* kind_out;           // dump / classify: kind of chunk g at [g]
    const uint8_t* kind_in;      // verify / restore: kind of chunk g
    const uint32_t* ref_crc;     // verify / restore: expected digest of chunk g
    const uint32_t* prev_crc;    // dump / classify: previous digest table or nullptr
    uint8_t* slot;               // staging window (dump: written; restore: read)
    const uint64_t* off;         // restore: payload offset of chunk g
    uint64_t slot_base;          // restore: payload offset of the window start
    uint64_t* status;            // dump: look-back status, indexed by g - g0
    uint64_t* wtotal;            // dump: payload bytes of the window
    unsigned long long* bad;     // verify / restore: lowest failing chunk (init ~0)
    uint32_t* err;               // internal error flag (look-back time-out)
    uint32_t epoch;              // look-back epoch of this launch (1 .. 2^22-1)
    uint32_t flags;              // kJob*
    const uint32_t* gate;        // restore / verify: when set and 0 at launch, the launch does nothing
};
// verify mode: check every chunk of the range whatever its kind (the strict
// re-read after a restore), not only UNCHANGED ones
constexpr uint32_t kJobVerifyAll = 1;

// Several jobs in one persistent launch (continuous batching): the jobs'
// chunk ranges are laid end to end in one ticket space; every job keeps its
// own descriptors, tables, staging window and look-back scope, so a job's
// result does not depend on what it shares the launch with. All jobs of a
// launch use the same chunk size and tile shape (one set of LDS tables).
constexpr int kMaxJobs = 16;
struct JobList {
    ChunkJob job[kMaxJobs];
    uint64_t prefix[kMaxJobs + 1];   // ticket range of job j: [prefix[j], prefix[j+1])
    uint32_t* ticket;                // shared ticket counter, zero before launch
    uint32_t n_jobs;
    uint32_t pad;
};

// Payload offsets of every chunk from the kind table (restore).
struct OffJob {
    const AllocDesc* allocs;
    uint32_t n_allocs;
    uint32_t C;
    const uint32_t* amap;        // allocation of chunk g, or nullptr
    uint64_t n_chunks;
    const uint8_t* kind;
    uint64_t* off;               // [n_chunks]
    uint64_t per_window;         // chunks per staging window G
    uint64_t* wb;                // [W + 1] payload offset at each window start, wb[W] = total
    uint64_t n_windows;          // W
    uint64_t* status;            // look-back, one word per tile
    uint32_t* ticket;
    unsigned long long* counts;  // [4]: zero, data, unchanged, invalid (zeroed before launch)
    uint32_t* err;
    uint32_t epoch;
    uint32_t pad;
    uint64_t g_base;             // the scan covers global chunks [g_base, g_base + n_chunks); off, kind
                                 // and amap are indexed globally, windows and wb relative to g_base
};

// Per-allocation combine of chunk digests into the whole-allocation CRC.
enum CombineMode : int { kCombineWrite = 0, kCombineCheck = 1, kCombineOut = 2 };
struct CombineJob {
    const AllocDesc* allocs;
    uint32_t n_allocs;
    uint32_t C;
    const uint32_t* crc;         // chunk digests (global index)
    const EngineConsts* ec;      // full_x and x2n for this C
    uint8_t* recs;               // write: AllocRec[n] (32 bytes each); check: read alloc_crc
    uint32_t* out;               // out mode: CRC of allocation a at [a]
    unsigned long long* bad;     // check mode
    int mode;
    int pad;
};

// Validation of a restore inside a captured graph: *gate = 1 when the
// tables digest combined from the device's two halves equals the expected
// value, the kinds are all ZERO or DATA and the payload total equals the
// expected D; else 0 (the gated kernels then write nothing).
struct GateJob {
    const uint32_t* dig;                 // [2]: digest of AllocRec || crc[], of kind[] || pad
    uint32_t xlen;                       // x^(8 len(kind[] || pad))
    uint32_t pad;
    const unsigned long long* counts;    // [4]: zero, data, unchanged, invalid
    const uint64_t* total;               // payload total of the offsets scan
    uint64_t n_chunks;
    const uint64_t* expect;              // [2]: tables digest, D (written before each launch)
    uint32_t* gate;
};

bool tile_supported(int T, int K);
hipError_t launch_gate(const GateJob& job, hipStream_t s);
hipError_t launch_chunks(int T, int K, int mode, const JobList& jl, int grid, hipStream_t s);
hipError_t chunks_occupancy(int T, int K, int mode, int* blocks_per_cu);
hipError_t launch_offsets(const OffJob& job, int grid, hipStream_t s);
hipError_t launch_combine(const CombineJob& job, hipStream_t s);
hipError_t launch_chunk_map(const AllocDesc* allocs, uint32_t n_allocs, uint32_t C, uint32_t* map, hipStream_t s);
hipError_t launch_store_descs(AllocDesc* dst, const AllocDesc& a, const AllocDesc& b, hipStream_t s);
hipError_t launch_fill64(uint64_t* p, uint64_t v, uint64_t n, hipStream_t s);
hipError_t launch_fill32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s);

}  // namespace mk
