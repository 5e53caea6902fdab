// Internal declarations shared by the runtime sources (runtime.hip,
// serve.hip): the context and image objects and the host-side helpers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/mickpt.h"
#include "codec.h"
#include "gather.h"
#include "common.h"
#include "kernels.h"

namespace mk {

// Fields of an image in host memory (format v1), after checking the header
// digest, the sizes and the allocation grid. With check_tables the tables
// digest, the kinds (and record lengths of the codec layout) and the payload
// length are checked as well and state_digest is filled in.
struct ImageView {
    uint32_t flags = 0, C = 0, n_allocs = 0, base_state = 0, tables_crc = 0, state_digest = 0;
    uint64_t n_chunks = 0, D = 0, N = 0, tl = 0;
    const uint8_t* recs = nullptr;
    const uint8_t* crcs = nullptr;
    const uint8_t* rlens = nullptr;   // u32 record lengths (codec layout), else nullptr
    const uint8_t* kinds = nullptr;
    const uint8_t* payload = nullptr;
};

int parse_image(const uint8_t* img, uint64_t len, ImageView* v, bool check_tables);
// Payload record length of chunk g (len = its length in bytes): 0 for ZERO
// and UNCHANGED, round16(len) for DATA, the table's value for PACKED; or
// kBadRecord when the kind or the record length breaks the format.
constexpr uint64_t kBadRecord = ~0ull;
uint64_t record_len(const ImageView& v, uint64_t g, uint64_t len);



struct DevBuf {
    void* p = nullptr;
    uint64_t cap = 0;
    hipError_t ensure(uint64_t n) {
        if (n <= cap) return hipSuccess;
        if (p) {
            hipError_t e = hipFree(p);
            if (e != hipSuccess) return e;
            p = nullptr;
            cap = 0;
        }
        uint64_t want = std::max<uint64_t>(n, 256);
        hipError_t e = hipMalloc(&p, want);
        if (e != hipSuccess) {
            (void)hipGetLastError();   // reported through the return value only
            p = nullptr;
            return e;
        }
        cap = want;
        return hipSuccess;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

// A captured single-window dump stage (batched form): replayed whenever the
// same table shape is dumped again with the same buffers.
struct GraphEntry {
    uint64_t key = 0;
    hipGraphExec_t exec = nullptr;
    DevBuf descs, dig;
    uint64_t last_use = 0;
};

// A resident digest table of an image: its crc[] on the device, kept for
// later delta dumps taken against that image.
struct DigestEntry {
    DevBuf crc;
    uint64_t n_chunks = 0;
    uint64_t last_use = 0;
};



constexpr uint64_t kNoChunk = ~0ull;
constexpr uint64_t kHeader = 64;
constexpr uint32_t kDefaultChunk = 65536;

uint64_t now_ns();
inline uint64_t round16(uint64_t n) { return (n + 15) & ~15ull; }
inline uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
inline bool valid_chunk(uint64_t c) { return c >= 16 && c <= (1ull << 30) && (c & (c - 1)) == 0; }
inline uint64_t tables_len(uint64_t n, uint64_t nc, bool codec = false) {
    return round16(32 * n + (codec ? 9 : 5) * nc);
}
constexpr uint32_t kFlagDelta = 1, kFlagCodec = 2;
inline void put32(uint8_t* p, uint32_t v) { memcpy(p, &v, 4); }
inline void put64(uint8_t* p, uint64_t v) { memcpy(p, &v, 8); }
inline uint32_t get32(const uint8_t* p) { uint32_t v; memcpy(&v, p, 4); return v; }
inline uint64_t get64(const uint8_t* p) { uint64_t v; memcpy(&v, p, 8); return v; }

}  // namespace mk

// An image in host memory: pinned when the driver grants it (the pinned
// pool), else pageable (copies through it are slower).
struct ckpt_image {
    uint8_t* p = nullptr;
    uint64_t n = 0;
    uint64_t cap = 0;
    uint64_t uid = 0;   // identity: key of the image's resident digest table
    bool pinned = true;
};

struct ckpt_ctx {
    int device = 0;
    uint64_t budget = 0;
    size_t digest_capacity = 8;                           // resident digest tables kept
    int num_cu = 0;
    hipStream_t s_main = nullptr;
    std::vector<hipStream_t> s_copy;
    std::mutex mu;
    uint32_t epoch = 0;
    uint64_t use_clock = 0;
    // device buffers
    mk::DevBuf descs, status, ctl, arc, kinds, prevcrc, off, wb, staging, dig, amap, rlen, cmeta;
    std::map<std::pair<int, uint32_t>, mk::DevBuf> consts;    // (T, C) -> EngineConsts
    std::map<uint32_t, mk::DevBuf> cconsts;                   // C -> CodecConsts
    std::map<std::tuple<int, int, int>, int> occ;          // (T, K, mode) -> blocks per CU
    std::unordered_map<uint64_t, mk::DigestEntry> digests;    // image uid -> resident crc[]
    std::vector<mk::GraphEntry> graphs;                       // captured dump stages (LRU)
    std::map<uint64_t, std::pair<ckpt_opts, double>> tuned;  // table shape class -> best options
    // pinned host scratch for small transfers
    uint8_t* hsmall = nullptr;
    uint64_t hsmall_cap = 0;
    // pinned host scratch for per-chunk tables, and a second compute stream
    // (codec dumps: encode on it while the main stream sizes later pieces)
    uint8_t* hpin = nullptr;
    uint64_t hpin_cap = 0;
    hipStream_t s_aux = nullptr;
    hipStream_t s_meta = nullptr;   // small host <-> device table transfers
    std::vector<hipEvent_t> events;
    std::vector<hipEvent_t> tevents;                      // timing events (begin, end) per launch
};

namespace mk {

// Plain restores of at least this many bytes held by one staging window are
// launched as all chunks but the last 1/64, then those.
constexpr uint64_t kTailMinBytes = 512ull << 20;

// Storage hooks. A dump told of a sink reports every payload copy into the
// image as it is queued (segments of at most kSinkSegment bytes), so the
// image can go to a file while the rest is still being copied; a restore
// given a gate waits, before uploading each staging window, until the
// image's bytes up to the window's end are in host memory.
constexpr uint64_t kSinkSegment = 256ull << 20;
struct PayloadSink {
    virtual ~PayloadSink() = default;
    virtual void begin(ckpt_image* im) = 0;                                    // before the first copy into im
    virtual hipError_t issued(hipStream_t s, uint64_t lo, uint64_t hi) = 0;    // image bytes [lo, hi), queued on s
    virtual void end() = 0;   // no more copies; returns once nothing of the sink reads the image
};
struct LoadGate {
    virtual ~LoadGate() = default;
    virtual bool wait(uint64_t hi) = 0;   // image bytes [0, hi) loaded; false when loading failed
};
int dump_impl(ckpt_ctx* c, const ckpt_alloc_table* table, const ckpt_image* prev, ckpt_image** out,
              const ckpt_opts* o, void* stream, ckpt_result* res, PayloadSink* sink);
int restore_impl(ckpt_ctx* c, const ckpt_image* img, const ckpt_alloc_table* table, const ckpt_opts* o,
                 void* stream, ckpt_result* res, bool some, LoadGate* gate);

ckpt_image* image_new(uint64_t cap);
void image_release(ckpt_image* im);   // returns the memory (pool or heap) and deletes im
uint32_t next_epoch(ckpt_ctx* c, bool* wrapped);
void pick_tile(uint32_t C, uint32_t want_t, int* T, int* K);
hipError_t get_consts(ckpt_ctx* c, int T, uint32_t C, const EngineConsts** out);
hipError_t get_codec_consts(ckpt_ctx* c, uint32_t C, const CodecConsts** out);
int unpack_grid(const ckpt_ctx* c, uint64_t chunks);
int pack_grid(const ckpt_ctx* c, uint64_t chunks);
hipError_t grid_for(ckpt_ctx* c, int T, int K, int mode, uint64_t work, int* grid);
void make_desc(AllocDesc* d, uint64_t id, const void* ptr, uint64_t size, uint64_t first, uint64_t prev_first,
               uint32_t C);
JobList one_job(const ChunkJob& j, uint32_t* ticket);
void digest_insert(ckpt_ctx* c, uint64_t uid, const uint32_t* crc_dev, uint64_t nc, hipStream_t s);
const uint32_t* digest_lookup(ckpt_ctx* c, uint64_t uid, uint64_t nc);

// Table digests on the device (state digest and kinds digest), in two halves
// so that a captured graph can hold the second.
struct DigestPlan {
    int T = 0, K = 0;
    const EngineConsts* ec = nullptr;
    uint64_t nk = 0;
    uint8_t* base = nullptr;
    uint64_t off_crc = 0, off_out = 0, off_tk = 0;
};
hipError_t digest_prepare(ckpt_ctx* c, DevBuf* dig, const uint8_t* recs_crc, uint64_t len_a,
                          const uint8_t* kinds_pad, uint64_t len_b, DigestPlan* p, hipStream_t s);
hipError_t digest_enqueue(ckpt_ctx* c, const DigestPlan& p, uint32_t* out_host, hipStream_t s);

}  // namespace mk
