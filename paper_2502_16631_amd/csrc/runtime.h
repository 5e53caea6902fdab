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



// A device buffer that grows on demand. With ext set it is a fixed slice of
// memory the buffer does not own (the no-allocation dump's static array):
// it never allocates or frees, and asking for more than its size fails.
struct DevBuf {
    void* p = nullptr;
    uint64_t cap = 0;
    bool ext = false;
    hipError_t ensure(uint64_t n) {
        if (n <= cap) return hipSuccess;
        if (ext) return hipErrorOutOfMemory;
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
        if (p && !ext) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
    void attach(void* q, uint64_t n) {   // a fixed slice (ext)
        p = q;
        cap = n;
        ext = true;
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

// Look-back status words of one buffer (flag | epoch | value). Every launch
// that uses the buffer takes the next epoch of the buffer's own counter, so
// no word left by an earlier launch carries the current epoch: the buffer
// is cleared when it is (re)allocated (fresh device memory may hold any
// words) and when its counter wraps.
struct StatusBuf {
    DevBuf buf;
    uint32_t epoch = 0;
    hipError_t ensure(uint64_t bytes, hipStream_t s) {
        if (bytes <= buf.cap) return hipSuccess;
        if (buf.ext) return hipErrorOutOfMemory;
        hipError_t e = buf.ensure(bytes);
        if (e != hipSuccess) return e;
        epoch = 0;
        return launch_fill64(buf.as<uint64_t>(), 0, buf.cap / 8, s);
    }
    // the epoch of the next launch on stream s (clears the words on a wrap)
    hipError_t next(hipStream_t s, uint32_t* ep) {
        if (++epoch > kEpochMask) {
            epoch = 1;
            hipError_t e = launch_fill64(buf.as<uint64_t>(), 0, buf.cap / 8, s);
            if (e != hipSuccess) return e;
        }
        *ep = epoch;
        return hipSuccess;
    }
    uint64_t* words() const { return buf.as<uint64_t>(); }
    void release() {
        buf.release();
        epoch = 0;
    }
};

// A captured single-window dump stage (batched form): replayed whenever the
// same table shape is dumped again with the same buffers. It owns its
// look-back words (cleared inside the graph at every replay, which reuses
// the epoch taken at capture).
struct GraphEntry {
    uint64_t key = 0;
    hipGraphExec_t exec = nullptr;
    DevBuf descs, dig, status;
    uint64_t last_use = 0;
};

// A resident digest table of an image: its crc[] on the device, kept for
// later delta dumps taken against that image. While pins > 0 a request in
// flight reads it and it is never evicted.
struct DigestEntry {
    DevBuf crc;
    uint64_t n_chunks = 0;
    uint64_t last_use = 0;
    uint32_t pins = 0;
};

// Eviction rule of the resident digest tables: the least recently used
// entry that no request has pinned, or `none` when every entry is pinned.
template <class Map>
typename Map::key_type digest_victim(const Map& m, typename Map::key_type none) {
    typename Map::key_type v = none;
    uint64_t best = ~0ull;
    for (const auto& kv : m)
        if (kv.second.pins == 0 && kv.second.last_use < best) {
            best = kv.second.last_use;
            v = kv.first;
        }
    return v;
}



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
    uint64_t use_clock = 0;
    // device buffers
    mk::StatusBuf status;
    mk::DevBuf descs, ctl, arc, kinds, prevcrc, off, wb, staging, dig, amap, rlen, cmeta;
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
    hipEvent_t ev_order = nullptr;                        // orders the main stream after the caller's
    hipEvent_t sev[8] = {};                               // timing events of the per-stage report
    mk::EngineConsts* hconsts = nullptr;                  // host build space of engine constants
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

// A dump into fixed buffers: every device buffer is a slice of one device
// array of kNaBytes (layout below), the image goes to the caller's host
// buffer, and nothing is allocated (no device, pinned, stream or event
// allocation; the context's set-up made those). Layout (byte offsets, every
// region 256-byte aligned; the look-back words come first and nothing else is
// ever written there, so words left by earlier calls carry older epochs of
// the array's own counter):
constexpr uint64_t kNaBytes = 128ull << 20;
constexpr uint32_t kNaMaxAllocs = 16384;
constexpr uint64_t kNaMaxChunks = 1ull << 20;
constexpr uint64_t kNaStatusWords = 1ull << 18;     // chunks per staging window, at most (less 64)
constexpr uint64_t na_round(uint64_t x) { return (x + 255) & ~255ull; }
constexpr uint64_t kNaTables = na_round(32ull * kNaMaxAllocs + 5 * kNaMaxChunks + 32);
constexpr uint64_t kNaStatus = 0;
constexpr uint64_t kNaCtl = kNaStatus + 8 * kNaStatusWords;
constexpr uint64_t kNaConsts = kNaCtl + (64 << 10);          // chunk engine constants (T, C)
constexpr uint64_t kNaDConsts = kNaConsts + (32 << 10);      // table-digest engine constants
constexpr uint64_t kNaDig = kNaDConsts + (32 << 10);
constexpr uint64_t kNaDescs = kNaDig + (64 << 10);
constexpr uint64_t kNaAmap = kNaDescs + 64ull * kNaMaxAllocs;
constexpr uint64_t kNaArc = kNaAmap + 4 * kNaMaxChunks;
constexpr uint64_t kNaKinds = kNaArc + kNaTables;
constexpr uint64_t kNaPrev = kNaKinds + kNaTables;
constexpr uint64_t kNaStaging = kNaPrev + 4 * kNaMaxChunks;
constexpr uint64_t kNaSlot = ((kNaBytes - kNaStaging) / 2) & ~4095ull;   // two staging slots
static_assert(sizeof(EngineConsts) <= (32 << 10), "engine constants region");
static_assert(kNaStaging + 2 * kNaSlot <= kNaBytes && kNaSlot >= (32ull << 20), "array layout");

// One device's array: its address, its look-back words with their own epoch
// counter, which engine constants it holds; mu serializes the calls that use
// it within this process.
struct NaDevice {
    std::mutex mu;
    uint8_t* ptr = nullptr;
    StatusBuf status;
    bool cleared = false;
    int T = 0;
    uint32_t C = 0;
    bool dconsts = false;
};

// A fixed-buffer dump: the caller's host buffer and the device's array
// (its lock held by the caller for the whole call).
struct NaCall {
    uint8_t* out;
    uint64_t cap;
    NaDevice* dev;
    uint64_t* len;   // receives the image length
};
// Address of the array of `device`, looked up once per device with that
// device current (the context's set-up calls it).
hipError_t na_setup(int device);
// The context's lock must be held. Fails with CKPT_ELIMIT beyond the array's
// limits, before any work is queued.
int dump_fixed(ckpt_ctx* c, const ckpt_alloc_table* table, const ckpt_image* prev, const ckpt_opts* o,
               void* stream, ckpt_result* res, const NaCall& na);

void fill_result(ckpt_result* res);   // a fresh report: zeros, no bad chunk
// A small pinned host buffer; when the driver's pinned limit is reached,
// cached image buffers of the pinned pool are given back until it succeeds.
hipError_t pinned_small(void** p, uint64_t n);
ckpt_image* image_new(uint64_t cap);
void image_release(ckpt_image* im);   // returns the memory (pool or heap) and deletes im
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
// The resident digest table of image uid (nc chunks), or nullptr. With pin
// the entry is pinned until digest_unpin: it stays resident while a request
// that outlives this call reads it.
const uint32_t* digest_lookup(ckpt_ctx* c, uint64_t uid, uint64_t nc, bool pin = false);
void digest_unpin(ckpt_ctx* c, uint64_t uid);

// Table digests on the device (state digest and kinds digest), in two halves
// so that a captured graph can hold the second.
struct DigestPlan {
    int T = 0, K = 0;
    const EngineConsts* ec = nullptr;
    uint64_t nk = 0;
    uint8_t* base = nullptr;
    uint64_t off_crc = 0, off_out = 0, off_tk = 0;
};
// ec: the engine constants for the digest tile (T 256, C 16 KiB), or nullptr
// to take them from the context's cache.
hipError_t digest_prepare(ckpt_ctx* c, DevBuf* dig, const uint8_t* recs_crc, uint64_t len_a,
                          const uint8_t* kinds_pad, uint64_t len_b, DigestPlan* p, hipStream_t s,
                          const EngineConsts* ec = nullptr);
hipError_t digest_enqueue(ckpt_ctx* c, const DigestPlan& p, uint32_t* out_host, hipStream_t s);

}  // namespace mk
