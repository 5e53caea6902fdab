// Served form: a request loop over one context.
//
// Requests (dump or restore of one tenant's allocation table) are queued by
// any thread. A scheduler thread admits them in arrival order while a lane
// (per-request device buffers) is free and the staging they need (two
// windows) fits the budget, then drives every admitted request through its
// windows. Continuous batching: on every tick the next ready window of every
// active dump request goes into one persistent launch of the chunk engine
// (a job list, one job per request), and likewise for restores, so requests
// that arrive while others are on the GPU join the next launch. Each job
// keeps its own descriptors, tables, staging window and look-back scope, so
// a request's image is the same whether it runs alone or in a mix.
//
// Pipelines per request are those of the plain form (runtime.hip): dump =
// windows (kernel -> payload length -> D2H copy) then tables and header;
// restore = validation (tables digest, offsets, counts), a base check for
// deltas, then windows (H2D copy -> kernel), then the per-allocation check.
// Tenants' digest tables stay resident in the context (keyed by image) for
// their incremental dumps.
//
// Host memory. A copy between the device and a pageable host image returns
// only once it is done (the runtime stages it through pinned buffers on the
// calling thread), and so would stall every request on the scheduler
// thread. Such copies, and the allocation of dump images, go to a pool of
// host worker threads (each with a stream of its own); the scheduler learns
// of their completion from per-lane flags instead of events. Dump images
// are pinned while the pinned pool grants them (the driver pins a limited
// amount per process), pageable beyond. Small tables of pageable images go
// through a pinned bounce buffer of the lane.
#include <hip/hip_runtime.h>

#include <stdlib.h>

#include <atomic>
#include <condition_variable>
#include <deque>
#include <memory>
#include <thread>
#include <unordered_set>

#include "hostmath.h"
#include "runtime.h"

using namespace mk;

namespace {

constexpr uint64_t kDefaultSlot = 256ull << 20;

// Flags a lane's host work reports through (stored or counted by a worker
// thread with release order once the work is done): pieces copied out of
// dump slot 0 / 1 and into restore slot 0 / 1 for the window the slot holds
// (counts), the dump image allocated (1), a failed task (kTaskFailed). All
// are cleared when a request is given the lane. A window's copy is split
// into pieces of kCopyPiece bytes, so that several workers move one window.
enum { kFlDown0 = 0, kFlUp0 = 2, kFlAlloc = 4, kFlFail = 5, kLaneFlags = 6 };
constexpr uint64_t kTaskFailed = ~0ull;
constexpr uint64_t kCopyPiece = 64ull << 20;

struct Lane {
    DevBuf descs, arc, kinds, ctl, off, wb, staging, dig, prevcrc, amap;
    StatusBuf status;
    uint8_t* hs = nullptr;   // pinned: per-window payload lengths / offsets, digests, flags
    uint64_t hs_cap = 0;
    uint8_t* ht = nullptr;   // pinned bounce buffer for the tables of pageable images
    uint64_t ht_cap = 0;
    std::atomic<uint64_t>* fl = nullptr;   // kLaneFlags flags (owned by the server)
    uint64_t win[4] = {};                   // the window whose pieces fl[0..3] count
    uint64_t need[4] = {};                  // how many pieces it has
    hipError_t ensure_ht(uint64_t n) {
        if (n <= ht_cap) return hipSuccess;
        if (ht) hipHostFree(ht);
        ht = nullptr;
        ht_cap = 0;
        hipError_t e = pinned_small((void**)&ht, n);
        if (e == hipSuccess) ht_cap = n;
        return e;
    }
    std::vector<hipEvent_t> ev;   // per window: kernel done (dump) or copy done (restore)
    hipEvent_t slot_ev[2] = {nullptr, nullptr};   // dump: copy of the slot done; restore: kernel done
    hipEvent_t fin = nullptr;
    bool busy = false;
    hipError_t ensure_hs(uint64_t n) {
        if (n <= hs_cap) return hipSuccess;
        if (hs) hipHostFree(hs);
        hs = nullptr;
        hs_cap = 0;
        hipError_t e = pinned_small((void**)&hs, n);
        if (e == hipSuccess) hs_cap = n;
        return e;
    }
    hipError_t ensure_events(size_t n) {
        auto mk_ev = [](hipEvent_t* e) { return hipEventCreateWithFlags(e, hipEventDisableTiming); };
        for (int i = 0; i < 2; ++i)
            if (!slot_ev[i] && mk_ev(&slot_ev[i]) != hipSuccess) return hipErrorOutOfMemory;
        if (!fin && mk_ev(&fin) != hipSuccess) return hipErrorOutOfMemory;
        while (ev.size() < n) {
            hipEvent_t e;
            if (mk_ev(&e) != hipSuccess) return hipErrorOutOfMemory;
            ev.push_back(e);
        }
        return hipSuccess;
    }
    void release() {
        DevBuf* b[] = {&descs, &arc, &kinds, &ctl, &off, &wb, &staging, &dig, &prevcrc, &amap};
        for (DevBuf* x : b) x->release();
        status.release();
        for (hipEvent_t e : ev) hipEventDestroy(e);
        for (hipEvent_t e : slot_ev) if (e) hipEventDestroy(e);
        if (fin) hipEventDestroy(fin);
        if (hs) hipHostFree(hs);
        if (ht) hipHostFree(ht);
    }
};

enum Phase { kQueued, kAlloc, kValidate, kVerify, kRun, kFinal, kDrain, kDone };

struct Req {
    uint64_t ticket = 0;
    ckpt_request rq{};
    std::vector<ckpt_alloc> table;
    uint64_t t_submit = 0, t_admit = 0, t_done = 0;
    int rc = 0;
    ckpt_image* out = nullptr;
    Phase phase = kQueued;
    bool retired = false;      // done and out of the scheduler's lists: may be polled and freed
    int lane = -1;
    // plan
    uint32_t C = 0;
    uint32_t n = 0;
    uint64_t nc = 0, tl = 0, upper = 0, per = 0, W = 0, N = 0;
    std::vector<AllocDesc> d;
    const uint32_t* prev_dev = nullptr;
    uint64_t prev_pinned = 0;  // uid of the resident digest table pinned for this request, or 0
    uint32_t prev_digest = 0;
    ImageView v;               // restore: the image
    // progress
    uint64_t launched = 0;     // windows whose kernel is enqueued
    uint64_t staged = 0;       // restore: windows whose H2D copy is enqueued
    uint64_t copied = 0;       // dump: windows whose D2H copy is enqueued
    uint64_t pos = 0;          // dump: payload bytes so far
    uint64_t nu = 0;           // restore: UNCHANGED chunks
    bool pinned = true;        // the host image (dump: out, restore: img) is pinned
    uint64_t alloc_bytes = 0;  // dump: image size to allocate
    int drain_rc = 0;          // kDrain: the result once the request's host tasks are done
    std::atomic<uint32_t> tasks{0};   // host tasks queued or running for this request
};

// Host work for the worker threads.
struct HostTask {
    enum Kind { kD2H, kH2D, kAlloc } kind;
    Req* r;
    void* dst;
    const void* src;
    uint64_t n;
    hipEvent_t after;              // device work to wait for first (nullptr: none)
    std::atomic<uint64_t>* flag;   // copy: raised by one when done; allocation: set to value
    uint64_t value;
    std::atomic<uint64_t>* fail;   // copy: set to kTaskFailed on a failure
};

}  // namespace

struct ckpt_server {
    ckpt_ctx* ctx = nullptr;
    uint32_t max_active = 0;
    uint64_t budget = 0, slot = kDefaultSlot, reserved = 0;
    hipStream_t s_dump = nullptr, s_rest = nullptr, s_up = nullptr, s_down = nullptr;
    DevBuf tickets;                 // shared ticket counters of merged launches
    uint32_t ticket_next = 0;
    std::vector<Lane> lanes;
    std::thread th;
    std::mutex mu;
    std::condition_variable cv, done_cv;
    bool stop = false;
    std::deque<Req*> pending;
    std::vector<Req*> active;
    std::unordered_map<uint64_t, Req*> reqs;   // all not yet polled
    uint64_t next_ticket = 1;
    uint64_t in_system = 0;                    // submitted and not completed
    // stats
    uint64_t submitted = 0, completed = 0, failed = 0, bytes_logical = 0, bytes_link = 0, launches = 0,
             max_batch = 0, wait_sum = 0, max_wait = 0;
    std::atomic<uint64_t> host_copies{0}, host_copy_bytes{0};
    std::vector<uint64_t> lat;
    // host workers
    std::unique_ptr<std::atomic<uint64_t>[]> flags;   // kLaneFlags per lane
    std::vector<std::thread> workers;
    std::mutex tmu;
    std::condition_variable tcv;
    std::deque<HostTask> tasks;
    bool tstop = false;
};

namespace {

// Called by the scheduler thread with the context's lock held.
void finish(ckpt_server* s, Req* r, int rc) {
    r->rc = rc;
    r->t_done = now_ns();
    if (r->prev_pinned) {
        digest_unpin(s->ctx, r->prev_pinned);   // no launch of the request reads it any more
        r->prev_pinned = 0;
    }
    if (rc != CKPT_OK && r->out) {
        ckpt_image_free(r->out);
        r->out = nullptr;
    }
    std::lock_guard<std::mutex> g(s->mu);
    if (r->lane >= 0) {
        s->lanes[r->lane].busy = false;
        s->reserved -= 2 * s->slot;
        r->lane = -1;
    }
    s->completed++;
    if (rc != CKPT_OK) s->failed++;
    else {
        s->bytes_logical += r->N;
        s->bytes_link += kHeader + r->tl + (r->rq.kind == CKPT_REQ_DUMP ? r->pos : r->v.D);
    }
    s->lat.push_back(r->t_done - r->t_submit);
    const uint64_t wait = (r->t_admit ? r->t_admit : r->t_done) - r->t_submit;
    s->wait_sum += wait;
    s->max_wait = std::max(s->max_wait, wait);
    s->in_system--;
    r->phase = kDone;
    s->done_cv.notify_all();
}

// A request that failed after admission: it ends (kDone) once no host task
// of it is queued or running and the server's streams have drained, so that
// nothing still reads or writes its lane when the lane is handed on.
void fail_req(ckpt_server* s, Req* r, int rc) {
    (void)s;
    if (r->phase == kDrain || r->phase == kDone) return;
    r->drain_rc = rc;
    r->phase = kDrain;
}

void drain_step(ckpt_server* s, Req* r) {
    if (r->tasks.load(std::memory_order_acquire) != 0) return;
    hipStream_t ss[] = {s->s_dump, s->s_rest, s->s_up, s->s_down};
    for (hipStream_t x : ss) (void)hipStreamSynchronize(x);
    (void)hipGetLastError();
    finish(s, r, r->drain_rc);
}

// Queue host work for the workers; the task counts as the request's until
// the worker is done with it.
void host_task(ckpt_server* s, HostTask t) {
    t.r->tasks.fetch_add(1, std::memory_order_acq_rel);
    {
        std::lock_guard<std::mutex> g(s->tmu);
        s->tasks.push_back(t);
    }
    s->tcv.notify_one();
}

// A worker: takes tasks in order. A copy that involves pageable memory runs
// synchronously on the worker's own stream; its slot's piece count is
// raised (release) before the request's task count drops, and the worker
// touches neither after that. An allocation stores its flag.
void worker(ckpt_server* s) {
    (void)hipSetDevice(s->ctx->device);
    hipStream_t st = nullptr;
    const bool have_stream = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
    for (;;) {
        HostTask t;
        {
            std::unique_lock<std::mutex> g(s->tmu);
            s->tcv.wait(g, [s] { return s->tstop || !s->tasks.empty(); });
            if (s->tasks.empty()) break;   // stopping, and nothing left to do
            t = s->tasks.front();
            s->tasks.pop_front();
        }
        Req* r = t.r;
        if (t.kind == HostTask::kAlloc) {
            ckpt_image* im = image_new(t.n);   // the image of a dump
            r->out = im;   // read by the scheduler only after the flag
            t.flag->store(im ? t.value : kTaskFailed, std::memory_order_release);
        } else {
            hipError_t e = have_stream ? hipSuccess : hipErrorOutOfMemory;
            if (e == hipSuccess && t.after) e = hipEventSynchronize(t.after);
            if (e == hipSuccess && t.n)
                e = hipMemcpyAsync(t.dst, t.src, t.n,
                                   t.kind == HostTask::kD2H ? hipMemcpyDeviceToHost : hipMemcpyHostToDevice, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                t.fail->store(kTaskFailed, std::memory_order_release);
            } else {
                s->host_copies++;
                s->host_copy_bytes += t.n;
            }
            t.flag->fetch_add(1, std::memory_order_release);
        }
        r->tasks.fetch_sub(1, std::memory_order_acq_rel);
    }
    if (st) (void)hipStreamDestroy(st);
}

// Dump slot x % 2 holds no payload still to be copied out of window x.
bool down_done(const Req* r, const Lane& L, uint64_t x) {
    if (r->pinned) return hipEventQuery(L.slot_ev[x % 2]) == hipSuccess;
    const int f = kFlDown0 + (int)(x % 2);
    return L.win[f] == x && L.fl[f].load(std::memory_order_acquire) == L.need[f];
}

// Restore slot x % 2 holds the payload of window x.
bool up_done(const Lane& L, uint64_t x) {
    const int f = kFlUp0 + (int)(x % 2);
    return L.win[f] == x && L.fl[f].load(std::memory_order_acquire) == L.need[f];
}

// A host task of the request's lane failed.
bool lane_failed(const Lane& L) {
    return L.fl[kFlAlloc].load(std::memory_order_acquire) == kTaskFailed ||
           L.fl[kFlFail].load(std::memory_order_acquire) == kTaskFailed;
}

// A window's copy between a staging slot and a pageable image, in pieces of
// kCopyPiece bytes for the workers; slot flag f then counts them.
void host_copy(ckpt_server* s, Req* r, Lane& L, int f, uint64_t w, HostTask::Kind kind, uint8_t* dst,
               const uint8_t* src, uint64_t len, hipEvent_t after) {
    const uint64_t k = ceil_div(len, kCopyPiece);
    L.win[f] = w;
    L.need[f] = k;
    L.fl[f].store(0, std::memory_order_relaxed);   // published to the workers by the queue's lock
    for (uint64_t i = 0; i < k; ++i) {
        const uint64_t lo = i * kCopyPiece, n = std::min(kCopyPiece, len - lo);
        HostTask t{};
        t.kind = kind;
        t.r = r;
        t.dst = dst + lo;
        t.src = src + lo;
        t.n = n;
        t.after = after;
        t.flag = &L.fl[f];
        t.fail = &L.fl[kFlFail];
        host_task(s, t);
    }
}

uint32_t* next_ticket_slot(ckpt_server* s) {
    uint32_t* t = s->tickets.as<uint32_t>() + (s->ticket_next % 1024);
    s->ticket_next++;
    return t;
}

#define SCHK(call)                                   \
    do {                                             \
        hipError_t e_ = (call);                      \
        if (e_ != hipSuccess) { fail_req(s, r, CKPT_EHIP); return; } \
    } while (0)

// ---------------------------------------------------------------- admission
void admit_dump(ckpt_server* s, Req* r) {
    ckpt_ctx* c = s->ctx;
    Lane& L = s->lanes[r->lane];
    r->C = kDefaultChunk;
    r->n = (uint32_t)r->table.size();
    std::unordered_set<uint64_t> ids;
    for (const ckpt_alloc& e : r->table) {
        if (!ids.insert(e.id).second || (e.size && (!e.dev_ptr || (reinterpret_cast<uintptr_t>(e.dev_ptr) & 15)))) {
            finish(s, r, CKPT_EINVAL);
            return;
        }
    }
    ImageView pv;
    std::unordered_map<uint64_t, std::pair<uint64_t, uint64_t>> pm;
    if (r->rq.prev) {
        int rc = parse_image(r->rq.prev->p, r->rq.prev->n, &pv, true);   // tables digest included
        if (rc) { finish(s, r, rc); return; }
        if (pv.C != r->C) { finish(s, r, CKPT_EINVAL); return; }
        r->prev_digest = pv.state_digest;
        for (uint64_t a = 0; a < pv.n_allocs; ++a)
            pm.emplace(get64(pv.recs + 32 * a), std::make_pair(get64(pv.recs + 32 * a + 8), get64(pv.recs + 32 * a + 16)));
    }
    r->d.resize(r->n);
    uint64_t g = 0;
    for (uint32_t a = 0; a < r->n; ++a) {
        const ckpt_alloc& e = r->table[a];
        uint64_t pf = kNoChunk;
        auto it = pm.find(e.id);
        if (it != pm.end() && it->second.first == e.size) pf = it->second.second;
        make_desc(&r->d[a], e.id, e.dev_ptr, e.size, g, pf, r->C);
        const uint64_t nk = ceil_div(e.size, r->C);
        g += nk;
        r->N += e.size;
        if (nk) r->upper += (nk - 1) * r->C + round16(r->d[a].tail_len);
    }
    r->nc = g;
    r->tl = tables_len(r->n, r->nc);
    r->per = s->slot / r->C;
    r->W = ceil_div(r->nc, r->per);
    SCHK(L.descs.ensure(sizeof(AllocDesc) * std::max<uint32_t>(r->n, 1)));
    SCHK(L.arc.ensure(r->tl + 16));
    SCHK(L.kinds.ensure(r->tl + 16));
    SCHK(L.status.ensure(8 * (r->per + 64), s->s_dump));
    SCHK(L.ctl.ensure(16 * (r->W + 2) + 64));
    SCHK(L.staging.ensure(2 * s->slot));
    SCHK(L.ensure_hs(8 * (r->W + 2) + 64));
    SCHK(L.ensure_events(r->W + 1));
    // the image is allocated by a worker (pinning gigabytes takes tens of
    // milliseconds); the request's first windows may run meanwhile
    r->alloc_bytes = kHeader + r->tl + r->upper;
    {
        HostTask t{};
        t.kind = HostTask::kAlloc;
        t.r = r;
        t.n = r->alloc_bytes;
        t.flag = &L.fl[kFlAlloc];
        t.value = 1;
        host_task(s, t);
    }
    if (r->rq.prev && pv.n_chunks) {
        // pinned: later windows of this request read it while other requests
        // complete and insert their own tables
        r->prev_dev = digest_lookup(c, r->rq.prev->uid, pv.n_chunks, true);
        if (r->prev_dev) r->prev_pinned = r->rq.prev->uid;
        if (!r->prev_dev) {
            SCHK(L.prevcrc.ensure(4 * pv.n_chunks));
            SCHK(hipMemcpyAsync(L.prevcrc.p, pv.crcs, 4 * pv.n_chunks, hipMemcpyHostToDevice, s->s_dump));
            r->prev_dev = L.prevcrc.as<uint32_t>();
        }
    }
    SCHK(L.amap.ensure(4 * std::max<uint64_t>(r->nc, 1)));
    SCHK(hipMemcpyAsync(L.descs.p, r->d.data(), sizeof(AllocDesc) * r->n, hipMemcpyHostToDevice, s->s_dump));
    SCHK(launch_chunk_map(L.descs.as<AllocDesc>(), r->n, r->C, L.amap.as<uint32_t>(), s->s_dump));
    SCHK(launch_fill32(L.ctl.as<uint32_t>(), 0, (16 * (r->W + 2) + 64) / 4, s->s_dump));
    SCHK(launch_fill32(L.kinds.as<uint32_t>(), 0, ceil_div(r->tl - 32ull * r->n - 4 * r->nc, 4), s->s_dump));
    r->phase = kAlloc;
}

void admit_restore(ckpt_server* s, Req* r) {
    ckpt_ctx* c = s->ctx;
    Lane& L = s->lanes[r->lane];
    int rc = parse_image(r->rq.img->p, r->rq.img->n, &r->v, false);
    if (rc) { finish(s, r, rc); return; }
    // the served loop restores the plain layout; codec images go through ckpt_restore
    if (r->v.flags & kFlagCodec) { finish(s, r, CKPT_EINVAL); return; }
    const ImageView& v = r->v;
    r->C = v.C;
    r->n = (uint32_t)r->table.size();
    r->nc = v.n_chunks;
    r->tl = v.tl;
    r->N = v.N;
    for (uint32_t a = 0; a < r->n && a < v.n_allocs; ++a) {
        const ckpt_alloc& e = r->table[a];
        if (e.size && (!e.dev_ptr || (reinterpret_cast<uintptr_t>(e.dev_ptr) & 15))) { finish(s, r, CKPT_EINVAL); return; }
    }
    r->d.resize(v.n_allocs);
    for (uint64_t a = 0; a < v.n_allocs; ++a) {
        const uint8_t* rec = v.recs + 32 * a;
        make_desc(&r->d[a], get64(rec), a < r->n ? r->table[a].dev_ptr : nullptr, get64(rec + 8), get64(rec + 16),
                  kNoChunk, r->C);
    }
    r->per = std::max<uint64_t>(1, s->slot / r->C);
    r->W = ceil_div(std::max<uint64_t>(r->nc, 1), r->per);
    const uint64_t len_a = 32ull * v.n_allocs + 4 * v.n_chunks, len_b = v.tl - len_a;
    SCHK(L.descs.ensure(sizeof(AllocDesc) * std::max<uint64_t>(v.n_allocs, 1)));
    SCHK(L.arc.ensure(v.tl + 16));
    SCHK(L.kinds.ensure(v.tl + 16));
    SCHK(L.off.ensure(8 * std::max<uint64_t>(v.n_chunks, 1)));
    SCHK(L.wb.ensure(8 * (r->W + 2)));
    SCHK(L.status.ensure(8 * (ceil_div(v.n_chunks, 256) + 64), s->s_rest));
    // ctl: [0] offsets ticket | [8] counts[4] | [40] bad | [48] bad2 | [56] err | [64..] window tickets
    SCHK(L.ctl.ensure(64 + 4 * (r->W + 4)));
    SCHK(L.staging.ensure(2 * s->slot));
    SCHK(L.ensure_hs(128 + 8 * (r->W + 2)));
    SCHK(L.ensure_events(r->W + 1));
    uint8_t* ctl = L.ctl.as<uint8_t>();
    hipStream_t st = s->s_rest;
    SCHK(L.amap.ensure(4 * std::max<uint64_t>(v.n_chunks, 1)));
    SCHK(hipMemcpyAsync(L.descs.p, r->d.data(), sizeof(AllocDesc) * r->d.size(), hipMemcpyHostToDevice, st));
    SCHK(launch_chunk_map(L.descs.as<AllocDesc>(), (uint32_t)r->d.size(), r->C, L.amap.as<uint32_t>(), st));
    r->pinned = r->rq.img->pinned;
    if (r->pinned) {
        SCHK(hipMemcpyAsync(L.arc.p, v.recs, len_a, hipMemcpyHostToDevice, st));
        SCHK(hipMemcpyAsync(L.kinds.p, v.kinds, len_b, hipMemcpyHostToDevice, st));
    } else {
        // tables of a pageable image: host copy into the lane's pinned bounce
        // buffer (the previous request's uploads from it are done: the lane
        // was free), then an asynchronous upload
        SCHK(L.ensure_ht(v.tl));
        memcpy(L.ht, v.recs, v.tl);
        SCHK(hipMemcpyAsync(L.arc.p, L.ht, len_a, hipMemcpyHostToDevice, st));
        SCHK(hipMemcpyAsync(L.kinds.p, L.ht + len_a, len_b, hipMemcpyHostToDevice, st));
    }
    SCHK(launch_fill32(reinterpret_cast<uint32_t*>(ctl), 0, (64 + 4 * (r->W + 4)) / 4, st));
    SCHK(launch_fill64(reinterpret_cast<uint64_t*>(ctl + 40), ~0ull, 2, st));
    DigestPlan dp;
    SCHK(digest_prepare(c, &L.dig, L.arc.as<uint8_t>(), len_a, L.kinds.as<uint8_t>(), len_b, &dp, st));
    SCHK(digest_enqueue(c, dp, reinterpret_cast<uint32_t*>(L.hs), st));
    if (v.n_chunks) {
        uint32_t ep;
        SCHK(L.status.next(st, &ep));
        OffJob oj;
        memset(&oj, 0, sizeof(oj));
        oj.allocs = L.descs.as<AllocDesc>();
        oj.n_allocs = v.n_allocs;
        oj.C = r->C;
        oj.amap = L.amap.as<uint32_t>();
        oj.n_chunks = v.n_chunks;
        oj.kind = L.kinds.as<uint8_t>();
        oj.off = L.off.as<uint64_t>();
        oj.per_window = r->per;
        oj.wb = L.wb.as<uint64_t>();
        oj.n_windows = r->W;
        oj.status = L.status.words();
        oj.ticket = reinterpret_cast<uint32_t*>(ctl);
        oj.counts = reinterpret_cast<unsigned long long*>(ctl + 8);
        oj.err = reinterpret_cast<uint32_t*>(ctl + 56);
        oj.epoch = ep;
        SCHK(launch_offsets(oj, (int)std::min<uint64_t>(ceil_div(v.n_chunks, 256), 8ull * c->num_cu), st));
        SCHK(hipMemcpyAsync(L.hs + 128, L.wb.p, 8 * (r->W + 1), hipMemcpyDeviceToHost, st));
    }
    SCHK(hipMemcpyAsync(L.hs + 16, ctl + 8, 32, hipMemcpyDeviceToHost, st));
    SCHK(hipEventRecord(L.fin, st));
    r->phase = kValidate;
}

// ---------------------------------------------------------------- restore checks
void restore_validated(ckpt_server* s, Req* r) {
    ckpt_ctx* c = s->ctx;
    Lane& L = s->lanes[r->lane];
    const ImageView& v = r->v;
    const uint32_t* dig = reinterpret_cast<const uint32_t*>(L.hs);
    const uint64_t* cnt = reinterpret_cast<const uint64_t*>(L.hs + 16);
    const uint64_t len_a = 32ull * v.n_allocs + 4 * v.n_chunks, len_b = v.tl - len_a;
    if (crc_combine(dig[0], dig[1], len_b) != v.tables_crc) { fail_req(s, r, CKPT_ECORRUPT); return; }
    const uint64_t nz = cnt[0], nd = cnt[1], nu = cnt[2], ninv = cnt[3];
    if (ninv || (nu && !(v.flags & 1u)) || nz + nd + nu != v.n_chunks) { fail_req(s, r, CKPT_ECORRUPT); return; }
    const uint64_t* wb = reinterpret_cast<const uint64_t*>(L.hs + 128);
    if ((v.n_chunks ? wb[r->W] : 0) != v.D) { fail_req(s, r, CKPT_ECORRUPT); return; }
    if (v.n_allocs != r->n) { fail_req(s, r, CKPT_EMISMATCH); return; }
    for (uint32_t a = 0; a < r->n; ++a)
        if (r->table[a].id != r->d[a].id || r->table[a].size != r->d[a].size) { fail_req(s, r, CKPT_EMISMATCH); return; }
    r->nu = nu;
    if (nu) {
        int T, K;
        pick_tile(r->C, 0, &T, &K);
        const EngineConsts* ec;
        SCHK(get_consts(c, T, r->C, &ec));
        uint8_t* ctl = L.ctl.as<uint8_t>();
        ChunkJob j;
        memset(&j, 0, sizeof(j));
        j.allocs = L.descs.as<AllocDesc>();
        j.n_allocs = r->n;
        j.C = r->C;
        j.amap = L.amap.as<uint32_t>();
        j.g0 = 0;
        j.g1 = r->nc;
        j.ec = ec;
        j.kind_in = L.kinds.as<uint8_t>();
        j.ref_crc = reinterpret_cast<const uint32_t*>(L.arc.as<uint8_t>() + 32ull * r->n);
        j.bad = reinterpret_cast<unsigned long long*>(ctl + 40);
        j.err = reinterpret_cast<uint32_t*>(ctl + 56);
        int grid;
        SCHK(grid_for(c, T, K, kModeVerify, r->nc, &grid));
        uint32_t* tk = next_ticket_slot(s);
        SCHK(launch_fill32(tk, 0, 1, s->s_rest));
        SCHK(launch_chunks(T, K, kModeVerify, one_job(j, tk), grid, s->s_rest));
        SCHK(hipMemcpyAsync(L.hs + 64, ctl + 40, 8, hipMemcpyDeviceToHost, s->s_rest));
        SCHK(hipEventRecord(L.fin, s->s_rest));
        r->phase = kVerify;
        return;
    }
    r->phase = kRun;
}

// ---------------------------------------------------------------- merged launches
// One launch per mode over the next ready window of every active request.
void launch_merged(ckpt_server* s, bool dump) {
    ckpt_ctx* c = s->ctx;
    std::vector<Req*> batch;
    for (Req* r : s->active) {
        // a dump's windows may run while its image is being allocated
        if ((r->phase != kRun && !(dump && r->phase == kAlloc)) || (r->rq.kind == CKPT_REQ_DUMP) != dump ||
            r->launched >= r->W)
            continue;
        Lane& L = s->lanes[r->lane];
        const uint64_t w = r->launched;
        if (dump) {
            // at most two windows in flight: slot w%2 must have been copied out
            if (w >= 2 && (r->copied < w - 1 || !down_done(r, L, w - 2))) continue;
        } else {
            if (r->staged <= w) continue;   // payload not up yet
            if (r->pinned ? hipEventQuery(L.ev[w]) != hipSuccess : !up_done(L, w)) continue;
        }
        if (r->nc == 0) { r->launched = r->W; continue; }
        batch.push_back(r);
        if (batch.size() == (size_t)kMaxJobs) break;
    }
    if (batch.empty()) return;
    // group by chunk size: the first request's chunk size goes now
    const uint32_t C = batch[0]->C;
    int T, K;
    pick_tile(C, 0, &T, &K);
    const EngineConsts* ec;
    if (get_consts(c, T, C, &ec) != hipSuccess) return;
    hipStream_t st = dump ? s->s_dump : s->s_rest;
    JobList jl;
    memset(&jl, 0, sizeof(jl));
    std::vector<Req*> used;
    uint64_t total = 0;
    for (Req* r : batch) {
        if (r->C != C) continue;
        Lane& L = s->lanes[r->lane];
        const uint64_t w = r->launched;
        ChunkJob& j = jl.job[jl.n_jobs];
        memset(&j, 0, sizeof(j));
        j.allocs = L.descs.as<AllocDesc>();
        j.n_allocs = r->n;
        j.C = C;
        j.amap = L.amap.as<uint32_t>();
        j.g0 = w * r->per;
        j.g1 = std::min(r->nc, (w + 1) * r->per);
        j.ec = ec;
        uint8_t* slotp = L.staging.as<uint8_t>() + (w % 2) * s->slot;
        j.slot = slotp;
        if (dump) {
            if (L.status.next(st, &j.epoch) != hipSuccess) {
                // a request whose launch cannot be prepared fails alone
                fail_req(s, r, CKPT_EHIP);
                continue;
            }
            j.crc_out = reinterpret_cast<uint32_t*>(L.arc.as<uint8_t>() + 32ull * r->n);
            j.kind_out = L.kinds.as<uint8_t>();
            j.prev_crc = r->prev_dev;
            j.status = L.status.words();
            j.wtotal = reinterpret_cast<uint64_t*>(L.ctl.as<uint8_t>()) + w;
            j.err = reinterpret_cast<uint32_t*>(L.ctl.as<uint8_t>() + 16 * (r->W + 2));
            // the slot's previous copy must be finished before it is overwritten
            // (a pageable image's copy is: its flag was seen above)
            if (w >= 2 && r->pinned) hipStreamWaitEvent(st, L.slot_ev[w % 2], 0);
        } else {
            uint8_t* ctl = L.ctl.as<uint8_t>();
            const uint64_t* wb = reinterpret_cast<const uint64_t*>(L.hs + 128);
            j.kind_in = L.kinds.as<uint8_t>();
            j.ref_crc = reinterpret_cast<const uint32_t*>(L.arc.as<uint8_t>() + 32ull * r->n);
            j.off = L.off.as<uint64_t>();
            j.slot_base = wb[w];
            j.bad = reinterpret_cast<unsigned long long*>(ctl + 40);
            j.err = reinterpret_cast<uint32_t*>(ctl + 56);
            if (r->pinned) hipStreamWaitEvent(st, L.ev[w], 0);   // payload copy of this window
        }
        jl.prefix[jl.n_jobs] = total;
        total += j.g1 - j.g0;
        jl.n_jobs++;
        used.push_back(r);
    }
    if (used.empty()) return;
    jl.prefix[jl.n_jobs] = total;
    uint32_t* tk = next_ticket_slot(s);
    jl.ticket = tk;
    int grid;
    hipError_t e = launch_fill32(tk, 0, 1, st);
    if (e == hipSuccess) e = grid_for(c, T, K, dump ? kModeDump : kModeRestore, total, &grid);
    if (e == hipSuccess) e = launch_chunks(T, K, dump ? kModeDump : kModeRestore, jl, grid, st);
    for (Req* r : used) {
        Lane& L = s->lanes[r->lane];
        const uint64_t w = r->launched;
        if (e == hipSuccess && dump)
            e = hipMemcpyAsync(L.hs + 8 * w, L.ctl.as<uint64_t>() + w, 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipEventRecord(dump ? L.ev[w] : L.slot_ev[w % 2], st);
        r->launched++;
    }
    s->launches++;
    s->max_batch = std::max<uint64_t>(s->max_batch, used.size());
    if (e != hipSuccess)
        for (Req* r : used) fail_req(s, r, CKPT_EHIP);
}

// ---------------------------------------------------------------- per-request progress
void progress_dump(ckpt_server* s, Req* r) {
    ckpt_ctx* c = s->ctx;
    Lane& L = s->lanes[r->lane];
    if (lane_failed(L)) {
        fail_req(s, r, L.fl[kFlAlloc].load(std::memory_order_acquire) == kTaskFailed ? CKPT_ENOMEM : CKPT_EHIP);
        return;
    }
    if (r->phase == kAlloc) {
        if (L.fl[kFlAlloc].load(std::memory_order_acquire) != 1) return;   // image not allocated yet
        r->pinned = r->out->pinned;
        r->phase = kRun;
    }
    // copy out finished windows, in order: pinned images by the copy engine
    // on the download stream, pageable ones by a worker
    while (r->copied < r->launched && hipEventQuery(L.ev[r->copied]) == hipSuccess) {
        const uint64_t w = r->copied;
        const uint64_t dw = reinterpret_cast<const uint64_t*>(L.hs)[w];
        if (dw > s->slot || r->pos + dw > r->upper) { fail_req(s, r, CKPT_EHIP); return; }
        uint8_t* dst = r->out->p + kHeader + r->tl + r->pos;
        const uint8_t* src = L.staging.as<uint8_t>() + (w % 2) * s->slot;
        if (r->pinned) {
            SCHK(hipStreamWaitEvent(s->s_down, L.ev[w], 0));
            if (dw) SCHK(hipMemcpyAsync(dst, src, dw, hipMemcpyDeviceToHost, s->s_down));
            SCHK(hipEventRecord(L.slot_ev[w % 2], s->s_down));
        } else {
            // the window's kernel is done (its event was seen above)
            host_copy(s, r, L, kFlDown0 + (int)(w % 2), w, HostTask::kD2H, dst, src, dw, nullptr);
        }
        r->pos += dw;
        r->copied++;
    }
    if (r->phase == kRun && r->copied == r->W) {
        // tables: per-allocation CRCs, digests, copy-out
        int T, K;
        pick_tile(r->C, 0, &T, &K);
        const EngineConsts* ec;
        SCHK(get_consts(c, T, r->C, &ec));
        uint32_t* crc_dev = reinterpret_cast<uint32_t*>(L.arc.as<uint8_t>() + 32ull * r->n);
        CombineJob cj;
        memset(&cj, 0, sizeof(cj));
        cj.allocs = L.descs.as<AllocDesc>();
        cj.n_allocs = r->n;
        cj.C = r->C;
        cj.crc = crc_dev;
        cj.ec = ec;
        cj.recs = L.arc.as<uint8_t>();
        cj.mode = kCombineWrite;
        SCHK(launch_combine(cj, s->s_dump));
        const uint64_t len_a = 32ull * r->n + 4 * r->nc, len_b = r->tl - len_a;
        uint32_t* hdig = reinterpret_cast<uint32_t*>(L.hs + 8 * (r->W + 1));
        DigestPlan dp;
        SCHK(digest_prepare(c, &L.dig, L.arc.as<uint8_t>(), len_a, L.kinds.as<uint8_t>(), len_b, &dp, s->s_dump));
        SCHK(digest_enqueue(c, dp, hdig, s->s_dump));
        // tables: straight into a pinned image, through the lane's pinned
        // bounce buffer for a pageable one (moved on the host at the end)
        uint8_t* tdst = r->out->p + kHeader;
        if (!r->pinned) {
            SCHK(L.ensure_ht(r->tl));
            tdst = L.ht;
        }
        SCHK(hipMemcpyAsync(tdst, L.arc.p, len_a, hipMemcpyDeviceToHost, s->s_dump));
        SCHK(hipMemcpyAsync(tdst + len_a, L.kinds.p, len_b, hipMemcpyDeviceToHost, s->s_dump));
        SCHK(hipMemcpyAsync(hdig + 2, L.ctl.as<uint8_t>() + 16 * (r->W + 2), 4, hipMemcpyDeviceToHost, s->s_dump));
        digest_insert(c, r->out->uid, crc_dev, r->nc, s->s_dump);
        SCHK(hipEventRecord(L.fin, s->s_dump));
        r->phase = kFinal;
        return;
    }
    if (r->phase == kFinal && hipEventQuery(L.fin) == hipSuccess) {
        if (r->W && !down_done(r, L, r->W - 1)) return;
        if (r->W > 1 && !down_done(r, L, r->W - 2)) return;
        if (r->tasks.load(std::memory_order_acquire) != 0) return;
        const uint32_t* hdig = reinterpret_cast<const uint32_t*>(L.hs + 8 * (r->W + 1));
        if (hdig[2]) { fail_req(s, r, CKPT_EHIP); return; }
        const uint64_t len_a = 32ull * r->n + 4 * r->nc, len_b = r->tl - len_a;
        uint8_t* h = r->out->p;
        if (!r->pinned) memcpy(h + kHeader, L.ht, r->tl);
        memcpy(h, "MICKPT01", 8);
        put32(h + 8, 1);
        put32(h + 12, r->rq.prev ? 1u : 0u);
        put32(h + 16, r->C);
        put32(h + 20, r->n);
        put64(h + 24, r->nc);
        put64(h + 32, r->pos);
        put32(h + 40, r->rq.prev ? r->prev_digest : 0u);
        put32(h + 44, 0);
        put64(h + 48, r->N);
        put32(h + 56, crc_combine(hdig[0], hdig[1], len_b));
        put32(h + 60, host_crc32c(h, 60));
        r->out->n = kHeader + r->tl + r->pos;
        finish(s, r, CKPT_OK);
    }
}

void progress_restore(ckpt_server* s, Req* r) {
    ckpt_ctx* c = s->ctx;
    Lane& L = s->lanes[r->lane];
    if (r->phase == kValidate) {
        if (hipEventQuery(L.fin) != hipSuccess) return;
        restore_validated(s, r);
        return;
    }
    if (r->phase == kVerify) {
        if (hipEventQuery(L.fin) != hipSuccess) return;
        const uint64_t bad = *reinterpret_cast<const uint64_t*>(L.hs + 64);
        if (bad != kNoChunk) { fail_req(s, r, CKPT_EBASE); return; }
        r->phase = kRun;
        return;
    }
    if (r->phase == kRun) {
        if (lane_failed(L)) { fail_req(s, r, CKPT_EHIP); return; }
        // stage payload windows ahead of the kernels: two slots; a pinned
        // image by the copy engine on the upload stream, a pageable one by a
        // worker (which first waits for the kernel that last read the slot)
        const uint64_t* wb = reinterpret_cast<const uint64_t*>(L.hs + 128);
        while (r->staged < r->W && r->staged < r->launched + 2) {
            const uint64_t w = r->staged;
            if (w >= 2 && r->launched < w - 1) break;
            const uint64_t len = r->nc ? wb[w + 1] - wb[w] : 0;
            if (len > s->slot) { fail_req(s, r, CKPT_ECORRUPT); return; }
            uint8_t* dst = L.staging.as<uint8_t>() + (w % 2) * s->slot;
            if (r->pinned) {
                if (w >= 2) SCHK(hipStreamWaitEvent(s->s_up, L.slot_ev[w % 2], 0));   // kernel of window w-2 done
                if (len) SCHK(hipMemcpyAsync(dst, r->v.payload + wb[w], len, hipMemcpyHostToDevice, s->s_up));
                SCHK(hipEventRecord(L.ev[w], s->s_up));
            } else {
                // slot_ev[w % 2] was recorded with window w-2's kernel and is
                // recorded again only with window w's, after this copy
                host_copy(s, r, L, kFlUp0 + (int)(w % 2), w, HostTask::kH2D, dst, r->v.payload + wb[w], len,
                          w >= 2 ? L.slot_ev[w % 2] : nullptr);
            }
            r->staged++;
        }
        if (r->launched == r->W) {
            int T, K;
            pick_tile(r->C, 0, &T, &K);
            const EngineConsts* ec;
            SCHK(get_consts(c, T, r->C, &ec));
            uint8_t* ctl = L.ctl.as<uint8_t>();
            CombineJob cj;
            memset(&cj, 0, sizeof(cj));
            cj.allocs = L.descs.as<AllocDesc>();
            cj.n_allocs = r->n;
            cj.C = r->C;
            cj.crc = reinterpret_cast<const uint32_t*>(L.arc.as<uint8_t>() + 32ull * r->n);
            cj.ec = ec;
            cj.recs = L.arc.as<uint8_t>();
            cj.bad = reinterpret_cast<unsigned long long*>(ctl + 48);
            cj.mode = kCombineCheck;
            SCHK(launch_combine(cj, s->s_rest));
            SCHK(hipMemcpyAsync(L.hs + 64, ctl + 40, 24, hipMemcpyDeviceToHost, s->s_rest));
            SCHK(hipEventRecord(L.fin, s->s_rest));
            r->phase = kFinal;
        }
        return;
    }
    if (r->phase == kFinal) {
        if (hipEventQuery(L.fin) != hipSuccess || r->tasks.load(std::memory_order_acquire) != 0) return;
        const uint64_t* q = reinterpret_cast<const uint64_t*>(L.hs + 64);
        if ((uint32_t)q[2]) { fail_req(s, r, CKPT_EHIP); return; }
        if (q[0] != kNoChunk || q[1] != kNoChunk) { fail_req(s, r, CKPT_ECORRUPT); return; }
        finish(s, r, CKPT_OK);
    }
}

void loop(ckpt_server* s) {
    hipSetDevice(s->ctx->device);
    for (;;) {
        std::vector<Req*> fresh;
        {
            std::unique_lock<std::mutex> g(s->mu);
            if (s->active.empty() && s->pending.empty())
                s->cv.wait(g, [s] { return s->stop || !s->pending.empty(); });
            if (s->stop && s->active.empty() && s->pending.empty()) return;
            // admission: arrival order, a free lane and two staging windows of budget
            const uint64_t now = now_ns();
            while (!s->pending.empty()) {
                Req* r = s->pending.front();
                if (r->rq.deadline_ns && now > r->rq.deadline_ns) {
                    s->pending.pop_front();
                    fresh.push_back(r);   // finished below as timed out
                    continue;
                }
                if (s->active.size() >= s->max_active || s->reserved + 2 * s->slot > s->budget) break;
                int lane = -1;
                for (size_t i = 0; i < s->lanes.size(); ++i)
                    if (!s->lanes[i].busy) { lane = (int)i; break; }
                if (lane < 0) break;
                s->pending.pop_front();
                s->lanes[lane].busy = true;
                // no task of the lane's previous request is left (it ended
                // only once its count was 0)
                for (int i = 0; i < kLaneFlags; ++i) s->lanes[lane].fl[i].store(0, std::memory_order_relaxed);
                for (int i = 0; i < 4; ++i) {
                    s->lanes[lane].win[i] = ~0ull;
                    s->lanes[lane].need[i] = 0;
                }
                s->reserved += 2 * s->slot;
                r->lane = lane;
                r->t_admit = now;
                s->active.push_back(r);
                fresh.push_back(r);
            }
        }
        std::lock_guard<std::mutex> cg(s->ctx->mu);
        for (Req* r : fresh) {
            if (r->lane < 0) {
                finish(s, r, CKPT_ETIMEOUT);
                std::lock_guard<std::mutex> g(s->mu);
                r->retired = true;
                continue;
            }
            if (r->rq.kind == CKPT_REQ_DUMP) admit_dump(s, r);
            else admit_restore(s, r);
        }
        for (Req* r : s->active) {
            if (r->phase == kDone) continue;
            if (r->phase == kDrain) drain_step(s, r);
            else if (r->rq.kind == CKPT_REQ_DUMP) progress_dump(s, r);
            else progress_restore(s, r);
        }
        launch_merged(s, true);
        launch_merged(s, false);
        for (Req* r : s->active) {
            if (r->phase == kDone || r->phase == kDrain) continue;
            if (r->rq.kind == CKPT_REQ_DUMP) progress_dump(s, r);
            else progress_restore(s, r);
        }
        {
            std::lock_guard<std::mutex> g(s->mu);
            for (Req* r : s->active)
                if (r->phase == kDone) r->retired = true;
            s->active.erase(std::remove_if(s->active.begin(), s->active.end(),
                                           [](Req* r) { return r->phase == kDone; }),
                            s->active.end());
        }
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

}  // namespace

extern "C" int ckpt_serve_create(ckpt_ctx* ctx, uint32_t max_active, uint64_t budget, ckpt_server** out) {
    if (!ctx || !out) return CKPT_EINVAL;
    *out = nullptr;
    if (max_active == 0 || max_active > (uint32_t)kMaxJobs) max_active = kMaxJobs;
    ckpt_server* s = new ckpt_server();
    s->ctx = ctx;
    s->max_active = max_active;
    s->budget = budget ? budget : ctx->budget;
    if (const char* env = getenv("MICKPT_SERVE_WINDOW")) s->slot = std::max<uint64_t>(strtoull(env, nullptr, 0), 1 << 20);
    s->slot = s->slot / kDefaultChunk * kDefaultChunk;
    if (s->budget < 2 * s->slot) { delete s; return CKPT_ENOMEM; }
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        ctx->digest_capacity = std::max<size_t>(ctx->digest_capacity, 128);
    }
    if (hipSetDevice(ctx->device) != hipSuccess) { delete s; return CKPT_EHIP; }
    hipStream_t* ss[] = {&s->s_dump, &s->s_rest, &s->s_up, &s->s_down};
    for (hipStream_t* p : ss)
        if (hipStreamCreateWithFlags(p, hipStreamNonBlocking) != hipSuccess) { delete s; return CKPT_EHIP; }
    if (s->tickets.ensure(4 * 1024) != hipSuccess) { delete s; return CKPT_ENOMEM; }
    s->lanes.resize(max_active);
    s->flags.reset(new std::atomic<uint64_t>[kLaneFlags * max_active]);
    for (uint32_t i = 0; i < kLaneFlags * max_active; ++i) s->flags[i].store(0);
    for (uint32_t i = 0; i < max_active; ++i) s->lanes[i].fl = &s->flags[kLaneFlags * i];
    // each lane's pinned read-back and bounce buffers, made before images
    // take the pinned memory the driver grants (they grow if a request needs more)
    for (Lane& L : s->lanes)
        if (L.ensure_hs(64 << 10) != hipSuccess || L.ensure_ht(8 << 20) != hipSuccess) {
            for (Lane& x : s->lanes) x.release();
            delete s;
            return CKPT_ENOMEM;
        }
    // host workers for copies that involve pageable images (one thread made
    // 17-27 GB/s of pageable copies, four ~48 GB/s together; on the served
    // configuration twelve workers gave p99 4.2 s against 5.6 s with eight)
    int nw = 12;
    if (const char* env = getenv("MICKPT_SERVE_HOST_THREADS")) nw = std::max(1, std::min(32, atoi(env)));
    for (int i = 0; i < nw; ++i) s->workers.emplace_back(worker, s);
    s->th = std::thread(loop, s);
    *out = s;
    return CKPT_OK;
}

extern "C" int ckpt_serve_submit(ckpt_server* s, const ckpt_request* rq, uint64_t* ticket) {
    if (!s || !rq || !ticket || !rq->table || (rq->table->n && !rq->table->v)) return CKPT_EINVAL;
    if (rq->kind != CKPT_REQ_DUMP && rq->kind != CKPT_REQ_RESTORE) return CKPT_EINVAL;
    if (rq->kind == CKPT_REQ_RESTORE && !rq->img) return CKPT_EINVAL;
    Req* r = new Req();
    r->rq = *rq;
    r->table.assign(rq->table->v, rq->table->v + rq->table->n);
    r->t_submit = now_ns();
    {
        std::lock_guard<std::mutex> g(s->mu);
        r->ticket = s->next_ticket++;
        s->reqs[r->ticket] = r;
        s->pending.push_back(r);
        s->submitted++;
        s->in_system++;
        *ticket = r->ticket;
    }
    s->cv.notify_one();
    return CKPT_OK;
}

extern "C" int ckpt_serve_poll(ckpt_server* s, uint64_t ticket, int* rc, ckpt_image** out, uint64_t* latency_ns) {
    if (!s) return CKPT_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return CKPT_EINVAL;
    Req* r = it->second;
    if (r->phase != kDone || !r->retired) return 0;
    if (rc) *rc = r->rc;
    if (out) *out = r->out;
    else if (r->out) ckpt_image_free(r->out);
    if (latency_ns) *latency_ns = r->t_done - r->t_submit;
    s->reqs.erase(it);
    delete r;
    return 1;
}

extern "C" int ckpt_serve_drain(ckpt_server* s) {
    if (!s) return CKPT_EINVAL;
    std::unique_lock<std::mutex> g(s->mu);
    s->done_cv.wait(g, [s] { return s->in_system == 0; });
    return CKPT_OK;
}

extern "C" int ckpt_serve_stats(ckpt_server* s, ckpt_server_stats* st) {
    if (!s || !st) return CKPT_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    memset(st, 0, sizeof(*st));
    st->submitted = s->submitted;
    st->completed = s->completed;
    st->failed = s->failed;
    st->bytes_logical = s->bytes_logical;
    st->bytes_link = s->bytes_link;
    st->launches = s->launches;
    st->max_batch = s->max_batch;
    if (!s->lat.empty()) {
        std::vector<uint64_t> l = s->lat;
        std::sort(l.begin(), l.end());
        auto q = [&l](double p) { return l[std::min(l.size() - 1, (size_t)(p * (l.size() - 1) + 0.5))]; };
        st->p50_ns = q(0.50);
        st->p99_ns = q(0.99);
        st->mean_wait_ns = s->wait_sum / s->lat.size();
    }
    st->max_wait_ns = s->max_wait;
    st->host_copies = s->host_copies.load();
    st->host_copy_bytes = s->host_copy_bytes.load();
    return CKPT_OK;
}

extern "C" void ckpt_serve_destroy(ckpt_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->th.joinable()) s->th.join();
    {
        std::lock_guard<std::mutex> g(s->tmu);
        s->tstop = true;
    }
    s->tcv.notify_all();
    for (std::thread& t : s->workers) t.join();
    hipStream_t ss[] = {s->s_dump, s->s_rest, s->s_up, s->s_down};
    for (hipStream_t x : ss)
        if (x) { hipStreamSynchronize(x); hipStreamDestroy(x); }
    for (Lane& L : s->lanes) L.release();
    s->tickets.release();
    for (auto& kv : s->reqs) {
        if (kv.second->out) ckpt_image_free(kv.second->out);
        delete kv.second;
    }
    delete s;
}
