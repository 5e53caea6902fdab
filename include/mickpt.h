/*
 * mickpt.h -- C ABI of the MI355X checkpoint-image engine (libmickpt.so).
 *
 * The library turns a process's set of device allocations into a verified,
 * restorable memory image in host memory (pinned while the driver grants
 * pinned memory, pageable beyond that), and writes such an image
 * back byte for byte. It follows the problem statement of transparent GPU
 * checkpointing (CRIUgpu, arXiv 2502.16631):
 *   - section 3.1.1: the checkpoint action copies the GPU state (device
 *     memory) into host memory; the restore action puts device memory back;
 *   - section 3.1.2: a buffer record carries handle, size, virtual address
 *     and memory contents; a restore needs a compatible target;
 *   - section 3.1: operations are dump, pre-dump (incremental) and restore,
 *     and the exit callback reports success so that a failed operation can
 *     be cleaned up (hence: no partial outputs);
 *   - section 6: restores are deterministic (hence: 0-byte tolerance);
 *   - section 7: incremental / differential checkpointing.
 * The image format (v1), the CRC-32C chunk digests and the chunk grid are
 * this library's definition; the paper specifies none of them.
 *
 * Plain C: only fixed-width integers and pointers. Device pointers are HIP
 * device addresses; a stream is a hipStream_t passed as void* (NULL = the
 * null stream). All functions are synchronous: they return when the result
 * is complete on the host (dump) or the allocations are written and
 * verified (restore).
 */
#ifndef MICKPT_H
#define MICKPT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ errors */
#define CKPT_OK         0
#define CKPT_EINVAL    -1  /* bad argument: NULL, chunk size not a power of two in [16, 2^30],
                              duplicate ids, misaligned device pointer, unknown flag          */
#define CKPT_ENOMEM    -2  /* device staging, host image or descriptor allocation failed, or
                              the request does not fit the staging budget                     */
#define CKPT_EHIP      -3  /* a HIP call failed (ckpt_result.hip_error holds its code) or a
                              kernel reported an internal error                               */
#define CKPT_ECORRUPT  -4  /* image header / tables digest mismatch, inconsistent tables,
                              or a restored chunk / allocation failed verification
                              (ckpt_result.first_bad_chunk = lowest failing chunk)             */
#define CKPT_EMISMATCH -5  /* allocation table differs from the image: count, id or size
                              (the compatibility requirement of section 3.1.2)                */
#define CKPT_EBASE     -6  /* delta without its base: restore target does not hold the base
                              state (first_bad_chunk set), or merge with the wrong base       */
#define CKPT_ETIMEOUT  -7  /* serving: request deadline passed before completion            */
#define CKPT_EIO       -8  /* a file could not be opened, written, synced or read            */
#define CKPT_ELIMIT    -9  /* a dump into fixed buffers: the table, its previous image or the
                              chunk size exceeds what the buffers hold (nothing done)         */

/* chunk kinds stored in an image */
#define CKPT_KIND_ZERO      0
#define CKPT_KIND_DATA      1
#define CKPT_KIND_UNCHANGED 2

/* ------------------------------------------------------------------ types */
/* One device buffer (section 3.1.2 buffer record: handle, address, size).
 * dev_ptr must be 16-byte aligned (hipMalloc and torch allocations are);
 * size may be 0. id is the caller's stable handle and must be unique in a
 * table. */
typedef struct {
    uint64_t id;
    void*    dev_ptr;
    uint64_t size;
} ckpt_alloc;

/* Caller-owned table; entries are kept in this order in the image. */
typedef struct {
    const ckpt_alloc* v;
    uint32_t n;
} ckpt_alloc_table;

typedef struct ckpt_ctx ckpt_ctx;       /* device context: staging, streams, digest cache */
typedef struct ckpt_image ckpt_image;   /* an image in host memory (pinned if available)  */

/* Tuning knobs. None of them changes the bytes of an image except
 * chunk_size, which is recorded in its header, and CKPT_OPT_CODEC. Pass NULL
 * for defaults. */
#define CKPT_OPT_PER_ALLOC  1u   /* launch the kernels once per allocation (baseline form)   */
#define CKPT_OPT_GRAPH      2u   /* batched form: capture the device stage in a hipGraph and
                                    replay it (cached per table shape)                      */
#define CKPT_OPT_NO_TIMING  4u   /* skip per-stage device timing events                      */
/* Dump only (ignored by restore, where the image says how it is stored):
 * store each full-length DATA chunk as a byte-plane record when that record
 * is shorter (kind PACKED = 3; the image gets header flag bit 1 and a u32
 * record-length table between the digest and kind tables). The paper names
 * data compression as a way to speed up checkpoint and restore of large
 * models (section 5.2) and among the optimisations its method can take on
 * (section 7); the codec is this library's: 8 byte planes per chunk, each
 * stored as one value, as 4-bit codes into a 15-entry dictionary of its most
 * frequent bytes plus escaped bytes, or raw. It needs 4096 <= chunk_size <=
 * 65536 and no CKPT_OPT_PER_ALLOC or CKPT_OPT_GRAPH (CKPT_EINVAL
 * otherwise). Restoring PACKED records needs the same chunk sizes
 * (CKPT_EINVAL otherwise). */
#define CKPT_OPT_CODEC      8u
typedef struct {
    uint32_t chunk_size;     /* bytes per chunk; 0 = 65536                                   */
    uint32_t wg_threads;     /* work-group size of the chunk kernels; 0 = chosen per size   */
    uint32_t copy_streams;   /* side streams for host-link copies; 0 = 2                     */
    uint32_t slots;          /* staging ring slots; 0 = chosen from the budget              */
    uint64_t window_bytes;   /* staging slot size; 0 = chosen from the budget               */
    uint32_t flags;          /* CKPT_OPT_*                                                  */
    uint32_t strict_verify;  /* restore: 1 = after the writes, re-read every restored chunk
                                from HBM and check its CRC-32C again (the default check runs
                                on the data in registers as it is written; section 6 asks
                                for deterministic restores); 0 = off; other values:
                                CKPT_EINVAL. dump: ignored                                   */
} ckpt_opts;

/* Optional per-call report. */
typedef struct {
    uint64_t first_bad_chunk;   /* UINT64_MAX if none                                       */
    int32_t  hip_error;         /* first failing hipError_t, 0 if none                      */
    uint32_t windows;           /* staging windows used (a plain restore of >= 512 MiB held  */
                                /* by one window is launched as two parts and reports 2)    */
    uint64_t n_logical;         /* N: sum of allocation sizes                               */
    uint64_t n_payload;         /* D: payload bytes                                         */
    uint64_t n_chunks;
    uint64_t n_zero, n_data, n_unchanged;
    uint64_t link_bytes;        /* bytes moved over the host link                           */
    uint64_t ns_total;          /* wall time of the call                                    */
    uint64_t ns_kernel;         /* summed device time of the chunk kernels                  */
    uint64_t ns_link;           /* wall time from first to last host-link copy              */
    uint64_t n_packed;          /* PACKED chunks (codec records; not counted in n_data)     */
    uint64_t reserved[3];
    /* Time per stage in ns (section 5.1 measures checkpoint and restore by the
     * time spent in each of their stages). 0 when a stage did not run or, for
     * device stages, with CKPT_OPT_NO_TIMING;
     * device stages are HIP-event times on the stream they run on, link and host
     * stages wall times).
     * dump:    [0] set-up (descriptors, chunk map, table clears)  [1] chunk kernels
     *          on the main stream (single pass: the whole dump kernel, which also
     *          scans and gathers; delta in one window: digest + kind pass; codec:
     *          digest + kind and size passes)  [2] offsets scan (delta in one
     *          window)  [3] gather (delta in one window) or gather + encode
     *          (codec)  [4] host link: first to last payload copy, wall time
     *          [5] finalize (per-allocation combine, table digests, tables copied
     *          out)  [6] unused  [7] whole call, wall time;
     * restore: [0] validate (tables up, digest, offsets scan, host checks), wall
     *          time  [1] base check of a delta (a plain full restore runs it on
     *          the device beside the upload: its HIP-event time; otherwise the
     *          host waits for it: wall time)  [2] host link: first to
     *          last payload copy, wall time  [3] scatter + fused verify kernels
     *          (codec decode included)  [4] strict re-read  [5] finalize
     *          (per-allocation check)  [6] unused  [7] whole call, wall time. */
    uint64_t ns_stage[8];
} ckpt_result;

/* ------------------------------------------------------------------ context */
/* The paper defines no such call: a context is this library's holder of the
 * device resources its calls share. Its nearest counterpart in the paper is
 * the plugin's initialization callback (section 3.1), which runs once before
 * the operations. Create a context on HIP device `device`. staging_budget =
 * bytes of device memory the context may use for staging windows (0 = 4 GiB).
 * Set-up made here once: the streams, events and pinned scratch the calls
 * use.
 * Returns CKPT_OK and *out, or an error (CKPT_EINVAL for a device that does
 * not exist, CKPT_EHIP / CKPT_ENOMEM when the set-up fails) and *out = NULL. */
int  ckpt_ctx_create(int device, uint64_t staging_budget, ckpt_ctx** out);
/* Free a context and everything it owns except images (the counterpart of
 * the plugin's exit callback, section 3.1). NULL is a no-op. */
void ckpt_ctx_destroy(ckpt_ctx* ctx);

/* ------------------------------------------------------------------ dump */
/* Checkpoint (section 3.1.1 checkpoint action; section 3.1 pre-dump).
 * Reads every allocation of `table` and writes a new image to *out.
 * prev = NULL: full image. prev = an earlier image: delta image; a chunk
 * whose CRC-32C equals the same chunk's digest in prev (allocation with the
 * same id and size) is UNCHANGED and has no payload; all-zero chunks are
 * ZERO either way. prev is borrowed and must have the same chunk size.
 * The allocations must not be modified during the call (the caller's
 * analogue of the paper's lock action). On failure *out = NULL and no
 * allocation has been written. Work is ordered after prior work on stream. */
int  ckpt_dump(ckpt_ctx* ctx, const ckpt_alloc_table* table, const ckpt_image* prev,
               ckpt_image** out, const ckpt_opts* opts, void* stream, ckpt_result* res);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): ckpt_dump into fixed
 * buffers. The image (the same bytes ckpt_dump would return for these
 * arguments) is written to the caller's host buffer out[0, out_cap) and its
 * length to *out_len; the device work runs in one array of 128 MiB per GPU
 * that the library holds from the first context on that GPU until the
 * process ends. Nothing is allocated: no device, pinned or pageable image
 * memory, streams or events (ckpt_ctx_create made those).
 * Limits (CKPT_ELIMIT, returned before any work is queued): at most 16,384
 * allocations and 2^20 chunks in the table and in prev, and a chunk size
 * whose staging slot (about 52 MiB) holds at least one chunk; larger
 * payloads run as several windows on two slots. CKPT_OPT_PER_ALLOC,
 * CKPT_OPT_GRAPH and CKPT_OPT_CODEC are not accepted (CKPT_EINVAL). An out
 * buffer too small for the image gives CKPT_ENOMEM and *out_len = 0. The
 * call keeps nothing between calls except the array's contents: every call
 * clears what it needs at zero. Calls on one GPU are serialized within the
 * process; calls from several processes on one GPU each have their own
 * array. On failure *out_len = 0 and the contents of out are unspecified. */
int  ckpt_dump_into(ckpt_ctx* ctx, const ckpt_alloc_table* table, const ckpt_image* prev, void* out,
                    uint64_t out_cap, uint64_t* out_len, const ckpt_opts* opts, void* stream,
                    ckpt_result* res);

/* ------------------------------------------------------------------ restore */
/* Restore (section 3.1.1 restore action; section 6 deterministic restore).
 * Validates the image (header and tables digests, structure), checks that
 * `table` matches it (count, ids, sizes in order: CKPT_EMISMATCH), then
 * writes DATA chunks from the payload and zero-fills ZERO chunks,
 * verifying every written chunk and every allocation against the image's
 * digests (with opts->strict_verify also by re-reading every restored chunk
 * once all writes are done; the lowest failing chunk of either check is
 * reported). A delta image is applied in place: its UNCHANGED chunks must
 * already hold the base state, which is checked before anything is written
 * (CKPT_EBASE). After a CKPT_ECORRUPT the contents of the allocations are
 * unspecified. */
int  ckpt_restore(ckpt_ctx* ctx, const ckpt_image* img, const ckpt_alloc_table* table,
                  const ckpt_opts* opts, void* stream, ckpt_result* res);

/* On-demand restore (section 5.2 names on-demand restore among the ways to
 * cut restore time; section 7 cites on-demand checkpoint/restore of GPU
 * applications). Like ckpt_restore, but `table` lists only the allocations
 * wanted now, each matched to the image's allocation with the same id (any
 * order; sizes must match: CKPT_EMISMATCH for an unknown id or another
 * size; CKPT_EINVAL for an id listed twice). Only those allocations' payload
 * crosses the link and only their memory is written and verified; the rest
 * can follow in later calls. For a delta image the UNCHANGED chunks of the
 * listed allocations must hold the base state (CKPT_EBASE). ckpt_result
 * reports the logical and payload bytes of the listed allocations. */
int  ckpt_restore_some(ckpt_ctx* ctx, const ckpt_image* img, const ckpt_alloc_table* table,
                       const ckpt_opts* opts, void* stream, ckpt_result* res);

/* ------------------------------------------------------------------ autotuner */
/* This library's own call: the paper tunes nothing. Batched form: choose chunk size (16, 64 or 256 KiB), work-group width and
 * copy-stream count for `table` by timing trial dumps of a bounded sample of
 * it (allocations spread over the table, about sample_bytes in total; 0 =
 * 2 GB). flags are the CKPT_OPT_* flags the caller will dump with. Fills
 * *best (to pass to ckpt_dump) and, if non-NULL, *gbps with the best trial's
 * logical GB/s. Results are cached in the context per table shape (count and
 * size class of the allocations), so later calls return at once. The
 * allocations are only read. */
int  ckpt_autotune(ckpt_ctx* ctx, const ckpt_alloc_table* table, uint64_t sample_bytes, uint32_t flags,
                   ckpt_opts* best, double* gbps);

/* ------------------------------------------------------------------ host ops */
/* The image format's own calls (the paper defines no image format).
 * ckpt_merge folds a delta into the full image of its base (host memory
 * only): the result equals a full dump of the delta's state. Section 7
 * names incremental / differential checkpointing among the optimisations the
 * method can take on; merging is how a chain of such images is compacted. CKPT_EINVAL if base is a
 * delta or delta is not one, CKPT_EBASE if delta was not taken against
 * base. */
int  ckpt_merge(const ckpt_image* base, const ckpt_image* delta, ckpt_image** out);
/* Borrow the bytes of an image (valid until ckpt_image_free): the image's
 * memory stays the library's; *p and *n describe it. */
int  ckpt_image_bytes(const ckpt_image* img, const void** p, uint64_t* n);
/* Copy n bytes (the caller's, only read) into a new image owned by the
 * library after validating header, tables digest and structure
 * (CKPT_ECORRUPT if invalid; payload records are verified by a restore). */
int  ckpt_image_import(const void* p, uint64_t n, ckpt_image** out);
/* Free an image (its memory returns to the library's pinned pool). NULL is a
 * no-op. */
void ckpt_image_free(ckpt_image* img);

/* Storage. In the paper's checkpoint/restore workflow (section 3.2, its
 * second step) the AMD GPU plugin writes the captured GPU state, whose buffer
 * objects section 3.1.2 lists, out to checkpoint files; section 5.1 times
 * the write of the memory state to persistent storage, and section 5.2 finds
 * restores bounded also by how fast checkpoint data is read from disk. ckpt_image_save writes the image's bytes to `path`
 * (created or truncated) with `threads` threads (0 = 8) of positional writes,
 * O_DIRECT for the page-aligned prefix when the file system accepts it, and
 * syncs the file before returning. ckpt_image_load reads such a file into a
 * new image (pinned if available) and validates it like ckpt_image_import
 * (CKPT_ECORRUPT on a bad header or tables digest; payload records are
 * verified by the restore). Both return CKPT_EIO when the file cannot be
 * opened, written, synced or read in full. */
int  ckpt_image_save(const ckpt_image* img, const char* path, uint32_t threads);
int  ckpt_image_load(const char* path, uint32_t threads, ckpt_image** out);
/* Dump straight to a file, and restore straight from one, with the file I/O
 * overlapping the host-link copies (checkpoint files: section 3.2; their
 * write and read times: sections 5.1 and 5.2).
 * ckpt_dump_file: as ckpt_dump, and the image is written to `path` (created
 * or truncated) by `io_threads` threads (0 = 8) as the dump copies it out:
 * every 64 MiB piece of the file goes to disk as soon as all its bytes are
 * in host memory, the pieces holding the header and tables and the last one
 * once the dump is done; the file is synced before the call returns. *out
 * (may be NULL) receives the image, else it is freed. On any failure no
 * image is returned and the file is removed; CKPT_EIO when the file cannot
 * be written or synced, else the codes of ckpt_dump.
 * ckpt_restore_file: as ckpt_restore of the image in `path`: the header and
 * tables are read first and checked as in ckpt_restore, then `io_threads`
 * threads (0 = 8) load the rest in 64 MiB pieces while the restore uploads
 * each staging window once the file up to its end is loaded (without
 * opts->window_bytes, eight windows on a ring of up to three slots).
 * CKPT_EIO when the file cannot be read in full, else the codes of
 * ckpt_restore. */
int  ckpt_dump_file(ckpt_ctx* ctx, const ckpt_alloc_table* table, const ckpt_image* prev, const char* path,
                    uint32_t io_threads, const ckpt_opts* opts, void* stream, ckpt_result* res,
                    ckpt_image** out);
int  ckpt_restore_file(ckpt_ctx* ctx, const char* path, uint32_t io_threads, const ckpt_alloc_table* table,
                       const ckpt_opts* opts, void* stream, ckpt_result* res);
/* Static description of an error code (this library's own call). */
const char* ckpt_strerror(int code);
/* CRC-32C (reflected 0x82F63B78, preset and final complement) of host bytes:
 * the image format's chunk digest (this library's choice; the paper names
 * none), exposed so that callers can check images. */
uint32_t ckpt_crc32c(const void* p, uint64_t n);

/* ------------------------------------------------------------------ serving */
/* The paper defines no serving loop; section 7 relates GPU inference on
 * serverless platforms and on-demand restore of GPU workloads, where many
 * tenants' checkpoints and restores share one device. This loop is the
 * library's. A request loop over one context (served form). Dump and restore requests
 * from many tenants are admitted in arrival order as lanes and staging
 * memory free up (each admitted request holds two staging windows of the
 * budget); the next ready window of every admitted request joins one shared
 * persistent launch per tick (continuous batching), dumps and restores on
 * separate streams so their work overlaps on the device. Each request's
 * result is the same as that of the plain calls (its image is byte-identical
 * to ckpt_dump's with 64 KiB chunks). Tenants' digest tables stay resident
 * in the context for their incremental dumps. Copies between the device and
 * images in pageable host memory (beyond the pinned budget) and the
 * allocation of dump images run on host worker threads of the server, so
 * that they never hold up the other requests. */
typedef struct ckpt_server ckpt_server;
#define CKPT_REQ_DUMP     1
#define CKPT_REQ_RESTORE  2
typedef struct {
    uint32_t kind;                   /* CKPT_REQ_DUMP or CKPT_REQ_RESTORE                          */
    uint32_t tenant;                 /* caller's tenant number (informational)                   */
    const ckpt_alloc_table* table;   /* entries copied at submit; buffers borrowed until done    */
    const ckpt_image* prev;          /* dump: previous image (delta), or NULL; borrowed           */
    const ckpt_image* img;           /* restore: image to apply; borrowed until done             */
    uint64_t deadline_ns;            /* 0 = none; else CLOCK_MONOTONIC time after which a request
                                        still waiting for admission fails with CKPT_ETIMEOUT     */
} ckpt_request;
typedef struct {
    uint64_t submitted, completed, failed;
    uint64_t bytes_logical;          /* sum of N over completed requests                          */
    uint64_t bytes_link;             /* sum of image bytes moved over the host link              */
    uint64_t launches;               /* merged kernel launches                                    */
    uint64_t max_batch;              /* most requests sharing one launch                          */
    uint64_t p50_ns, p99_ns;         /* latency percentiles, submit to completion                 */
    uint64_t mean_wait_ns;           /* mean wait for admission                                   */
    uint64_t max_wait_ns;            /* longest wait for admission                                */
    uint64_t host_copies;            /* payload copies of pageable images made by host workers    */
    uint64_t host_copy_bytes;        /* their bytes                                               */
} ckpt_server_stats;
/* Create a server that drives ctx from its own thread (other calls on ctx
 * are serialized with it) with at most max_active requests in flight
 * (1..16; 0 = 16) and `budget` bytes of staging for admission (0 = the
 * context's budget; at least two 256 MiB windows). */
int  ckpt_serve_create(ckpt_ctx* ctx, uint32_t max_active, uint64_t budget, ckpt_server** out);
/* Queue a request; *ticket >= 1 identifies it. Does not wait for the GPU. */
int  ckpt_serve_submit(ckpt_server* s, const ckpt_request* rq, uint64_t* ticket);
/* 1 if the request is done (*rc = its result code; *out = the new image of a
 * dump, owned by the caller, or freed if out is NULL; *latency_ns = submit
 * to completion), 0 if pending, CKPT_EINVAL for an unknown ticket. A done
 * ticket is forgotten after it has been polled. */
int  ckpt_serve_poll(ckpt_server* s, uint64_t ticket, int* rc, ckpt_image** out, uint64_t* latency_ns);
/* Wait until every submitted request has completed. */
int  ckpt_serve_drain(ckpt_server* s);
int  ckpt_serve_stats(ckpt_server* s, ckpt_server_stats* st);
/* Finish the queued work, stop the thread, free lanes and unpolled results. */
void ckpt_serve_destroy(ckpt_server* s);

#ifdef __cplusplus
}
#endif
#endif /* MICKPT_H */
