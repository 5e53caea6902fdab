/*
 * ckpt_oracle.c -- plain CPU oracle for the checkpoint image (format v1).
 *
 * TEST INFRASTRUCTURE ONLY. Only tests/, __graft_entry__.smoke() and
 * bench.py's CPU-baseline leg may load this library. It shares no code,
 * header, table or constant with the GPU library; the two are written
 * independently from the same format definition.
 *
 * What it computes follows the paper's problem statement (section 3,
 * "Transparent GPU Checkpointing"): capture the memory contents of every
 * device buffer into host memory (3.1.1, checkpoint action; 3.1.2, buffer
 * records with handle, size and contents), restore them byte for byte
 * (3.1.1, restore action; section 6, deterministic restore) onto a target
 * with the same buffers and sizes (3.1.2, topology compatibility), and the
 * incremental form (3.1, pre-dump operation; section 7, incremental /
 * differential checkpointing). The image layout, the CRC-32C digest and the
 * chunk grid are this project's reading; the paper defines none of them
 * (parity of the layout is unpinned by the paper; see the Python spec
 * oracle's header for the field list).
 *
 * CRC-32C: reflected Castagnoli polynomial 0x82F63B78, preset and final
 * complement (the iSCSI CRC of RFC 3720). One table lookup per byte
 * (Sarwate); the 256-entry table is generated here from the polynomial by
 * the bit-serial shift register. No SIMD, no hardware CRC instruction.
 *
 * Threads: chunk digests, zero tests and whole-allocation digests are
 * computed by `threads` POSIX threads over contiguous ranges; assembling the
 * image is one sequential pass in chunk order.
 *
 * Byte-plane codec (header flag bit 1; kind PACKED): the paper names data
 * compression as a way to speed up checkpoint and restore of large models
 * (section 5.2) and compression among the optimisations its method can take
 * on (section 7), but defines no codec; this one is the project's. Layout
 * with the flag: AllocRec[] | u32 crc[] | u32 rlen[] | u8 kind[] | pad16,
 * rlen[g] = payload record length of chunk g. A full-length DATA chunk is
 * split into 8 byte planes (plane p = bytes p, p+8, ...); each plane becomes
 * CONST (one value), DICT (15-entry dictionary of its most frequent bytes,
 * 4-bit codes, escapes) or RAW; the record (48-byte head of modes and escape
 * counts, then the 16-byte-aligned sections) replaces the chunk when it is
 * strictly shorter. The Python spec oracle's header has the byte layout.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_ECORRUPT = -4,
       ORC_EMISMATCH = -5, ORC_EBASE = -6 };
enum { K_ZERO = 0, K_DATA = 1, K_UNCHANGED = 2, K_PACKED = 3 };
enum { F_DELTA = 1, F_CODEC = 2 };
enum { PM_RAW = 0, PM_CONST = 1, PM_DICT = 2 };
#define NO_CHUNK UINT64_MAX

/* ------------------------------------------------------------ CRC-32C */
static uint32_t g_table[256];
static pthread_once_t g_once = PTHREAD_ONCE_INIT;

static void make_table(void) {
    for (uint32_t b = 0; b < 256; ++b) {
        uint32_t r = b;
        for (int i = 0; i < 8; ++i) r = (r >> 1) ^ ((r & 1u) ? 0x82F63B78u : 0u);
        g_table[b] = r;
    }
}

/* Continue a CRC register (already preset) over n bytes. */
static uint32_t crc_update(uint32_t reg, const uint8_t* p, uint64_t n) {
    for (uint64_t i = 0; i < n; ++i) reg = (reg >> 8) ^ g_table[(reg ^ p[i]) & 0xFFu];
    return reg;
}

uint32_t orc_crc32c(const uint8_t* p, uint64_t n) {
    pthread_once(&g_once, make_table);
    return ~crc_update(0xFFFFFFFFu, p, n);
}

/* ------------------------------------------------------------ LE access */
static void put32(uint8_t* p, uint32_t v) { for (int i = 0; i < 4; ++i) p[i] = (uint8_t)(v >> (8 * i)); }
static void put64(uint8_t* p, uint64_t v) { for (int i = 0; i < 8; ++i) p[i] = (uint8_t)(v >> (8 * i)); }
static uint32_t get32(const uint8_t* p) { uint32_t v = 0; for (int i = 3; i >= 0; --i) v = (v << 8) | p[i]; return v; }
static uint64_t get64(const uint8_t* p) { uint64_t v = 0; for (int i = 7; i >= 0; --i) v = (v << 8) | p[i]; return v; }

static uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
static uint64_t round16(uint64_t n) { return (n + 15) & ~(uint64_t)15; }
static int valid_c(uint64_t c) { return c >= 16 && c <= (1ull << 30) && (c & (c - 1)) == 0; }
static uint64_t tables_len(uint64_t n_allocs, uint64_t n_chunks, int codec) {
    return round16(32 * n_allocs + (codec ? 9 : 5) * n_chunks);
}

/* ------------------------------------------------------------ codec */
/* Section bytes of one plane of a chunk of c bytes. */
static uint64_t sec_len(uint32_t c, int mode, uint64_t esc) {
    uint64_t lp = c / 8;
    if (mode == PM_CONST) return 16;
    if (mode == PM_DICT) return 16 + round16(lp / 2) + round16(esc);
    return round16(lp);
}

/* Encode a full chunk of c bytes into rec (capacity c). Returns the record
 * length, or 0 when the record would not be shorter than the chunk. */
static uint64_t codec_pack(const uint8_t* x, uint32_t c, uint8_t* rec) {
    const uint64_t lp = c / 8;
    int mode[8];
    uint32_t esc[8];
    uint8_t dict[8][16];
    int nused[8];
    uint64_t total = 48;
    for (int p = 0; p < 8; ++p) {
        uint64_t cnt[256];
        memset(cnt, 0, sizeof(cnt));
        for (uint64_t e = 0; e < lp; ++e) cnt[x[8 * e + p]]++;
        /* selection: repeatedly the largest count, smallest value on ties */
        memset(dict[p], 0, 16);
        uint64_t covered = 0;
        int n = 0;
        for (; n < 15; ++n) {
            int best = -1;
            for (int v = 0; v < 256; ++v)
                if (cnt[v] && (best < 0 || cnt[v] > cnt[best])) best = v;
            if (best < 0) break;
            dict[p][n] = (uint8_t)best;
            covered += cnt[best];
            if (n == 0 && cnt[best] == lp) { n = 1; cnt[best] = 0; break; }
            cnt[best] = 0;
        }
        nused[p] = n;
        if (covered == lp && n == 1) { mode[p] = PM_CONST; esc[p] = 0; }
        else {
            uint64_t e = lp - covered;
            if (sec_len(c, PM_DICT, e) < sec_len(c, PM_RAW, 0)) { mode[p] = PM_DICT; esc[p] = (uint32_t)e; }
            else { mode[p] = PM_RAW; esc[p] = 0; }
        }
        total += sec_len(c, mode[p], esc[p]);
    }
    if (total >= c) return 0;
    memset(rec, 0, total);
    for (int p = 0; p < 8; ++p) { rec[p] = (uint8_t)mode[p]; put32(rec + 8 + 4 * p, esc[p]); }
    uint64_t at = 48;
    for (int p = 0; p < 8; ++p) {
        uint8_t* s = rec + at;
        if (mode[p] == PM_CONST) {
            s[0] = x[p];
        } else if (mode[p] == PM_RAW) {
            for (uint64_t e = 0; e < lp; ++e) s[e] = x[8 * e + p];
        } else {
            memcpy(s, dict[p], 16);
            uint8_t* codes = s + 16;
            uint8_t* escs = codes + round16(lp / 2);
            uint64_t k = 0;
            for (uint64_t e = 0; e < lp; ++e) {
                uint8_t b = x[8 * e + p];
                int code = 15;
                for (int i = 0; i < nused[p]; ++i)
                    if (dict[p][i] == b) { code = i; break; }
                if (code == 15) escs[k++] = b;
                codes[e / 2] |= (uint8_t)(code << (4 * (e & 1)));
            }
        }
        at += sec_len(c, mode[p], esc[p]);
    }
    return total;
}

/* Decode a record of rlen bytes into a chunk of c bytes; 0 on success,
 * -1 when a checked rule is broken (nothing meaningful in out then). */
static int codec_unpack(const uint8_t* rec, uint64_t rlen, uint32_t c, uint8_t* out) {
    const uint64_t lp = c / 8;
    if (rlen < 48) return -1;
    for (int i = 40; i < 48; ++i)
        if (rec[i]) return -1;
    uint64_t total = 48;
    for (int p = 0; p < 8; ++p) {
        uint32_t e = get32(rec + 8 + 4 * p);
        if (rec[p] > PM_DICT || (rec[p] != PM_DICT && e != 0) || e > lp) return -1;
        total += sec_len(c, rec[p], e);
    }
    if (total != rlen) return -1;
    uint64_t at = 48;
    for (int p = 0; p < 8; ++p) {
        const uint8_t* s = rec + at;
        uint32_t e = get32(rec + 8 + 4 * p);
        if (rec[p] == PM_CONST) {
            for (uint64_t i = 0; i < lp; ++i) out[8 * i + p] = s[0];
        } else if (rec[p] == PM_RAW) {
            for (uint64_t i = 0; i < lp; ++i) out[8 * i + p] = s[i];
        } else {
            const uint8_t* codes = s + 16;
            const uint8_t* escs = codes + round16(lp / 2);
            uint64_t n15 = 0;
            for (uint64_t i = 0; i < lp; ++i) n15 += ((codes[i / 2] >> (4 * (i & 1))) & 15) == 15;
            if (n15 != e) return -1;
            uint64_t k = 0;
            for (uint64_t i = 0; i < lp; ++i) {
                int code = (codes[i / 2] >> (4 * (i & 1))) & 15;
                out[8 * i + p] = code == 15 ? escs[k++] : s[code];
            }
        }
        at += sec_len(c, rec[p], e);
    }
    return 0;
}

/* ------------------------------------------------------------ parsed image */
typedef struct {
    uint32_t flags, c, n_allocs, base_state, tables_crc, state_digest;
    uint64_t n_chunks, d, n;
    const uint8_t* recs;     /* AllocRec[n_allocs] */
    const uint8_t* crcs;     /* u32[n_chunks]      */
    const uint8_t* rlens;    /* u32[n_chunks] with the codec flag, else NULL */
    const uint8_t* kinds;    /* u8[n_chunks]       */
    const uint8_t* payload;  /* D bytes            */
} image_t;

static uint64_t rec_id(const image_t* im, uint64_t a) { return get64(im->recs + 32 * a); }
static uint64_t rec_size(const image_t* im, uint64_t a) { return get64(im->recs + 32 * a + 8); }
static uint64_t rec_first(const image_t* im, uint64_t a) { return get64(im->recs + 32 * a + 16); }
static uint32_t rec_crc(const image_t* im, uint64_t a) { return get32(im->recs + 32 * a + 24); }
static uint32_t chunk_crc(const image_t* im, uint64_t g) { return get32(im->crcs + 4 * g); }

/* payload record length of chunk g, whose real length is len */
static uint64_t rec_len(const image_t* im, uint64_t g, uint64_t len) {
    if (im->rlens) return get32(im->rlens + 4 * g);
    return im->kinds[g] == K_DATA ? round16(len) : 0;
}

/* Validate header and tables; fill *im. */
static int parse(const uint8_t* img, uint64_t len, image_t* im) {
    pthread_once(&g_once, make_table);
    if (len < 64 || memcmp(img, "MICKPT01", 8) != 0) return ORC_ECORRUPT;
    if (orc_crc32c(img, 60) != get32(img + 60)) return ORC_ECORRUPT;
    uint32_t version = get32(img + 8);
    im->flags = get32(img + 12);
    im->c = get32(img + 16);
    im->n_allocs = get32(img + 20);
    im->n_chunks = get64(img + 24);
    im->d = get64(img + 32);
    im->base_state = get32(img + 40);
    uint32_t reserved = get32(img + 44);
    im->n = get64(img + 48);
    im->tables_crc = get32(img + 56);
    if (version != 1 || (im->flags & ~(uint32_t)(F_DELTA | F_CODEC)) || reserved != 0 || !valid_c(im->c))
        return ORC_ECORRUPT;
    if (im->n_chunks > (1ull << 40) || im->n_allocs > (1u << 24)) return ORC_ECORRUPT;
    const int codec = (im->flags & F_CODEC) != 0;
    uint64_t tl = tables_len(im->n_allocs, im->n_chunks, codec);
    if (len != 64 + tl + im->d) return ORC_ECORRUPT;
    const uint8_t* tr = img + 64;
    if (orc_crc32c(tr, tl) != im->tables_crc) return ORC_ECORRUPT;
    im->recs = tr;
    im->crcs = tr + 32ull * im->n_allocs;
    im->rlens = codec ? im->crcs + 4 * im->n_chunks : NULL;
    im->kinds = im->crcs + (codec ? 8 : 4) * im->n_chunks;
    im->payload = img + 64 + tl;
    im->state_digest = orc_crc32c(tr, 32ull * im->n_allocs + 4 * im->n_chunks);
    /* structure */
    int delta = im->flags & 1u;
    uint64_t g = 0, total = 0, dsum = 0;
    for (uint64_t a = 0; a < im->n_allocs; ++a) {
        if (rec_first(im, a) != g || get32(im->recs + 32 * a + 28) != 0) return ORC_ECORRUPT;
        uint64_t size = rec_size(im, a), nk = ceil_div(size, im->c);
        if (g + nk > im->n_chunks) return ORC_ECORRUPT;
        for (uint64_t k = 0; k < nk; ++k, ++g) {
            uint8_t kd = im->kinds[g];
            if (kd > K_PACKED || (kd == K_UNCHANGED && !delta) || (kd == K_PACKED && !codec)) return ORC_ECORRUPT;
            uint64_t lo = k * im->c, hi = lo + im->c < size ? lo + im->c : size;
            uint64_t want = kd == K_DATA ? round16(hi - lo) : 0;
            if (kd == K_PACKED) {
                want = get32(im->rlens + 4 * g);
                if (hi - lo != im->c || (want & 15) || want < 48 + 8 * 16 || want >= im->c) return ORC_ECORRUPT;
            }
            if (codec && get32(im->rlens + 4 * g) != want) return ORC_ECORRUPT;
            dsum += want;
        }
        total += size;
    }
    if (g != im->n_chunks || total != im->n || dsum != im->d) return ORC_ECORRUPT;
    for (const uint8_t* p = im->kinds + im->n_chunks; p < tr + tl; ++p)
        if (*p) return ORC_ECORRUPT;
    if (!delta && im->base_state != 0) return ORC_ECORRUPT;
    return ORC_OK;
}

/* ------------------------------------------------------------ chunk grid */
typedef struct {
    uint32_t n, c;
    const uint64_t* sizes;
    const uint8_t* const* data;   /* dump: sources; restore: destinations */
    uint64_t* first;              /* first chunk of each allocation       */
    uint64_t n_chunks;
} grid_t;

static uint64_t grid_build(grid_t* gr) {
    uint64_t g = 0;
    for (uint32_t a = 0; a < gr->n; ++a) { gr->first[a] = g; g += ceil_div(gr->sizes[a], gr->c); }
    gr->n_chunks = g;
    return g;
}

/* allocation holding global chunk g: the last a with first[a] <= g (an
 * empty allocation shares first[] with its successor, so it is never last) */
static uint32_t grid_alloc_of(const grid_t* gr, uint64_t g) {
    uint32_t lo = 0, hi = gr->n;
    while (hi - lo > 1) {
        uint32_t mid = lo + (hi - lo) / 2;
        if (gr->first[mid] <= g) lo = mid; else hi = mid;
    }
    return lo;
}

/* ------------------------------------------------------------ threads */
typedef struct {
    const grid_t* gr;
    uint64_t g0, g1;          /* chunk range   */
    uint32_t a0, a1, astep;   /* alloc stripe  */
    uint32_t* crc;            /* per chunk     */
    uint8_t* zero;            /* per chunk     */
    uint32_t* alloc_crc;      /* per alloc     */
} work_t;

static void* chunk_worker(void* arg) {
    work_t* w = (work_t*)arg;
    const grid_t* gr = w->gr;
    if (w->g0 < w->g1) {
        uint32_t a = grid_alloc_of(gr, w->g0);
        for (uint64_t g = w->g0; g < w->g1; ++g) {
            while (g >= gr->first[a] + ceil_div(gr->sizes[a], gr->c)) ++a;
            uint64_t k = g - gr->first[a];
            uint64_t lo = k * gr->c, hi = lo + gr->c < gr->sizes[a] ? lo + gr->c : gr->sizes[a];
            const uint8_t* p = gr->data[a] + lo;
            w->crc[g] = orc_crc32c(p, hi - lo);
            uint8_t any = 0;
            for (uint64_t i = 0; i < hi - lo; ++i) any |= p[i];
            w->zero[g] = any == 0;
        }
    }
    if (w->alloc_crc)
        for (uint32_t a = w->a0; a < w->a1; a += w->astep)
            w->alloc_crc[a] = orc_crc32c(gr->data[a], gr->sizes[a]);
    return NULL;
}

/* crc[] and zero[] for every chunk, alloc_crc[] for every allocation */
static int run_workers(const grid_t* gr, int threads, uint32_t* crc, uint8_t* zero, uint32_t* alloc_crc) {
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    pthread_t tid[256];
    work_t w[256];
    for (int t = 0; t < threads; ++t) {
        w[t].gr = gr;
        w[t].g0 = gr->n_chunks * (uint64_t)t / (uint64_t)threads;
        w[t].g1 = gr->n_chunks * (uint64_t)(t + 1) / (uint64_t)threads;
        w[t].a0 = (uint32_t)t; w[t].a1 = gr->n; w[t].astep = (uint32_t)threads;
        w[t].crc = crc; w[t].zero = zero; w[t].alloc_crc = alloc_crc;
    }
    int spawned = 1;
    while (spawned < threads && pthread_create(&tid[spawned], NULL, chunk_worker, &w[spawned]) == 0) ++spawned;
    chunk_worker(&w[0]);
    for (int t = spawned; t < threads; ++t) chunk_worker(&w[t]);   /* could not spawn: run inline */
    for (int t = 1; t < spawned; ++t) pthread_join(tid[t], NULL);
    return ORC_OK;
}

/* ------------------------------------------------------------ public API */
/* Upper bound of the image size for a table. */
uint64_t orc_image_bound(uint32_t n, const uint64_t* sizes, uint32_t c) {
    uint64_t nc = 0, d = 0;
    for (uint32_t a = 0; a < n; ++a) { nc += ceil_div(sizes[a], c); d += round16(sizes[a]) + 16 * ceil_div(sizes[a], c); }
    return 64 + tables_len(n, nc, 1) + d;
}

static void write_header(uint8_t* out, uint32_t flags, uint32_t c, uint32_t n_allocs, uint64_t n_chunks,
                         uint64_t d, uint32_t base_state, uint64_t n_total, uint32_t tables_crc) {
    memcpy(out, "MICKPT01", 8);
    put32(out + 8, 1); put32(out + 12, flags); put32(out + 16, c); put32(out + 20, n_allocs);
    put64(out + 24, n_chunks); put64(out + 32, d); put32(out + 40, base_state); put32(out + 44, 0);
    put64(out + 48, n_total); put32(out + 56, tables_crc);
    put32(out + 60, orc_crc32c(out, 60));
}

int orc_dump(uint32_t n, const uint64_t* ids, const uint64_t* sizes, const uint8_t* const* data,
             uint32_t c, int codec, const uint8_t* prev, uint64_t prev_len, int threads,
             uint8_t* out, uint64_t out_cap, uint64_t* out_len) {
    pthread_once(&g_once, make_table);
    if (!valid_c(c)) return ORC_EINVAL;
    for (uint32_t a = 0; a < n; ++a)
        for (uint32_t b = a + 1; b < n; ++b)
            if (ids[a] == ids[b]) return ORC_EINVAL;
    image_t pv;
    int have_prev = prev != NULL;
    if (have_prev) {
        int rc = parse(prev, prev_len, &pv);
        if (rc) return rc;
        if (pv.c != c) return ORC_EINVAL;
    }
    grid_t gr = { n, c, sizes, data, (uint64_t*)malloc(sizeof(uint64_t) * (n ? n : 1)), 0 };
    if (!gr.first) return ORC_ENOMEM;
    uint64_t nc = grid_build(&gr);
    uint32_t* crc = (uint32_t*)malloc(4 * (nc ? nc : 1));
    uint8_t* zero = (uint8_t*)malloc(nc ? nc : 1);
    uint32_t* acrc = (uint32_t*)malloc(4 * (n ? n : 1));
    if (!crc || !zero || !acrc) { free(gr.first); free(crc); free(zero); free(acrc); return ORC_ENOMEM; }
    run_workers(&gr, threads, crc, zero, acrc);

    codec = codec != 0;
    uint64_t tl = tables_len(n, nc, codec);
    uint64_t need = 64 + tl;
    int rc = ORC_OK;
    if (need > out_cap) { rc = ORC_ENOMEM; goto done; }
    memset(out, 0, need);
    uint8_t* tr = out + 64;
    uint8_t* tcrc = tr + 32ull * n;
    uint8_t* trlen = codec ? tcrc + 4 * nc : NULL;
    uint8_t* tkind = tcrc + (codec ? 8 : 4) * nc;
    uint64_t pos = need;
    for (uint32_t a = 0; a < n; ++a) {
        put64(tr + 32ull * a, ids[a]); put64(tr + 32ull * a + 8, sizes[a]);
        put64(tr + 32ull * a + 16, gr.first[a]); put32(tr + 32ull * a + 24, acrc[a]);
        /* matching allocation of the previous image: same id, same size */
        int64_t pmatch = -1;
        if (have_prev)
            for (uint64_t b = 0; b < pv.n_allocs; ++b)
                if (rec_id(&pv, b) == ids[a] && rec_size(&pv, b) == sizes[a]) { pmatch = (int64_t)b; break; }
        uint64_t nk = ceil_div(sizes[a], c);
        for (uint64_t k = 0; k < nk; ++k) {
            uint64_t g = gr.first[a] + k;
            uint64_t lo = k * c, hi = lo + c < sizes[a] ? lo + c : sizes[a];
            uint8_t kind;
            if (zero[g]) kind = K_ZERO;
            else if (pmatch >= 0 && chunk_crc(&pv, rec_first(&pv, (uint64_t)pmatch) + k) == crc[g]) kind = K_UNCHANGED;
            else kind = K_DATA;
            put32(tcrc + 4 * g, crc[g]);
            uint64_t rl = 0;
            if (kind == K_DATA) {
                uint64_t len = hi - lo, l16 = round16(len);
                if (pos + l16 > out_cap) { rc = ORC_ENOMEM; goto done; }
                /* a full chunk is packed in place when its record is shorter */
                uint64_t packed = codec && len == c ? codec_pack(data[a] + lo, c, out + pos) : 0;
                if (packed) {
                    kind = K_PACKED;
                    rl = packed;
                } else {
                    memcpy(out + pos, data[a] + lo, len);
                    memset(out + pos + len, 0, l16 - len);
                    rl = l16;
                }
                pos += rl;
            }
            tkind[g] = kind;
            if (trlen) put32(trlen + 4 * g, (uint32_t)rl);
        }
    }
    uint64_t total = 0;
    for (uint32_t a = 0; a < n; ++a) total += sizes[a];
    write_header(out, (have_prev ? (uint32_t)F_DELTA : 0u) | (codec ? (uint32_t)F_CODEC : 0u), c, n, nc,
                 pos - need, have_prev ? pv.state_digest : 0u, total, orc_crc32c(tr, tl));
    *out_len = pos;
done:
    free(gr.first); free(crc); free(zero); free(acrc);
    return rc;
}

int orc_restore(const uint8_t* img, uint64_t len, uint32_t n, const uint64_t* ids, const uint64_t* sizes,
                uint8_t* const* data, int threads, uint64_t* first_bad) {
    *first_bad = NO_CHUNK;
    image_t im;
    int rc = parse(img, len, &im);
    if (rc) return rc;
    if (im.n_allocs != n) return ORC_EMISMATCH;
    for (uint32_t a = 0; a < n; ++a)
        if (rec_id(&im, a) != ids[a] || rec_size(&im, a) != sizes[a]) return ORC_EMISMATCH;
    grid_t gr = { n, im.c, sizes, (const uint8_t* const*)data, (uint64_t*)malloc(sizeof(uint64_t) * (n ? n : 1)), 0 };
    if (!gr.first) return ORC_ENOMEM;
    grid_build(&gr);
    uint64_t nc = gr.n_chunks;
    uint32_t* crc = (uint32_t*)malloc(4 * (nc ? nc : 1));
    uint8_t* zero = (uint8_t*)malloc(nc ? nc : 1);
    uint32_t* acrc = (uint32_t*)malloc(4 * (n ? n : 1));
    if (!crc || !zero || !acrc) { free(gr.first); free(crc); free(zero); free(acrc); return ORC_ENOMEM; }
    uint64_t bad = NO_CHUNK;
    /* 1) a delta needs its base in place: digest of every UNCHANGED chunk */
    if (im.flags & 1u) {
        run_workers(&gr, threads, crc, zero, NULL);
        for (uint64_t g = 0; g < nc && bad == NO_CHUNK; ++g)
            if (im.kinds[g] == K_UNCHANGED && crc[g] != chunk_crc(&im, g)) bad = g;
        if (bad != NO_CHUNK) { rc = ORC_EBASE; goto done; }
    }
    /* 2) write DATA and ZERO chunks */
    uint64_t pos = 0;
    for (uint32_t a = 0; a < n; ++a) {
        uint64_t nk = ceil_div(sizes[a], im.c);
        for (uint64_t k = 0; k < nk; ++k) {
            uint64_t g = gr.first[a] + k;
            uint64_t lo = k * im.c, hi = lo + im.c < sizes[a] ? lo + im.c : sizes[a];
            uint64_t ln = hi - lo;
            if (im.kinds[g] == K_PACKED) {
                uint64_t rl = rec_len(&im, g, ln);
                if (codec_unpack(im.payload + pos, rl, im.c, data[a] + lo) != 0 && g < bad) bad = g;
                pos += rl;
            } else if (im.kinds[g] == K_DATA) {
                memcpy(data[a] + lo, im.payload + pos, ln);
                for (uint64_t i = ln; i < round16(ln); ++i)
                    if (im.payload[pos + i] && g < bad) bad = g;
                pos += round16(ln);
            } else if (im.kinds[g] == K_ZERO) {
                memset(data[a] + lo, 0, ln);
            }
        }
    }
    /* 3) verify every written chunk and every allocation */
    run_workers(&gr, threads, crc, zero, acrc);
    for (uint64_t g = 0; g < nc; ++g)
        if (im.kinds[g] != K_UNCHANGED && crc[g] != chunk_crc(&im, g) && g < bad) bad = g;
    if (bad != NO_CHUNK) { rc = ORC_ECORRUPT; goto done; }
    for (uint32_t a = 0; a < n; ++a)
        if (acrc[a] != rec_crc(&im, a)) { bad = gr.first[a]; rc = ORC_ECORRUPT; goto done; }
done:
    *first_bad = bad;
    free(gr.first); free(crc); free(zero); free(acrc);
    return rc;
}

/* merge(base, delta): the full image of the delta's state. The result has
 * the codec layout when either input has it. */
int orc_merge(const uint8_t* base, uint64_t blen, const uint8_t* delta, uint64_t dlen,
              uint8_t* out, uint64_t out_cap, uint64_t* out_len) {
    image_t b, d;
    int rc = parse(base, blen, &b);
    if (rc) return rc;
    rc = parse(delta, dlen, &d);
    if (rc) return rc;
    if ((b.flags & F_DELTA) || !(d.flags & F_DELTA) || b.c != d.c) return ORC_EINVAL;
    if (d.base_state != b.state_digest) return ORC_EBASE;
    const int codec = ((b.flags | d.flags) & F_CODEC) != 0;
    /* payload offset of every chunk of the base */
    uint64_t* bpos = (uint64_t*)malloc(8 * (b.n_chunks ? b.n_chunks : 1));
    if (!bpos) return ORC_ENOMEM;
    uint64_t pos = 0;
    for (uint64_t a = 0; a < b.n_allocs; ++a) {
        uint64_t size = rec_size(&b, a), nk = ceil_div(size, b.c);
        for (uint64_t k = 0; k < nk; ++k) {
            uint64_t g = rec_first(&b, a) + k;
            uint64_t lo = k * b.c, hi = lo + b.c < size ? lo + b.c : size;
            bpos[g] = pos;
            pos += rec_len(&b, g, hi - lo);
        }
    }
    uint64_t tl = tables_len(d.n_allocs, d.n_chunks, codec);
    if (64 + tl > out_cap) { free(bpos); return ORC_ENOMEM; }
    memset(out, 0, 64 + tl);
    memcpy(out + 64, d.recs, 32ull * d.n_allocs + 4 * d.n_chunks);   /* recs and crc[] as in the delta */
    uint8_t* rlens = codec ? out + 64 + 32ull * d.n_allocs + 4 * d.n_chunks : NULL;
    uint8_t* kinds = out + 64 + 32ull * d.n_allocs + (codec ? 8 : 4) * d.n_chunks;
    uint64_t opos = 64 + tl, dpos = 0;
    rc = ORC_OK;
    for (uint64_t a = 0; a < d.n_allocs && rc == ORC_OK; ++a) {
        uint64_t size = rec_size(&d, a), nk = ceil_div(size, d.c), id = rec_id(&d, a);
        int64_t bm = -1;
        for (uint64_t x = 0; x < b.n_allocs; ++x)
            if (rec_id(&b, x) == id) { bm = (int64_t)x; break; }
        for (uint64_t k = 0; k < nk; ++k) {
            uint64_t g = rec_first(&d, a) + k;
            uint64_t lo = k * d.c, hi = lo + d.c < size ? lo + d.c : size;
            uint8_t kind = d.kinds[g];
            uint64_t rl = rec_len(&d, g, hi - lo);
            const uint8_t* src = d.payload + dpos;
            dpos += rl;
            if (kind == K_UNCHANGED) {
                if (bm < 0 || rec_size(&b, (uint64_t)bm) != size) { rc = ORC_EBASE; break; }
                uint64_t gb = rec_first(&b, (uint64_t)bm) + k;
                kind = b.kinds[gb];
                rl = rec_len(&b, gb, hi - lo);
                src = b.payload + bpos[gb];
            }
            kinds[g] = kind;
            if (rlens) put32(rlens + 4 * g, (uint32_t)rl);
            if (rl) {
                if (opos + rl > out_cap) { rc = ORC_ENOMEM; break; }
                memcpy(out + opos, src, rl);
                opos += rl;
            }
        }
    }
    free(bpos);
    if (rc) return rc;
    write_header(out, codec ? (uint32_t)F_CODEC : 0u, d.c, d.n_allocs, d.n_chunks, opos - 64 - tl, 0u, d.n,
                 orc_crc32c(out + 64, tl));
    *out_len = opos;
    return ORC_OK;
}

/* Fields of an image after validation (for tests): returns rc. */
int orc_parse(const uint8_t* img, uint64_t len, uint64_t* fields /* [8] */) {
    image_t im;
    int rc = parse(img, len, &im);
    if (rc) return rc;
    fields[0] = im.flags; fields[1] = im.c; fields[2] = im.n_allocs; fields[3] = im.n_chunks;
    fields[4] = im.d; fields[5] = im.base_state; fields[6] = im.n; fields[7] = im.state_digest;
    return ORC_OK;
}
