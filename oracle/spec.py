"""Spec oracle for the checkpoint image, in plain Python.

TEST INFRASTRUCTURE ONLY. Only tests/, __graft_entry__.smoke() and bench.py's
CPU-baseline leg may import this module. The product path never calls it.

This is the slow, obviously-correct statement of what the GPU path computes,
meant for tiny inputs (bitwise CRC: a few microseconds per byte). A second,
independent CPU implementation in plain C lives beside it (ckpt_oracle.c);
the two share no code and are checked against each other by brute force.

What the method computes (paper, section 3, "Transparent GPU Checkpointing"):
  * a checkpoint captures the memory contents of every device buffer of a
    process into host memory (section 3.1.1, the "checkpointing" action;
    section 3.1.2, buffer-object records carry handle, size, address and
    memory contents);
  * a restore writes that memory back so the process resumes with identical
    state (section 3.1.1, the "restore" action; section 6, deterministic
    restore);
  * restore requires a compatible target: same buffers, same sizes
    (section 3.1.2, topology compatibility);
  * the CRIU operation set includes a pre-dump before the final dump
    (section 3.1, plugin initialisation), and incremental / differential
    checkpointing is named as a complementary optimisation (section 7,
    "Checkpoint/Restore Optimizations").

The paper does not define an image format, a digest or a chunk grid. The
format below is this project's reading (image format v1); every choice is
listed with its reason in the design notes. Parity of the byte layout itself
is unpinned by the paper: it is pinned only by its own definition (field
offsets checked by struct-level tests), by published CRC-32C values, and by
agreement of two independent CPU implementations.

Image format v1 (all integers little-endian):
  header, 64 bytes:
     0  magic "MICKPT01"        8
     8  u32 version = 1
    12  u32 flags              bit0 = DELTA
    16  u32 C                  chunk size, power of two, 16 .. 2**30
    20  u32 n_allocs
    24  u64 n_chunks
    32  u64 D                  payload bytes
    40  u32 base_state         state digest of the base image (0 if full)
    44  u32 reserved = 0
    48  u64 N                  logical bytes (sum of allocation sizes)
    56  u32 tables_crc         CRC32C of the tables region TR
    60  u32 header_crc         CRC32C of header bytes [0, 60)
  tables region TR:
    AllocRec[n_allocs], 32 bytes each: u64 id | u64 size | u64 first_chunk |
                                       u32 alloc_crc | u32 0
    u32 crc[n_chunks]
    u8  kind[n_chunks]          ZERO=0, DATA=1, UNCHANGED=2
    zero padding so that |TR| is a multiple of 16
  payload: for every DATA chunk in increasing chunk index, its bytes followed
    by zeros up to a multiple of 16.
  state_digest = CRC32C(AllocRec[] || crc[])   (kinds excluded)
"""

import struct

# ---------------------------------------------------------------- constants
POLY_CRC32C_REFLECTED = 0x82F63B78      # Castagnoli 0x1EDC6F41, bit-reversed
MAGIC = b"MICKPT01"
VERSION = 1
FLAG_DELTA = 1
HEADER_BYTES = 64
ALLOCREC_BYTES = 32
ZERO, DATA, UNCHANGED = 0, 1, 2

OK, EINVAL, ENOMEM, EHIP, ECORRUPT, EMISMATCH, EBASE, ETIMEOUT = 0, -1, -2, -3, -4, -5, -6, -7
NO_CHUNK = (1 << 64) - 1
MASK32 = 0xFFFFFFFF


# ---------------------------------------------------------------- CRC core
def crc_bitwise(data, poly=POLY_CRC32C_REFLECTED, init=MASK32, xorout=MASK32):
    """Reflected CRC-32, one bit at a time (the textbook shift register).

    With the default arguments this is CRC-32C as used by iSCSI (RFC 3720):
    register preset to all ones, message bits fed least-significant first,
    final complement. With poly=0xEDB88320 it is the zlib / IEEE CRC-32.
    """
    crc = init
    for b in bytes(data):
        crc ^= b
        for _ in range(8):
            crc = (crc >> 1) ^ (poly if crc & 1 else 0)
    return crc ^ xorout


def crc32c(data):
    return crc_bitwise(data)


# ---------------------------------------------------------------- helpers
def _ceil_div(a, b):
    return (a + b - 1) // b


def _round16(n):
    return (n + 15) & ~15


def _tables_len(n_allocs, n_chunks):
    return _round16(ALLOCREC_BYTES * n_allocs + 5 * n_chunks)


def _valid_chunk_size(c):
    return 16 <= c <= (1 << 30) and (c & (c - 1)) == 0


def chunk_spans(size, c):
    """Chunk k of an allocation covers bytes [k*c, min((k+1)*c, size))."""
    return [(k * c, min((k + 1) * c, size)) for k in range(_ceil_div(size, c))]


def parse(image):
    """Split an image into its fields. Returns (rc, dict). Checks that the
    header is intact and that the tables region is self-consistent; does not
    look at any allocation table."""
    img = bytes(image)
    if len(img) < HEADER_BYTES or img[:8] != MAGIC:
        return ECORRUPT, None
    (version, flags, c, n_allocs, n_chunks, d, base_state, reserved, n_total,
     tables_crc, header_crc) = struct.unpack_from("<IIIIQQIIQII", img, 8)
    if header_crc != crc32c(img[:60]) or version != VERSION:
        return ECORRUPT, None
    if flags & ~FLAG_DELTA or reserved != 0 or not _valid_chunk_size(c):
        return ECORRUPT, None
    if n_chunks > (1 << 40) or n_allocs > (1 << 24):
        return ECORRUPT, None
    tl = _tables_len(n_allocs, n_chunks)
    if len(img) != HEADER_BYTES + tl + d:
        return ECORRUPT, None
    tr = img[HEADER_BYTES:HEADER_BYTES + tl]
    if crc32c(tr) != tables_crc:
        return ECORRUPT, None
    recs = []
    for a in range(n_allocs):
        aid, size, first, acrc, zero = struct.unpack_from("<QQQII", tr, a * ALLOCREC_BYTES)
        recs.append((aid, size, first, acrc, zero))
    off = ALLOCREC_BYTES * n_allocs
    crcs = list(struct.unpack_from("<%dI" % n_chunks, tr, off))
    kinds = list(tr[off + 4 * n_chunks: off + 5 * n_chunks])
    pad = tr[off + 5 * n_chunks:]
    # structural consistency of the tables with the header
    g = 0
    total = 0
    delta = bool(flags & FLAG_DELTA)
    dsum = 0
    for (aid, size, first, acrc, zero) in recs:
        if first != g or zero != 0:
            return ECORRUPT, None
        for (lo, hi) in chunk_spans(size, c):
            k = kinds[g]
            if k > UNCHANGED or (k == UNCHANGED and not delta):
                return ECORRUPT, None
            if k == DATA:
                dsum += _round16(hi - lo)
            g += 1
        total += size
    if g != n_chunks or total != n_total or dsum != d or any(pad):
        return ECORRUPT, None
    if (not delta) and base_state != 0:
        return ECORRUPT, None
    return OK, dict(version=version, flags=flags, C=c, n_allocs=n_allocs,
                    n_chunks=n_chunks, D=d, base_state=base_state, N=n_total,
                    tables_crc=tables_crc, header_crc=header_crc, recs=recs,
                    crcs=crcs, kinds=kinds,
                    payload=img[HEADER_BYTES + tl:],
                    state_digest=crc32c(tr[:off + 4 * n_chunks]))


def _build(c, flags, base_state, recs, crcs, kinds, payload):
    n_allocs, n_chunks = len(recs), len(crcs)
    tr = bytearray()
    for (aid, size, first, acrc) in recs:
        tr += struct.pack("<QQQII", aid, size, first, acrc, 0)
    tr += struct.pack("<%dI" % n_chunks, *crcs)
    tr += bytes(kinds)
    tr += bytes(_tables_len(n_allocs, n_chunks) - len(tr))
    n_total = sum(r[1] for r in recs)
    head = MAGIC + struct.pack("<IIIIQQIIQI", VERSION, flags, c, n_allocs, n_chunks,
                               len(payload), base_state, 0, n_total, crc32c(tr))
    head += struct.pack("<I", crc32c(head))
    return bytes(head) + bytes(tr) + bytes(payload)


# ---------------------------------------------------------------- dump
def dump(allocs, c, prev=None):
    """Checkpoint: allocs is a list of (id, bytes-like) in table order.

    Returns (rc, image bytes or None). With prev (an image), chunks whose
    digest equals the digest of the same chunk of the allocation with the
    same id and size in prev are marked UNCHANGED and carry no payload
    (the incremental / pre-dump reading). A zero chunk is ZERO whatever prev
    says (ZERO > UNCHANGED > DATA).
    """
    if not _valid_chunk_size(c):
        return EINVAL, None
    ids = [a for a, _ in allocs]
    if len(set(ids)) != len(ids):
        return EINVAL, None
    prev_map = {}
    base_state = 0
    flags = 0
    if prev is not None:
        rc, p = parse(prev)
        if rc != OK:
            return rc, None
        if p["C"] != c:
            return EINVAL, None
        flags = FLAG_DELTA
        base_state = p["state_digest"]
        for (aid, size, first, _, _) in p["recs"]:
            prev_map[aid] = (size, first)
    recs, crcs, kinds, payload = [], [], [], bytearray()
    g = 0
    for (aid, data) in allocs:
        data = bytes(data)
        size = len(data)
        match = prev_map.get(aid)
        if match is not None and match[0] != size:
            match = None
        recs.append((aid, size, g, crc32c(data)))
        for k, (lo, hi) in enumerate(chunk_spans(size, c)):
            piece = data[lo:hi]
            d = crc32c(piece)
            if not any(piece):
                kind = ZERO
            elif match is not None and p["crcs"][match[1] + k] == d:
                kind = UNCHANGED
            else:
                kind = DATA
                payload += piece + bytes(_round16(len(piece)) - len(piece))
            crcs.append(d)
            kinds.append(kind)
            g += 1
    return OK, _build(c, flags, base_state, recs, crcs, kinds, payload)


# ---------------------------------------------------------------- restore
def restore(image, allocs):
    """Restore: allocs is a list of (id, bytearray) in table order; the
    bytearrays are written in place. Returns (rc, first_bad_chunk)."""
    rc, p = parse(image)
    if rc != OK:
        return rc, NO_CHUNK
    if p["n_allocs"] != len(allocs):
        return EMISMATCH, NO_CHUNK
    for (aid, buf), rec in zip(allocs, p["recs"]):
        if aid != rec[0] or len(buf) != rec[1]:
            return EMISMATCH, NO_CHUNK
    c = p["C"]
    # 1) a delta needs the target to hold its base: every UNCHANGED chunk of
    #    the target must already carry the digest recorded for it
    bad = NO_CHUNK
    for (aid, buf), rec in zip(allocs, p["recs"]):
        for k, (lo, hi) in enumerate(chunk_spans(rec[1], c)):
            g = rec[2] + k
            if p["kinds"][g] == UNCHANGED and crc32c(bytes(buf[lo:hi])) != p["crcs"][g]:
                bad = min(bad, g)
    if bad != NO_CHUNK:
        return EBASE, bad
    # 2) write DATA and ZERO chunks, verifying each against its digest
    pay = p["payload"]
    pos = 0
    for (aid, buf), rec in zip(allocs, p["recs"]):
        for k, (lo, hi) in enumerate(chunk_spans(rec[1], c)):
            g = rec[2] + k
            kind = p["kinds"][g]
            n = hi - lo
            if kind == DATA:
                buf[lo:hi] = pay[pos:pos + n]
                if any(pay[pos + n:pos + _round16(n)]):
                    bad = min(bad, g)
                pos += _round16(n)
                if crc32c(bytes(buf[lo:hi])) != p["crcs"][g]:
                    bad = min(bad, g)
            elif kind == ZERO:
                buf[lo:hi] = bytes(n)
                if crc32c(bytes(n)) != p["crcs"][g]:
                    bad = min(bad, g)
    if bad != NO_CHUNK:
        return ECORRUPT, bad
    # 3) whole-allocation digests
    for (aid, buf), rec in zip(allocs, p["recs"]):
        if crc32c(bytes(buf)) != rec[3]:
            return ECORRUPT, rec[2]
    return OK, NO_CHUNK


# ---------------------------------------------------------------- merge
def merge(base, delta):
    """Fold a delta image into the full image of its base. Returns (rc, image)."""
    rc, b = parse(base)
    if rc != OK:
        return rc, None
    rc, d = parse(delta)
    if rc != OK:
        return rc, None
    if b["flags"] & FLAG_DELTA or not d["flags"] & FLAG_DELTA or b["C"] != d["C"]:
        return EINVAL, None
    if d["base_state"] != b["state_digest"]:
        return EBASE, None
    c = d["C"]
    # payload position of every DATA chunk of the base
    bpos, pos = {}, 0
    brecs = {}
    for rec in b["recs"]:
        brecs[rec[0]] = rec
        for k, (lo, hi) in enumerate(chunk_spans(rec[1], c)):
            g = rec[2] + k
            if b["kinds"][g] == DATA:
                bpos[g] = pos
                pos += _round16(hi - lo)
    kinds, payload, pos = [], bytearray(), 0
    for rec in d["recs"]:
        for k, (lo, hi) in enumerate(chunk_spans(rec[1], c)):
            g = rec[2] + k
            kind = d["kinds"][g]
            n16 = _round16(hi - lo)
            if kind == DATA:
                payload += d["payload"][pos:pos + n16]
                pos += n16
            elif kind == UNCHANGED:
                br = brecs.get(rec[0])
                if br is None or br[1] != rec[1]:
                    return EBASE, None
                gb = br[2] + k
                kind = b["kinds"][gb]
                if kind == DATA:
                    payload += b["payload"][bpos[gb]:bpos[gb] + n16]
            kinds.append(kind)
    recs = [(r[0], r[1], r[2], r[3]) for r in d["recs"]]
    return OK, _build(c, 0, 0, recs, d["crcs"], kinds, payload)
