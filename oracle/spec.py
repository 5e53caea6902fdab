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

Byte-plane codec (an extension of format v1; the paper names data
compression among the techniques that could speed up checkpoint and restore
of large models, section 5.2, and counts compression and quantised snapshots
among the optimisations its method can take on, section 7; it defines no
codec, so the one below is this project's):
  header flag bit1 = CODEC. With it the tables region is
    AllocRec[n_allocs] | u32 crc[n_chunks] | u32 rlen[n_chunks] |
    u8 kind[n_chunks] | zero padding to a multiple of 16
  and kinds may also be PACKED=3. rlen[g] is the length of chunk g's payload
  record: 0 for ZERO and UNCHANGED, round16(len) for DATA, the record length
  for PACKED; D = sum(rlen). A chunk is PACKED only when it has the full
  length C, is neither ZERO nor UNCHANGED, and its record is strictly
  shorter than C. state_digest is still CRC32C(AllocRec[] || crc[]).
  Record of a PACKED chunk of C bytes, whose byte 8e+p is element e of plane
  p (8 planes of L = C/8 bytes):
    48-byte head: u8 mode[8] | u32 esc[8] | 8 zero bytes
    then one section per plane, in plane order, each a multiple of 16 bytes:
      CONST (mode 1), when all L bytes of the plane are equal:
          the value, then 15 zero bytes;
      DICT (mode 2): the dictionary, 16 bytes: the (at most 15) most
          frequent byte values of the plane, by count descending then value
          ascending (only values that occur), unused entries and byte 15
          zero; the codes, L/2 bytes, byte j = code(2j) | code(2j+1) << 4,
          where code(e) is the index of element e's byte among the used
          entries, or 15 (escape), zero-padded to 16; the escapes, the bytes
          of the escaped elements in element order (esc[p] of them),
          zero-padded to 16;
      RAW (mode 0): the L bytes of the plane, zero-padded to 16.
    A plane that is not CONST is DICT when its DICT section is strictly
    shorter than its RAW section, else RAW. esc[p] is 0 unless DICT.
  Restore of a PACKED record checks: every mode <= 2, the 8 reserved head
  bytes zero, esc[p] = 0 unless DICT and esc[p] <= L, the length the head
  implies equals rlen[g], and each DICT plane holds exactly esc[p] escape
  codes; then the decoded chunk's digest against crc[g]. Padding and unused
  dictionary entries do not reach the decoded chunk and are not checked.
"""

import struct

# ---------------------------------------------------------------- constants
POLY_CRC32C_REFLECTED = 0x82F63B78      # Castagnoli 0x1EDC6F41, bit-reversed
MAGIC = b"MICKPT01"
VERSION = 1
FLAG_DELTA = 1
FLAG_CODEC = 2
HEADER_BYTES = 64
ALLOCREC_BYTES = 32
ZERO, DATA, UNCHANGED, PACKED = 0, 1, 2, 3
PLANES = 8
RECORD_HEAD = 48
MODE_RAW, MODE_CONST, MODE_DICT = 0, 1, 2

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


def _tables_len(n_allocs, n_chunks, codec=False):
    return _round16(ALLOCREC_BYTES * n_allocs + (9 if codec else 5) * n_chunks)


def _valid_chunk_size(c):
    return 16 <= c <= (1 << 30) and (c & (c - 1)) == 0


def chunk_spans(size, c):
    """Chunk k of an allocation covers bytes [k*c, min((k+1)*c, size))."""
    return [(k * c, min((k + 1) * c, size)) for k in range(_ceil_div(size, c))]


# ---------------------------------------------------------------- codec
def _plane_sections(c):
    """Section lengths of a plane of L = c/8 bytes: (raw, const, dict(E))."""
    L = c // PLANES
    return _round16(L), 16, (lambda e: 16 + _round16(L // 2) + _round16(e))


def pack_chunk(chunk):
    """Record of a full chunk under the byte-plane codec, or None when the
    record would not be strictly shorter than the chunk."""
    chunk = bytes(chunk)
    c = len(chunk)
    L = c // PLANES
    raw_len, const_len, dict_len = _plane_sections(c)
    modes, escs, sections = [], [], []
    for p in range(PLANES):
        plane = chunk[p::PLANES]
        counts = {}
        for b in plane:
            counts[b] = counts.get(b, 0) + 1
        if len(counts) == 1:
            modes.append(MODE_CONST)
            escs.append(0)
            sections.append(bytes([plane[0]]) + bytes(15))
            continue
        ranked = sorted(counts, key=lambda v: (-counts[v], v))[:15]
        index = {v: i for i, v in enumerate(ranked)}
        codes = [index.get(b, 15) for b in plane]
        escapes = bytes(b for b, k in zip(plane, codes) if k == 15)
        if dict_len(len(escapes)) < raw_len:
            dictionary = bytes(ranked) + bytes(16 - len(ranked))
            packed = bytes(codes[2 * j] | (codes[2 * j + 1] << 4) for j in range(L // 2))
            sec = (dictionary + packed + bytes(_round16(len(packed)) - len(packed))
                   + escapes + bytes(_round16(len(escapes)) - len(escapes)))
            modes.append(MODE_DICT)
            escs.append(len(escapes))
        else:
            sec = plane + bytes(raw_len - L)
            modes.append(MODE_RAW)
            escs.append(0)
        sections.append(sec)
    head = bytes(modes) + struct.pack("<8I", *escs) + bytes(8)
    record = head + b"".join(sections)
    return record if len(record) < c else None


def unpack_record(record, c):
    """Decode a PACKED record of a chunk of c bytes. Returns the chunk, or
    None when the record breaks one of the checked rules."""
    rec = bytes(record)
    L = c // PLANES
    raw_len, const_len, dict_len = _plane_sections(c)
    if len(rec) < RECORD_HEAD:
        return None
    modes = list(rec[:PLANES])
    escs = list(struct.unpack_from("<8I", rec, PLANES))
    if any(rec[40:48]):
        return None
    length = RECORD_HEAD
    for m, e in zip(modes, escs):
        if m > MODE_DICT or (m != MODE_DICT and e != 0) or e > L:
            return None
        length += raw_len if m == MODE_RAW else const_len if m == MODE_CONST else dict_len(e)
    if length != len(rec):
        return None
    planes = []
    pos = RECORD_HEAD
    for m, e in zip(modes, escs):
        if m == MODE_RAW:
            planes.append(rec[pos:pos + L])
            pos += raw_len
        elif m == MODE_CONST:
            planes.append(bytes([rec[pos]]) * L)
            pos += const_len
        else:
            dictionary = rec[pos:pos + 16]
            packed = rec[pos + 16:pos + 16 + L // 2]
            codes = []
            for byte in packed:
                codes += [byte & 15, byte >> 4]
            if codes.count(15) != e:
                return None
            esc_at = pos + 16 + _round16(L // 2)
            out, i = bytearray(), 0
            for k in codes:
                if k == 15:
                    out.append(rec[esc_at + i])
                    i += 1
                else:
                    out.append(dictionary[k])
            planes.append(bytes(out))
            pos += dict_len(e)
    chunk = bytearray(c)
    for p in range(PLANES):
        chunk[p::PLANES] = planes[p]
    return bytes(chunk)


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
    if flags & ~(FLAG_DELTA | FLAG_CODEC) or reserved != 0 or not _valid_chunk_size(c):
        return ECORRUPT, None
    if n_chunks > (1 << 40) or n_allocs > (1 << 24):
        return ECORRUPT, None
    codec = bool(flags & FLAG_CODEC)
    tl = _tables_len(n_allocs, n_chunks, codec)
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
    koff = off + 4 * n_chunks
    rlens = None
    if codec:
        rlens = list(struct.unpack_from("<%dI" % n_chunks, tr, koff))
        koff += 4 * n_chunks
    kinds = list(tr[koff: koff + n_chunks])
    pad = tr[koff + n_chunks:]
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
            if k > PACKED or (k == UNCHANGED and not delta) or (k == PACKED and not codec):
                return ECORRUPT, None
            want = _round16(hi - lo) if k == DATA else 0
            if k == PACKED:
                # a full chunk whose record is shorter than the chunk
                want = rlens[g]
                if hi - lo != c or want % 16 or not RECORD_HEAD + 16 * PLANES <= want < c:
                    return ECORRUPT, None
            if codec and rlens[g] != want:
                return ECORRUPT, None
            dsum += want
            g += 1
        total += size
    if g != n_chunks or total != n_total or dsum != d or any(pad):
        return ECORRUPT, None
    if (not delta) and base_state != 0:
        return ECORRUPT, None
    return OK, dict(version=version, flags=flags, C=c, n_allocs=n_allocs,
                    n_chunks=n_chunks, D=d, base_state=base_state, N=n_total,
                    tables_crc=tables_crc, header_crc=header_crc, recs=recs,
                    crcs=crcs, kinds=kinds, rlens=rlens,
                    payload=img[HEADER_BYTES + tl:],
                    state_digest=crc32c(tr[:off + 4 * n_chunks]))


def _build(c, flags, base_state, recs, crcs, kinds, payload, rlens=None):
    n_allocs, n_chunks = len(recs), len(crcs)
    tr = bytearray()
    for (aid, size, first, acrc) in recs:
        tr += struct.pack("<QQQII", aid, size, first, acrc, 0)
    tr += struct.pack("<%dI" % n_chunks, *crcs)
    if flags & FLAG_CODEC:
        tr += struct.pack("<%dI" % n_chunks, *rlens)
    tr += bytes(kinds)
    tr += bytes(_tables_len(n_allocs, n_chunks, bool(flags & FLAG_CODEC)) - len(tr))
    n_total = sum(r[1] for r in recs)
    head = MAGIC + struct.pack("<IIIIQQIIQI", VERSION, flags, c, n_allocs, n_chunks,
                               len(payload), base_state, 0, n_total, crc32c(tr))
    head += struct.pack("<I", crc32c(head))
    return bytes(head) + bytes(tr) + bytes(payload)


# ---------------------------------------------------------------- dump
def dump(allocs, c, prev=None, codec=False):
    """Checkpoint: allocs is a list of (id, bytes-like) in table order.

    Returns (rc, image bytes or None). With prev (an image), chunks whose
    digest equals the digest of the same chunk of the allocation with the
    same id and size in prev are marked UNCHANGED and carry no payload
    (the incremental / pre-dump reading). A zero chunk is ZERO whatever prev
    says (ZERO > UNCHANGED > DATA). With codec, a full DATA chunk whose
    byte-plane record is shorter than the chunk is stored as that record
    (PACKED).
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
    if codec:
        flags |= FLAG_CODEC
    recs, crcs, kinds, rlens, payload = [], [], [], [], bytearray()
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
                record = pack_chunk(piece) if codec and len(piece) == c else None
                if record is not None:
                    kind = PACKED
                else:
                    record = piece + bytes(_round16(len(piece)) - len(piece))
                payload += record
            crcs.append(d)
            kinds.append(kind)
            rlens.append(len(record) if kind in (DATA, PACKED) else 0)
            g += 1
    return OK, _build(c, flags, base_state, recs, crcs, kinds, payload, rlens)


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
    # 2) write DATA, PACKED and ZERO chunks, verifying each against its digest
    pay = p["payload"]
    pos = 0
    for (aid, buf), rec in zip(allocs, p["recs"]):
        for k, (lo, hi) in enumerate(chunk_spans(rec[1], c)):
            g = rec[2] + k
            kind = p["kinds"][g]
            n = hi - lo
            if kind == PACKED:
                rl = p["rlens"][g]
                chunk = unpack_record(pay[pos:pos + rl], c)
                pos += rl
                if chunk is None:
                    bad = min(bad, g)
                    continue
                buf[lo:hi] = chunk
                if crc32c(chunk) != p["crcs"][g]:
                    bad = min(bad, g)
            elif kind == DATA:
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

    def rlen_of(img, g, lo, hi):
        if img["rlens"] is not None:
            return img["rlens"][g]
        return _round16(hi - lo) if img["kinds"][g] == DATA else 0

    # payload position and record length of every chunk of the base
    bpos, pos = {}, 0
    brecs = {}
    for rec in b["recs"]:
        brecs[rec[0]] = rec
        for k, (lo, hi) in enumerate(chunk_spans(rec[1], c)):
            g = rec[2] + k
            bpos[g] = (pos, rlen_of(b, g, lo, hi))
            pos += bpos[g][1]
    # the merged image carries the codec layout when either input does
    flags = (b["flags"] | d["flags"]) & FLAG_CODEC
    kinds, rlens, payload, pos = [], [], bytearray(), 0
    for rec in d["recs"]:
        for k, (lo, hi) in enumerate(chunk_spans(rec[1], c)):
            g = rec[2] + k
            kind = d["kinds"][g]
            rl = rlen_of(d, g, lo, hi)
            if kind in (DATA, PACKED):
                payload += d["payload"][pos:pos + rl]
            pos += rl
            if kind == UNCHANGED:
                br = brecs.get(rec[0])
                if br is None or br[1] != rec[1]:
                    return EBASE, None
                gb = br[2] + k
                kind = b["kinds"][gb]
                bp, rl = bpos[gb]
                payload += b["payload"][bp:bp + rl]
            kinds.append(kind)
            rlens.append(rl)
    recs = [(r[0], r[1], r[2], r[3]) for r in d["recs"]]
    return OK, _build(c, flags, 0, recs, d["crcs"], kinds, payload, rlens)
