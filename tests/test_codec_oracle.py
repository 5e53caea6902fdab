"""Pins of the byte-plane codec in both CPU oracles.

The paper names data compression as a way to speed up checkpoint and restore
(section 5.2) but defines no codec, so parity of the record layout is not
pinned by the paper. It is pinned here by worked records derived by hand from
the layout definition (nibble order, dictionary order and ties, escapes,
padding), closed-form record sizes, round trips, the merge invariant, and
agreement of the two independent oracles on images and on every corruption
of one.
"""
import struct

import numpy as np
import pytest

from oracle import oracle as corc
from oracle import spec

OK, ECORRUPT = 0, -4
ZERO, DATA, UNCHANGED, PACKED = 0, 1, 2, 3
NO_CHUNK = (1 << 64) - 1


def r16(n):
    return (n + 15) & ~15


def planes_to_chunk(planes):
    """Interleave 8 planes (element e of plane p is byte 8e+p)."""
    L = len(planes[0])
    out = bytearray(8 * L)
    for p, pl in enumerate(planes):
        out[p::8] = bytes(pl)
    return bytes(out)


# ------------------------------------------------------------------ worked records
def test_worked_record_two_values_and_constant_planes():
    # C = 512, L = 64: plane 0 alternates 1, 2 (equal counts: the dictionary
    # is [1, 2], ascending on the tie), planes 1..7 hold a constant 0x00 ..
    # 0x06 (CONST). Derived by hand: head = modes 2,1,1,1,1,1,1,1, escape
    # counts 0, 8 zero bytes; plane 0 = dictionary 01 02 + 14 zeros, then 32
    # code bytes 0x10 (code 0 in the low nibble, code 1 in the high one);
    # planes 1..7 = the value then 15 zeros. 48 + 48 + 7 * 16 = 208 bytes.
    planes = [bytes([1, 2] * 32)] + [bytes([p - 1]) * 64 for p in range(1, 8)]
    chunk = planes_to_chunk(planes)
    want = (bytes([2, 1, 1, 1, 1, 1, 1, 1]) + bytes(32) + bytes(8)
            + bytes([1, 2]) + bytes(14) + bytes([0x10]) * 32
            + b"".join(bytes([p - 1]) + bytes(15) for p in range(1, 8)))
    assert len(want) == 208
    assert spec.pack_chunk(chunk) == want
    rc, img = corc.dump([(9, np.frombuffer(chunk, np.uint8))], 512, codec=True)
    assert rc == OK
    assert img[-208:].tobytes() == want
    assert spec.unpack_record(want, 512) == chunk


def test_worked_record_with_escapes():
    # C = 1024, L = 128: plane 3 cycles through 0..15 (8 of each): the
    # dictionary is 0..14 (ties ascending), value 15 is escaped 8 times.
    # Code byte j = code(2j) | code(2j+1) << 4 -> 0x10, 0x32, ..., 0xFE,
    # repeated; escapes = eight 0x0F then 8 zero bytes of padding. DICT
    # section 16 + 64 + 16 = 96 < 128 (RAW). The other planes are random
    # bytes (RAW, 128 bytes each).
    rng = np.random.default_rng(7)
    planes = [rng.integers(0, 256, 128, dtype=np.uint8).tobytes() for _ in range(8)]
    planes[3] = bytes(e % 16 for e in range(128))
    chunk = planes_to_chunk(planes)
    rec = spec.pack_chunk(chunk)
    head = bytes([0, 0, 0, 2, 0, 0, 0, 0]) + struct.pack("<8I", 0, 0, 0, 8, 0, 0, 0, 0) + bytes(8)
    sec3 = (bytes(range(15)) + bytes(1)
            + bytes([0x10, 0x32, 0x54, 0x76, 0x98, 0xBA, 0xDC, 0xFE]) * 8
            + bytes([15]) * 8 + bytes(8))
    want = head + b"".join(planes[p] if p != 3 else sec3 for p in range(8))
    assert len(want) == 48 + 7 * 128 + 96 == 1040 > 1024
    # 1040 is not shorter than the chunk: the chunk stays DATA
    assert rec is None
    # with two more compressible planes the record is taken
    planes[0] = bytes(e % 16 for e in range(128))
    planes[5] = bytes([0xAB]) * 128
    chunk = planes_to_chunk(planes)
    rec = spec.pack_chunk(chunk)
    assert rec is not None and len(rec) == 48 + 5 * 128 + 2 * 96 + 16
    assert rec[:8] == bytes([2, 0, 0, 2, 0, 1, 0, 0])
    assert struct.unpack_from("<8I", rec, 8) == (8, 0, 0, 8, 0, 0, 0, 0)
    assert rec[48:48 + 96] == sec3
    assert spec.unpack_record(rec, 1024) == chunk


def test_dictionary_takes_most_frequent_values():
    # C = 4096, L = 512: plane 7 holds value v with count 40 - v for v < 20
    # (sum 610 > 512, so the counts are cut to fit), the dictionary must be
    # the 15 most frequent, most frequent first
    counts = [40 - v for v in range(20)]
    vals = []
    for v, n in enumerate(counts):
        vals += [v] * n
    vals = vals[:512]
    rng = np.random.default_rng(1)
    rng.shuffle(vals)
    planes = [bytes(512)] * 7 + [bytes(vals)]
    rec = spec.pack_chunk(planes_to_chunk(planes))
    assert rec[7] == 2
    off = 48 + 7 * 16
    assert list(rec[off:off + 15]) == list(range(15)) and rec[off + 15] == 0
    kept = sum(min(vals.count(v), 99) for v in range(15))
    assert struct.unpack_from("<I", rec, 8 + 4 * 7)[0] == 512 - kept


# ------------------------------------------------------------------ closed forms
@pytest.mark.parametrize("c", [512, 1024, 4096, 65536])
def test_record_sizes_in_closed_form(c):
    L = c // 8
    rng = np.random.default_rng(c)
    # every plane constant: 48 + 8 * 16
    planes = [bytes([p * 17]) * L for p in range(8)]
    assert len(spec.pack_chunk(planes_to_chunk(planes))) == 48 + 8 * 16
    # every plane from at most 15 values, not constant: no escapes
    planes = [rng.integers(0, 15, L, dtype=np.uint8).tobytes() for _ in range(8)]
    rec = spec.pack_chunk(planes_to_chunk(planes))
    assert len(rec) == 48 + 8 * (16 + r16(L // 2))
    assert struct.unpack_from("<8I", rec, 8) == (0,) * 8
    # uniformly random bytes: no record shorter than the chunk
    assert spec.pack_chunk(rng.integers(0, 256, c, dtype=np.uint8).tobytes()) is None


def test_planted_tie_break_mistake_is_caught(monkeypatch):
    # a codec that orders equal counts by descending value must fail the
    # worked record
    real_sorted = sorted

    def wrong_sorted(it, key=None, reverse=False):
        out = real_sorted(it, key=key, reverse=reverse)
        if key is not None and len(out) == 2:
            out = out[::-1]
        return out

    monkeypatch.setattr(spec, "sorted", wrong_sorted, raising=False)
    with pytest.raises(AssertionError):
        test_worked_record_two_values_and_constant_planes()


# ------------------------------------------------------------------ images
def _families(rng, c):
    def bf16(n, s):
        x = (rng.standard_normal(n) * s).astype(np.float32)
        return (x.view(np.uint32) >> 16).astype(np.uint16).view(np.uint8)
    return [
        (1, bf16(3 * c // 2 + 7, 0.02)),
        (2, (rng.standard_normal(c // 2) * 1e-3).astype(np.float32).view(np.uint8)),
        (3, rng.integers(0, 256, c + 48, dtype=np.uint8)),
        (4, np.zeros(2 * c, np.uint8)),
        (5, np.tile(np.arange(8, dtype=np.uint8), c // 4)),
        (6, rng.integers(0, 3, 2 * c, dtype=np.uint8)),
        (7, np.zeros(0, np.uint8)),
        (8, rng.standard_normal(c // 4).view(np.uint8)),
    ]


@pytest.mark.parametrize("c", [256, 512, 1024, 4096])
def test_codec_images_spec_equals_c_and_restore(c):
    rng = np.random.default_rng(c + 1)
    allocs = _families(rng, c)
    rc1, a = spec.dump([(i, x.tobytes()) for i, x in allocs], c, codec=True)
    rc2, b = corc.dump(allocs, c, codec=True)
    assert rc1 == rc2 == OK
    assert a == b.tobytes()
    rc, p = spec.parse(a)
    assert rc == OK and p["flags"] == 2
    assert p["D"] == sum(p["rlens"])
    if c >= 512:
        assert PACKED in p["kinds"]
    for k, rl in zip(p["kinds"], p["rlens"]):
        if k == PACKED:
            assert rl % 16 == 0 and 176 <= rl < c
    # both restores give the bytes back
    for impl in (spec, corc):
        bufs = [(i, np.zeros_like(x)) for i, x in allocs]
        if impl is spec:
            bb = [(i, bytearray(x.size)) for i, x in allocs]
            assert spec.restore(a, bb) == (OK, NO_CHUNK)
            assert all(bytes(y) == x.tobytes() for (_, y), (_, x) in zip(bb, allocs))
        else:
            assert corc.restore(a, bufs) == (OK, NO_CHUNK)
            assert all((y == x).all() for (_, y), (_, x) in zip(bufs, allocs))
    # same digests and state digest as the plain image
    rc, plain = corc.dump(allocs, c)
    rc, q = spec.parse(plain.tobytes())
    assert q["crcs"] == p["crcs"] and q["state_digest"] == p["state_digest"]
    assert [k if k != PACKED else DATA for k in p["kinds"]] == q["kinds"]


def test_codec_delta_and_merge():
    c = 1024
    rng = np.random.default_rng(21)
    base = _families(rng, c)
    new = [(i, x.copy()) for i, x in base]
    new[0][1][5] ^= 1            # one chunk of allocation 1 changes
    new[5][1][:c] = 7            # a chunk of allocation 6 becomes constant
    rc, b_img = corc.dump(base, c, codec=True)
    rc, d_img = corc.dump(new, c, prev=b_img, codec=True)
    rc, f_img = corc.dump(new, c, codec=True)
    rc1, m1 = corc.merge(b_img, d_img)
    rc2, m2 = spec.merge(b_img.tobytes(), d_img.tobytes())
    assert rc1 == rc2 == OK
    assert m1.tobytes() == m2 == f_img.tobytes()
    rc, d_spec = spec.dump([(i, x.tobytes()) for i, x in new], c, prev=b_img.tobytes(), codec=True)
    assert d_spec == d_img.tobytes()
    # a plain base with a codec delta: the merge has the codec layout and
    # restores the new state
    rc, pb = corc.dump(base, c)
    rc, pd = corc.dump(new, c, prev=pb, codec=True)
    rc, mm = corc.merge(pb, pd)
    assert rc == OK and spec.parse(mm.tobytes())[1]["flags"] == 2
    bufs = [(i, np.zeros_like(x)) for i, x in new]
    assert corc.restore(mm, bufs) == (OK, NO_CHUNK)
    assert all((y == x).all() for (_, y), (_, x) in zip(bufs, new))
    # in-place delta restore over the base
    bufs = [(i, x.copy()) for i, x in base]
    assert corc.restore(d_img, bufs) == (OK, NO_CHUNK)
    assert all((y == x).all() for (_, y), (_, x) in zip(bufs, new))


def _rewrite_tables(img, mutate):
    """Apply mutate(bytearray payload) and return the image (tables intact)."""
    b = bytearray(img)
    mutate(b)
    return bytes(b)


def test_corrupt_records_are_reported_at_their_chunk():
    c = 1024
    rng = np.random.default_rng(5)
    allocs = _families(rng, c)
    rc, img = corc.dump(allocs, c, codec=True)
    img = img.tobytes()
    rc, p = spec.parse(img)
    tl = len(img) - p["D"]
    g = p["kinds"].index(PACKED)
    at = tl + sum(p["rlens"][:g])
    rec = img[at:at + p["rlens"][g]]
    dict_planes = [q for q in range(8) if rec[q] == 2]
    cases = {
        "mode out of range": lambda b: b.__setitem__(at, 3),
        "reserved head byte": lambda b: b.__setitem__(at + 44, 1),
        "escape count off by one": lambda b: b.__setitem__(at + 8 + 4 * dict_planes[0],
                                                           b[at + 8 + 4 * dict_planes[0]] + 1),
    }
    for name, mut in cases.items():
        bad = _rewrite_tables(img, mut)
        for impl in (spec, corc):
            if impl is spec:
                bufs = [(i, bytearray(x.size)) for i, x in allocs]
                got = spec.restore(bad, bufs)
            else:
                bufs = [(i, np.zeros_like(x)) for i, x in allocs]
                got = corc.restore(bad, bufs)
            assert got == (ECORRUPT, g), (name, impl)


def test_every_byte_flip_of_a_codec_image_agrees_in_both_oracles():
    c = 256
    rng = np.random.default_rng(8)
    allocs = [(1, np.tile(np.arange(8, dtype=np.uint8), c // 8 * 2)),
              (2, rng.integers(0, 2, c, dtype=np.uint8) * 3),
              (3, np.zeros(c, np.uint8))]
    rc, img = corc.dump(allocs, c, codec=True)
    img = img.tobytes()
    assert PACKED in spec.parse(img)[1]["kinds"]
    for i in range(len(img)):
        bad = bytearray(img)
        bad[i] ^= 0x5A
        bb = [(k, bytearray(x.size)) for k, x in allocs]
        want = spec.restore(bytes(bad), bb)
        cb = [(k, np.zeros_like(x)) for k, x in allocs]
        assert corc.restore(bytes(bad), cb) == want, i
