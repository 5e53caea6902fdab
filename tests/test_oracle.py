"""Pins of the CPU oracles (plain-C oracle and Python spec oracle).

Nothing here trusts the oracle's own arithmetic: every check compares it with
something fixed elsewhere -- published CRC-32C values (golden files), the zlib
CRC-32 for the same shift-register engine with the IEEE polynomial, the SSE4.2
hardware CRC-32C instruction, the image format's field offsets read with
struct, closed-form invariants, and brute-force agreement of two independent
implementations.
"""
import itertools
import random
import struct
import zlib

import numpy as np
import pytest

from oracle import oracle as corc
from oracle import spec
from testlib import crc_collide as _collide, decode_input, golden_lines, hw_crc32c

OK, EINVAL, ECORRUPT, EMISMATCH, EBASE = 0, -1, -4, -5, -6
ZERO, DATA, UNCHANGED = 0, 1, 2
NO_CHUNK = (1 << 64) - 1


def r16(n):
    return (n + 15) & ~15


# ------------------------------------------------------------------ CRC core
@pytest.mark.parametrize("row", list(golden_lines("crc32c_vectors.txt")), ids=lambda r: r[0])
def test_crc_published_vectors(row):
    name, inp, want = row
    data = decode_input(inp)
    want = int(want, 16)
    assert spec.crc32c(data) == want
    assert corc.crc32c(data) == want
    assert hw_crc32c(data) == want     # the cross-check itself is sane


def test_crc_engine_is_zlib_crc32_with_ieee_polynomial():
    # the same shift register with the IEEE polynomial must be zlib's CRC-32:
    # pins bit order, preset and final complement of the engine
    rng = random.Random(5)
    for n in [0, 1, 2, 3, 7, 8, 9, 63, 64, 65, 300]:
        data = bytes(rng.randrange(256) for _ in range(n))
        assert spec.crc_bitwise(data, poly=0xEDB88320) == zlib.crc32(data)


def test_crc_matches_hardware_instruction():
    rng = np.random.default_rng(11)
    for n in [1, 2, 3, 4, 5, 15, 16, 17, 255, 256, 1000, 4096, 65536 + 3, 1 << 20]:
        data = rng.integers(0, 256, n, dtype=np.uint8)
        assert corc.crc32c(data) == hw_crc32c(data), n
        if n <= 1000:
            assert spec.crc32c(data.tobytes()) == hw_crc32c(data), n


def test_zero_chunk_digests():
    # CRC-32C of all-zero runs at the chunk sizes used by the workloads
    for n in [32, 16 << 10, 64 << 10, 256 << 10]:
        z = np.zeros(n, np.uint8)
        assert corc.crc32c(z) == hw_crc32c(z)
    assert corc.crc32c(np.zeros(32, np.uint8)) == 0x8A9136AA


# ------------------------------------------------------------------ golden image
def _golden_tiny():
    rows = list(golden_lines("tiny_image.txt"))
    c = int(rows[0][1])
    allocs, expect = [], []
    for r in rows[1:]:
        if r[0] == "payload_bytes":
            d = int(r[1])
            continue
        allocs.append((int(r[0]), decode_input(r[1])))
        expect.append((r[2], r[3], int(r[4], 16)))
    return c, allocs, expect, d


@pytest.mark.parametrize("impl", ["c", "spec"])
def test_golden_tiny_image(impl):
    c, allocs, expect, d = _golden_tiny()
    if impl == "c":
        rc, img = corc.dump([(i, np.frombuffer(b, np.uint8)) for i, b in allocs], c)
        img = bytes(img)
    else:
        rc, img = spec.dump(allocs, c)
    assert rc == OK
    n = len(allocs)
    (magic, ver, flags, cc, na, nc, dd, base, res, nn, tcrc, hcrc) = struct.unpack_from("<8sIIIIQQIIQII", img, 0)
    assert magic == b"MICKPT01" and ver == 1 and flags == 0 and cc == c and na == n
    assert dd == d and base == 0 and res == 0 and nn == sum(len(b) for _, b in allocs)
    kinds_expected = [e[0] for e in expect if e[0] != "-"]
    assert nc == len(kinds_expected)
    crcs = struct.unpack_from("<%dI" % nc, img, 64 + 32 * n)
    kinds = img[64 + 32 * n + 4 * nc: 64 + 32 * n + 5 * nc]
    names = {ZERO: "ZERO", DATA: "DATA", UNCHANGED: "UNCHANGED"}
    assert [names[k] for k in kinds] == kinds_expected
    assert list(crcs) == [int(e[1], 16) for e in expect if e[1] != "-"]
    for a, e in enumerate(expect):
        aid, size, first, acrc, zero = struct.unpack_from("<QQQII", img, 64 + 32 * a)
        assert acrc == e[2] and zero == 0 and aid == allocs[a][0] and size == len(allocs[a][1])


# ------------------------------------------------------------------ layout, field by field
def _random_table(rng, n, c, zero_p=0.3):
    allocs = []
    for a in range(n):
        size = int(rng.integers(0, 5 * c))
        buf = rng.integers(0, 256, size, dtype=np.uint8)
        for k in range(0, size, c):          # some chunks all-zero
            if rng.random() < zero_p:
                buf[k:k + c] = 0
        allocs.append((int(rng.integers(1, 1 << 62)), buf))
    return allocs


def test_layout_field_by_field_against_hardware_crc():
    rng = np.random.default_rng(3)
    c = 256
    allocs = _random_table(rng, 9, c)
    rc, img = corc.dump(allocs, c)
    assert rc == OK
    img = bytes(img)
    n = len(allocs)
    sizes = [b.size for _, b in allocs]
    nc = sum((s + c - 1) // c for s in sizes)
    hdr = struct.unpack_from("<8sIIIIQQIIQII", img, 0)
    assert hdr[0] == b"MICKPT01" and hdr[1] == 1 and hdr[2] == 0 and hdr[3] == c and hdr[4] == n
    assert hdr[5] == nc and hdr[9] == sum(sizes)
    assert hdr[11] == hw_crc32c(img[:60])
    tl = r16(32 * n + 5 * nc)
    assert hdr[10] == hw_crc32c(img[64:64 + tl])
    assert not any(img[64 + 32 * n + 5 * nc: 64 + tl])
    crcs = struct.unpack_from("<%dI" % nc, img, 64 + 32 * n)
    kinds = img[64 + 32 * n + 4 * nc: 64 + 32 * n + 5 * nc]
    payload = bytearray()
    g = 0
    for a, (aid, buf) in enumerate(allocs):
        rid, rsize, rfirst, racrc, rz = struct.unpack_from("<QQQII", img, 64 + 32 * a)
        assert (rid, rsize, rfirst, rz) == (aid, buf.size, g, 0)
        assert racrc == hw_crc32c(buf)
        for lo in range(0, buf.size, c):
            piece = buf[lo:lo + c]
            assert crcs[g] == hw_crc32c(piece)
            want = ZERO if not piece.any() else DATA
            assert kinds[g] == want
            if want == DATA:
                payload += piece.tobytes() + bytes(r16(piece.size) - piece.size)
            g += 1
    assert hdr[6] == len(payload)
    assert img[64 + tl:] == bytes(payload)
    # state digest = CRC32C(AllocRec || crc[])
    rc, f = corc.parse(img)
    assert rc == OK and f["state_digest"] == hw_crc32c(img[64:64 + 32 * n + 4 * nc])


# ------------------------------------------------------------------ invariants
@pytest.mark.parametrize("c", [16, 64, 1024, 65536])
def test_restore_of_dump_is_identity(c):
    rng = np.random.default_rng(c)
    allocs = _random_table(rng, 6, min(c, 4096))
    rc, img = corc.dump(allocs, c)
    assert rc == OK
    targets = [(i, np.full(b.size, 0xAB, np.uint8)) for i, b in allocs]
    rc, bad = corc.restore(img, targets)
    assert (rc, bad) == (OK, NO_CHUNK)
    for (_, b), (_, t) in zip(allocs, targets):
        assert np.array_equal(b, t)


def test_zero_elision_and_payload_size():
    rng = np.random.default_rng(7)
    c = 128
    allocs = _random_table(rng, 8, c, zero_p=0.5)
    allocs.append((999, np.zeros(3 * c + 7, np.uint8)))
    rc, img = corc.dump(allocs, c)
    rc, f = corc.parse(img)
    want = 0
    for _, b in allocs:
        for lo in range(0, b.size, c):
            piece = b[lo:lo + c]
            if piece.any():
                want += r16(piece.size)
    assert f["D"] == want
    # the all-zero allocation contributes nothing
    rc2, img2 = corc.dump(allocs[:-1], c)
    assert corc.parse(img2)[1]["D"] == want


def test_delta_of_same_state_is_empty_and_no_unchanged_without_prev():
    rng = np.random.default_rng(8)
    c = 64
    allocs = _random_table(rng, 5, c)
    rc, full = corc.dump(allocs, c)
    kinds = _kinds(full)
    assert UNCHANGED not in kinds
    rc, delta = corc.dump(allocs, c, prev=full)
    assert rc == OK
    f = corc.parse(delta)[1]
    assert f["D"] == 0 and f["flags"] == 1 and f["base_state"] == corc.parse(full)[1]["state_digest"]
    dk = _kinds(delta)
    assert all((k == ZERO) == (fk == ZERO) for k, fk in zip(dk, kinds))
    assert all(k in (ZERO, UNCHANGED) for k in dk)


def _kinds(img):
    img = bytes(img)
    n, nc = struct.unpack_from("<IQ", img, 20)
    return list(img[64 + 32 * n + 4 * nc: 64 + 32 * n + 5 * nc])


def _mutate(allocs, rng, frac=0.2, c=64):
    out = []
    for aid, b in allocs:
        x = b.copy()
        for lo in range(0, x.size, c):
            if rng.random() < frac:
                p = lo + int(rng.integers(0, min(c, x.size - lo)))
                x[p] ^= 0x5A
        out.append((aid, x))
    return out


def test_merge_of_base_and_delta_equals_full_dump():
    rng = np.random.default_rng(9)
    c = 64
    base = _random_table(rng, 7, c)
    new = _mutate(base, rng, c=c)
    new[2] = (new[2][0], np.zeros(new[2][1].size, np.uint8))   # an allocation zeroed
    new[3] = (12345, new[3][1])                               # an allocation renamed
    rc, ib = corc.dump(base, c)
    rc, idl = corc.dump(new, c, prev=ib)
    rc, ix = corc.dump(new, c)
    rc, im = corc.merge(ib, idl)
    assert rc == OK and bytes(im) == bytes(ix)
    # same through the spec
    rc, sm = spec.merge(bytes(ib), bytes(idl))
    assert rc == OK and sm == bytes(ix)


def test_in_place_delta_restore_gives_new_state():
    rng = np.random.default_rng(10)
    c = 32
    base = _random_table(rng, 6, c)
    new = _mutate(base, rng, c=c)
    rc, ib = corc.dump(base, c)
    rc, idl = corc.dump(new, c, prev=ib)
    tgt = [(i, np.zeros(b.size, np.uint8)) for i, b in base]
    assert corc.restore(ib, tgt)[0] == OK
    assert corc.restore(idl, tgt) == (OK, NO_CHUNK)
    for (_, x), (_, t) in zip(new, tgt):
        assert np.array_equal(x, t)


def test_chains_of_deltas():
    rng = np.random.default_rng(12)
    c = 64
    s0 = _random_table(rng, 4, c)
    s1 = _mutate(s0, rng, c=c)
    s2 = _mutate(s1, rng, c=c)
    _, i0 = corc.dump(s0, c)
    _, i1 = corc.dump(s1, c, prev=i0)
    _, i2 = corc.dump(s2, c, prev=i1)      # compares against i1's full digest table
    _, i2full = corc.dump(s2, c)
    _, m1 = corc.merge(i0, i1)
    rc, m2 = corc.merge(m1, i2)
    assert rc == OK and bytes(m2) == bytes(i2full)


# ------------------------------------------------------------------ error paths
def test_error_paths():
    rng = np.random.default_rng(13)
    c = 64
    allocs = _random_table(rng, 4, c, zero_p=0.0)
    allocs = [(i, b if b.size else np.ones(10, np.uint8)) for i, b in allocs]
    rc, img = corc.dump(allocs, c)
    img = bytes(img)
    tgt = lambda: [(i, np.zeros(b.size, np.uint8)) for i, b in allocs]
    # invalid arguments
    assert corc.dump(allocs, 48)[0] == EINVAL
    assert corc.dump(allocs + [allocs[0]], c)[0] == EINVAL
    # header, tables, truncation
    for pos in [0, 9, 20, 33, 59, 61]:
        bad = bytearray(img); bad[pos] ^= 1
        assert corc.restore(bytes(bad), tgt()) == (ECORRUPT, NO_CHUNK)
    n = len(allocs)
    bad = bytearray(img); bad[64 + 32 * n + 1] ^= 0x10
    assert corc.restore(bytes(bad), tgt())[0] == ECORRUPT
    assert corc.restore(img[:-1], tgt())[0] == ECORRUPT
    # payload byte flipped -> the chunk holding it
    nc = corc.parse(img)[1]["n_chunks"]
    tl = r16(32 * n + 5 * nc)
    bad = bytearray(img); bad[64 + tl + 3 * 64 + 5] ^= 0x80
    assert corc.restore(bytes(bad), tgt()) == (ECORRUPT, 3)
    # table mismatch
    t = tgt(); t[1] = (t[1][0] + 1, t[1][1])
    assert corc.restore(img, t)[0] == EMISMATCH
    t = tgt(); t[1] = (t[1][0], np.zeros(t[1][1].size + 1, np.uint8))
    assert corc.restore(img, t)[0] == EMISMATCH
    assert corc.restore(img, tgt()[:-1])[0] == EMISMATCH
    # delta over a target that does not hold the base
    new = _mutate(allocs, rng, frac=0.3, c=c)
    _, dl = corc.dump(new, c, prev=img)
    wrong = tgt()
    rc, bad_chunk = corc.restore(dl, wrong)
    kinds = _kinds(dl)
    assert rc == EBASE and bad_chunk == kinds.index(UNCHANGED)
    # merge against the wrong base
    _, other = corc.dump(_mutate(allocs, rng, frac=0.5, c=c), c)
    assert corc.merge(other, dl)[0] == EBASE
    assert corc.merge(dl, dl)[0] == EINVAL
    assert corc.merge(img, img)[0] == EINVAL


def test_spec_and_c_error_codes_agree():
    rng = np.random.default_rng(14)
    c = 16
    allocs = _random_table(rng, 3, c, zero_p=0.2)
    _, img = corc.dump(allocs, c)
    img = bytes(img)
    for pos in range(len(img)):
        bad = bytearray(img); bad[pos] ^= 0x04
        t1 = [(i, np.zeros(b.size, np.uint8)) for i, b in allocs]
        t2 = [(i, bytearray(b.size)) for i, b in allocs]
        assert corc.restore(bytes(bad), t1) == spec.restore(bytes(bad), t2), pos


# ------------------------------------------------------------------ forced collision
def test_forced_crc_collision_is_unchanged_in_both_oracles():
    c = 64
    rng = np.random.default_rng(15)
    base = rng.integers(0, 256, 3 * c, dtype=np.uint8)
    new = base.copy()
    new[c + 10] ^= 0xFF                              # modify chunk 1
    patched = _collide(base[c:2 * c].tobytes(), new[c:2 * c].tobytes(), 20)
    new[c:2 * c] = np.frombuffer(patched, np.uint8)
    assert not np.array_equal(new[c:2 * c], base[c:2 * c])
    assert hw_crc32c(new[c:2 * c]) == hw_crc32c(base[c:2 * c])
    _, ib = corc.dump([(1, base)], c)
    _, idl = corc.dump([(1, new)], c, prev=ib)
    assert _kinds(idl) == [UNCHANGED, UNCHANGED, UNCHANGED]
    rc, sdl = spec.dump([(1, new.tobytes())], c, prev=bytes(ib))
    assert rc == OK and sdl == bytes(idl)


# ------------------------------------------------------------------ brute force
def _contents(kind, size, rng):
    if kind == "zero":
        return bytes(size)
    if kind == "random":
        return bytes(rng.randrange(256) for _ in range(size))
    b = bytearray(size)
    if size:
        b[0 if kind == "first" else size - 1] = 1 + rng.randrange(255)
    return bytes(b)


def _variants(allocs, prevkind, rng):
    """The previous state for a brute-force case."""
    if prevkind == "same":
        return allocs
    if prevkind == "byte":
        out = []
        for aid, b in allocs:
            b = bytearray(b)
            if b:
                b[rng.randrange(len(b))] ^= 0x01
            out.append((aid, bytes(b)))
        return out
    if prevkind == "resized":
        return [(aid, b + b"\x07") for aid, b in allocs]
    if prevkind == "renamed":
        return [(aid + 1000, b) for aid, b in allocs]
    raise ValueError(prevkind)


def test_bruteforce_single_allocation_spec_equals_c():
    rng = random.Random(16)
    for c in (16, 32, 64):
        sizes = sorted({0, 1, 15, 16, 17, c - 1, c, c + 1, 2 * c, 2 * c + 5})
        for size, kind, prevkind in itertools.product(sizes, ["zero", "random", "first", "last"],
                                                      [None, "same", "byte", "resized", "renamed"]):
            allocs = [(3, _contents(kind, size, rng))]
            _check_case(allocs, c, prevkind, rng)


def test_bruteforce_multi_allocation_spec_equals_c():
    rng = random.Random(17)
    for trial in range(150):
        c = rng.choice((16, 32, 64))
        sizes = [0, 1, 15, 16, 17, c - 1, c, c + 1, 2 * c, 2 * c + 5]
        n = rng.randint(1, 3)
        allocs = [(10 + a, _contents(rng.choice(["zero", "random", "first", "last"]),
                                     rng.choice(sizes), rng)) for a in range(n)]
        _check_case(allocs, c, rng.choice([None, "same", "byte", "resized", "renamed"]), rng)


def _check_case(allocs, c, prevkind, rng):
    prev_s = prev_c = None
    if prevkind is not None:
        pa = _variants(allocs, prevkind, rng)
        rc, prev_s = spec.dump(pa, c)
        rc2, prev_c = corc.dump([(i, np.frombuffer(b, np.uint8)) for i, b in pa], c)
        assert rc == rc2 == OK and prev_s == bytes(prev_c)
    rc, img_s = spec.dump(allocs, c, prev=prev_s)
    rc2, img_c = corc.dump([(i, np.frombuffer(b, np.uint8)) for i, b in allocs], c, prev=prev_c)
    assert rc == rc2 == OK
    assert img_s == bytes(img_c)
    # both restores: a full image onto garbage, a delta onto its base
    if prevkind is None:
        t_s = [(i, bytearray(b"\xee" * len(b))) for i, b in allocs]
        t_c = [(i, np.full(len(b), 0xEE, np.uint8)) for i, b in allocs]
    else:
        pa = _variants(allocs, prevkind, rng) if prevkind in ("same", "resized", "renamed") else None
        if pa is None:
            return
        if prevkind in ("resized", "renamed"):
            return
        t_s = [(i, bytearray(b)) for i, b in pa]
        t_c = [(i, np.frombuffer(b, np.uint8).copy()) for i, b in pa]
    r1 = spec.restore(img_s, t_s)
    r2 = corc.restore(img_c, t_c)
    assert r1 == r2 == (OK, NO_CHUNK)
    for (_, b), (_, t1), (_, t2) in zip(allocs, t_s, t_c):
        assert bytes(t1) == b and t2.tobytes() == b


# ------------------------------------------------------------------ planted mistakes
PLANTED = {
    "no_final_complement": lambda d: spec.crc_bitwise(d, xorout=0),
    "zero_preset": lambda d: spec.crc_bitwise(d, init=0),
    "wrong_polynomial": lambda d: spec.crc_bitwise(d, poly=0xEDB88320),
    "byte_order_swapped": lambda d: spec.crc_bitwise(d[::-1]),
}


@pytest.mark.parametrize("name", sorted(PLANTED))
def test_planted_crc_mistake_is_caught_by_golden_vectors(name, monkeypatch):
    monkeypatch.setattr(spec, "crc32c", PLANTED[name])
    caught = False
    for _, inp, want in golden_lines("crc32c_vectors.txt"):
        if spec.crc32c(decode_input(inp)) != int(want, 16):
            caught = True
    assert caught


def test_planted_kind_precedence_mistake_is_caught():
    # swapping ZERO/UNCHANGED precedence changes the kinds of an all-zero chunk
    # of a delta against a zero base; the merge invariant then still holds but
    # the zero-elision invariant (ZERO chunks have no payload and need no base)
    # is what pins it: a delta of a zero state must restore onto ANY target.
    c = 16
    z = [(1, bytes(2 * c))]
    rc, base = spec.dump(z, c)
    rc, dl = spec.dump(z, c, prev=base)
    assert spec.parse(dl)[1]["kinds"] == [ZERO, ZERO]
    t = [(1, bytearray(b"\x01" * (2 * c)))]
    assert spec.restore(dl, t) == (OK, NO_CHUNK) and bytes(t[0][1]) == bytes(2 * c)
