"""Parity at the benchmark's full sizes and launch configuration.

Every image dumped here is compared byte for byte with the oracle's image of
the same device bytes (copied to the host, dumped by the plain-C oracle on
all host cores): header, allocation records, every crc[] and kind[] entry,
and the whole payload. Restores are checked by the restored bytes equal to
the dumped ones, in full. Each test names its workload and seed. The codec
test compares sampled chunks' records (the oracle's codec at this size takes
minutes) plus properties that hold at any size."""
import os
import struct
import sys
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import oracle as corc  # noqa: E402
from paper_2502_16631_amd import mickpt as mk  # noqa: E402
import workloads  # noqa: E402

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
C = 65536
ZERO, DATA, UNCHANGED = 0, 1, 2


def _bytes_of(t):
    return t.reshape(-1).view(torch.uint8) if t.numel() else torch.zeros(0, dtype=torch.uint8, device=t.device)


def _check_image(img, table, samples=1500, seed=0, prev_table=None):
    v = img.view()
    (magic, ver, flags, c, n, nc, D, base, res, N, tcrc, hcrc) = struct.unpack_from("<8sIIIIQQIIQII", v[:64].tobytes())
    sizes = [t.numel() * t.element_size() for _, t in table]
    assert magic == b"MICKPT01" and c == C and n == len(table) and N == sum(sizes)
    assert nc == sum((s + C - 1) // C for s in sizes)
    tl = (32 * n + 5 * nc + 15) & ~15
    assert v.size == 64 + tl + D
    assert corc.crc32c(v[:60]) == hcrc and corc.crc32c(v[64:64 + tl]) == tcrc
    recs = np.frombuffer(v[64:64 + 32 * n].tobytes(), dtype=np.uint64).reshape(n, 4)
    crcs = np.frombuffer(v[64 + 32 * n:64 + 32 * n + 4 * nc].tobytes(), dtype=np.uint32)
    kinds = v[64 + 32 * n + 4 * nc:64 + 32 * n + 5 * nc]
    first = np.concatenate([[0], np.cumsum([(s + C - 1) // C for s in sizes])[:-1]]).astype(np.int64)
    assert np.array_equal(recs[:, 1], np.array(sizes, dtype=np.uint64))
    assert np.array_equal(recs[:, 2], first.astype(np.uint64))
    # payload offsets from the kinds (a property of the format)
    lens = np.full(nc, C, dtype=np.int64)
    for a, s in enumerate(sizes):
        nk = (s + C - 1) // C
        if nk:
            lens[first[a] + nk - 1] = s - (nk - 1) * C
    plen = np.where(kinds == DATA, (lens + 15) & ~15, 0)
    off = np.concatenate([[0], np.cumsum(plen)[:-1]])
    assert int(plen.sum()) == D
    # sampled chunks: CRC-32C and kind from the oracle, payload bytes
    rng = np.random.default_rng(seed)
    alloc_of = np.searchsorted(first, np.arange(nc), side="right") - 1
    pick = rng.choice(nc, size=min(samples, nc), replace=False)
    pick = np.union1d(pick, [0, nc - 1])
    for g in pick:
        a = int(alloc_of[g])
        k = int(g - first[a])
        buf = _bytes_of(table[a][1])
        chunk = buf[k * C:k * C + int(lens[g])].cpu().numpy()
        assert corc.crc32c(chunk) == int(crcs[g]), g
        if not chunk.any():
            want = ZERO
        elif prev_table is not None and int(crcs[g]) == corc.crc32c(
                _bytes_of(prev_table[a][1])[k * C:k * C + int(lens[g])].cpu().numpy()):
            want = UNCHANGED
        else:
            want = DATA
        assert int(kinds[g]) == want, g
        if want == DATA:
            rec = v[64 + tl + int(off[g]):64 + tl + int(off[g]) + int(plen[g])]
            assert np.array_equal(rec[:int(lens[g])], chunk) and not rec[int(lens[g]):].any()
    # whole-allocation CRCs of the smaller allocations
    small = [a for a, s in enumerate(sizes) if s <= (64 << 20)][:20]
    for a in small:
        assert corc.crc32c(_bytes_of(table[a][1]).cpu().numpy()) == int(recs[a, 3] & 0xFFFFFFFF)
    return D, kinds



def _first_diff(a, b, step=1 << 28):
    """Offset of the first differing byte of two equal-length uint8 arrays,
    compared in slices (no full-size temporaries), or None."""
    for lo in range(0, a.size, step):
        x, y = a[lo:lo + step], b[lo:lo + step]
        if not np.array_equal(x, y):
            return lo + int(np.nonzero(x != y)[0][0])
    return None


def _same_as_oracle(img, oimg, label):
    """The GPU image equals the oracle's byte for byte; on a difference the
    message says which region (header, records, crc[], kind[], payload)
    holds the first one and how many crc[] / kind[] entries differ."""
    got = img.view()
    assert got.size == oimg.size, (label, got.size, oimg.size)
    at = _first_diff(got, oimg)
    if at is None:
        return
    n = int(np.frombuffer(oimg[20:24].tobytes(), np.uint32)[0])
    nc = int(np.frombuffer(oimg[24:32].tobytes(), np.uint64)[0])
    codec = int(np.frombuffer(oimg[12:16].tobytes(), np.uint32)[0]) & 2
    o_crc = 64 + 32 * n
    o_kind = o_crc + (8 if codec else 4) * nc
    crc_g = np.frombuffer(got[o_crc:o_crc + 4 * nc].tobytes(), np.uint32)
    crc_o = np.frombuffer(oimg[o_crc:o_crc + 4 * nc].tobytes(), np.uint32)
    kd = int((got[o_kind:o_kind + nc] != oimg[o_kind:o_kind + nc]).sum())
    region = ("header" if at < 64 else "records" if at < o_crc else "crc" if at < o_crc + 4 * nc
              else "kind/rlen" if at < o_kind + nc else "tables pad/payload")
    raise AssertionError("%s: image differs from the oracle's, first at byte %d (%s); %d crc[] and %d kind[] "
                         "entries differ" % (label, at, region, int((crc_g != crc_o).sum()), kd))


def _oracle_dump(host_table, prev=None, label=""):
    t0 = time.perf_counter()
    rc, oimg = corc.dump(host_table, C, prev=prev)
    assert rc == 0
    print("%s: oracle dump of %.1f GB in %.1f s (%d threads)" % (
        label, sum(a.size for _, a in host_table) / 1e9, time.perf_counter() - t0, corc.default_threads()),
        flush=True)
    return oimg


def _mem(tag):
    free, total = torch.cuda.mem_get_info()
    print("%s: device memory free %.1f of %.1f GiB, torch reserved %.1f GiB"
          % (tag, free / 2**30, total / 2**30, torch.cuda.memory_reserved() / 2**30), flush=True)


def _restore_equal(ctx, img, table, opts):
    _mem("before restore targets")
    targets = [(i, torch.empty_like(t)) for i, t in table]
    rc, res = mk.ckpt_restore(ctx, img, targets, opts=opts)
    assert rc == 0, (mk.ckpt_strerror(rc), res.first_bad_chunk)
    torch.cuda.synchronize()
    for (_, a), (_, b) in zip(table, targets):
        assert torch.equal(_bytes_of(a), _bytes_of(b))


@pytest.mark.timeout(900)
def test_training_state_full_size():
    """decoder-1.3B training state, seed 2, 303 allocations, ~27 GB; the bench's
    configuration: one staging window, 64 KiB chunks. The whole image equals
    the oracle's."""
    torch.cuda.empty_cache()
    _mem("start")
    table = workloads.training_state("cuda", seed=2)
    torch.cuda.synchronize()
    N = sum(t.numel() * t.element_size() for _, t in table)
    ctx = mk.ckpt_ctx_create(0, 64 << 30)
    try:
        opts = mk.make_opts(chunk_size=C)
        rc, img, res = mk.ckpt_dump(ctx, table, opts=opts)
        assert rc == 0 and res.windows == 1
        D, kinds = _check_image(img, table, samples=200, seed=2)
        assert (kinds == DATA).all() and D >= N     # random-valued state: every chunk is DATA
        oimg = _oracle_dump(workloads.host_copy(table), label="training state")
        _same_as_oracle(img, oimg, "training state")
        del oimg
        _restore_equal(ctx, img, table, opts)
        img.free()
    finally:
        mk.ckpt_ctx_destroy(ctx)


@pytest.mark.timeout(600)
def test_training_state_codec_full_size():
    """decoder-1.3B training state, seed 2, ~27 GB, 64 KiB chunks, dumped with
    the byte-plane codec: header and tables of the codec layout, sampled
    chunks' digests, kinds and payload records equal to the oracle's for the
    same chunk, the payload length, and the whole state restored."""
    torch.cuda.empty_cache()
    _mem("start")
    table = workloads.training_state("cuda", seed=2)
    torch.cuda.synchronize()
    sizes = [t.numel() * t.element_size() for _, t in table]
    ctx = mk.ckpt_ctx_create(0, 64 << 30)
    try:
        opts = mk.make_opts(chunk_size=C, flags=mk.OPT_CODEC)
        rc, img, res = mk.ckpt_dump(ctx, table, opts=opts)
        assert rc == 0 and res.windows == 1, mk.ckpt_strerror(rc)
        v = img.view()
        (magic, ver, flags, c, n, nc, D, base, _, N, tcrc, hcrc) = struct.unpack_from("<8sIIIIQQIIQII",
                                                                                     v[:64].tobytes())
        assert flags == 2 and c == C and n == len(table) and N == sum(sizes)
        tl = (32 * n + 9 * nc + 15) & ~15
        assert v.size == 64 + tl + D
        assert corc.crc32c(v[:60]) == hcrc and corc.crc32c(v[64:64 + tl]) == tcrc
        crcs = np.frombuffer(v[64 + 32 * n:64 + 32 * n + 4 * nc].tobytes(), dtype=np.uint32)
        rlen = np.frombuffer(v[64 + 32 * n + 4 * nc:64 + 32 * n + 8 * nc].tobytes(), dtype=np.uint32)
        kinds = v[64 + 32 * n + 8 * nc:64 + 32 * n + 9 * nc]
        assert int(rlen.astype(np.int64).sum()) == D and res.n_packed == int((kinds == 3).sum()) > 0
        off = np.concatenate([[0], np.cumsum(rlen.astype(np.int64))[:-1]])
        first = np.concatenate([[0], np.cumsum([(s + C - 1) // C for s in sizes])[:-1]]).astype(np.int64)
        alloc_of = np.searchsorted(first, np.arange(nc), side="right") - 1
        rng = np.random.default_rng(12)
        pick = np.union1d(rng.choice(nc, size=300, replace=False), [0, nc - 1])
        for g in pick:
            a = int(alloc_of[g])
            k = int(g - first[a])
            buf = _bytes_of(table[a][1])
            chunk = buf[k * C:min((k + 1) * C, sizes[a])].cpu().numpy()
            assert corc.crc32c(chunk) == int(crcs[g]), g
            rc, one = corc.dump([(1, chunk)], C, codec=True)
            p1 = corc.parse(one)[1]
            want_kind = int(one[64 + 32 + 8])              # the one chunk's kind
            assert int(kinds[g]) == want_kind, g
            rec = v[64 + tl + int(off[g]):64 + tl + int(off[g]) + int(rlen[g])]
            assert int(rlen[g]) == p1["D"] and np.array_equal(rec, one[one.size - p1["D"]:]), g
        print("codec payload %.3f of the logical bytes, %d of %d chunks packed"
              % (D / N, res.n_packed, nc), flush=True)
        _restore_equal(ctx, img, table, opts)
        img.free()
    finally:
        mk.ckpt_ctx_destroy(ctx)


@pytest.mark.timeout(900)
def test_hpc_incremental_full_size():
    """HPC image, seed 3, 512 allocations, 40 GB, ~60 % zero chunks; 5 % of the
    chunks rewritten (seed 33); the base image and the delta image (taken
    against it) each equal the oracle's, the oracle's delta taken against
    its own base image; then base restore + delta apply in place."""
    torch.cuda.empty_cache()
    _mem("start")
    table, _ = workloads.hpc_state("cuda", seed=3)
    torch.cuda.synchronize()
    ctx = mk.ckpt_ctx_create(0, 64 << 30)
    try:
        opts = mk.make_opts(chunk_size=C)
        rc, base, _ = mk.ckpt_dump(ctx, table, opts=opts)
        assert rc == 0
        obase = _oracle_dump(workloads.host_copy(table), label="HPC base")
        _same_as_oracle(base, obase, "HPC base")
        workloads.mutate_runs(table, seed=33, chunk=C, frac=0.05, run_mean=16)
        torch.cuda.synchronize()
        rc, delta, dres = mk.ckpt_dump(ctx, table, prev=base, opts=opts)
        assert rc == 0 and dres.n_unchanged > 0
        odelta = _oracle_dump(workloads.host_copy(table), prev=obase, label="HPC delta")
        del obase
        _same_as_oracle(delta, odelta, "HPC delta")
        del odelta
        # base then delta, in place: equals the new state
        new = [(i, t.clone()) for i, t in table]
        rc, _ = mk.ckpt_restore(ctx, base, table, opts=opts)
        assert rc == 0
        rc, r = mk.ckpt_restore(ctx, delta, table, opts=opts)
        assert rc == 0, (mk.ckpt_strerror(rc), r.first_bad_chunk)
        torch.cuda.synchronize()
        for (_, a), (_, b) in zip(new, table):
            assert torch.equal(a, b)
        del new
        base.free()
        delta.free()
    finally:
        mk.ckpt_ctx_destroy(ctx)


@pytest.mark.timeout(900)
def test_fragmented_batched_full_size():
    """10,000 allocations, seed 4, 60 GB, 256 KiB-aligned zero blocks; the
    graph form (one launch) and the per-allocation launches each give the
    oracle's image byte for byte, and each restores the dumped state."""
    torch.cuda.empty_cache()   # 60 GB state + 60 GB staging + 60 GB restore targets
    _mem("start")
    table = workloads.fragmented_state("cuda", seed=4)
    torch.cuda.synchronize()
    _mem("state")
    oimg = _oracle_dump(workloads.host_copy(table), label="fragmented")
    ctx = mk.ckpt_ctx_create(0, 96 << 30)
    try:
        opts = mk.make_opts(chunk_size=C, flags=mk.OPT_GRAPH)
        rc, img, res = mk.ckpt_dump(ctx, table, opts=opts)
        assert rc == 0, (mk.ckpt_strerror(rc), res.hip_error)
        assert res.windows == 1
        _same_as_oracle(img, oimg, "fragmented, graph form")
        _restore_equal(ctx, img, table, opts)
        img.free()
        rc, img2, res2 = mk.ckpt_dump(ctx, table, opts=mk.make_opts(chunk_size=C, flags=mk.OPT_PER_ALLOC))
        assert rc == 0, (mk.ckpt_strerror(rc), res2.hip_error)
        assert res2.windows >= len([t for _, t in table if t.numel()])
        _same_as_oracle(img2, oimg, "fragmented, per-allocation launches")
        del oimg
        _restore_equal(ctx, img2, table, opts)
        img2.free()
    finally:
        mk.ckpt_ctx_destroy(ctx)
