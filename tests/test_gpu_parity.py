"""GPU parity: images from the HIP path are byte-identical to the CPU
oracle's, and restores write back exactly the dumped bytes. Tolerance is
0 bytes (integer / byte work). Every call goes through the C ABI."""
import os
import random
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import oracle as corc  # noqa: E402
from paper_2502_16631_amd import mickpt as mk  # noqa: E402
import workloads  # noqa: E402
from testlib import crc_collide  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda"
ZERO, DATA, UNCHANGED = 0, 1, 2


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = mk.ckpt_ctx_create(0, 1 << 30)
    yield c
    mk.ckpt_ctx_destroy(c)


def host(table):
    return workloads.host_copy(table)


def gpu_dump(ctx, table, prev=None, **kw):
    rc, img, res = mk.ckpt_dump(ctx, table, prev=prev, opts=mk.make_opts(**kw))
    assert rc == 0, mk.ckpt_strerror(rc)
    return img, res


def check_parity(ctx, table, c, prev_gpu=None, prev_oracle=None, **kw):
    img, res = gpu_dump(ctx, table, prev=prev_gpu, chunk_size=c, **kw)
    rc, oimg = corc.dump(host(table), c, prev=prev_oracle)
    assert rc == 0
    got = img.view()
    assert got.size == oimg.size, (got.size, oimg.size)
    if not np.array_equal(got, oimg):
        diff = np.nonzero(got != oimg)[0]
        raise AssertionError("image differs at %d bytes, first at %d" % (diff.size, diff[0]))
    # the reported kind counts are those of the oracle's kind table
    # (plain layout: header, AllocRec[n], crc[n_c], kind[n_c])
    _, hdr = corc.parse(oimg)
    n, nc = hdr["n_allocs"], hdr["n_chunks"]
    kinds = oimg[64 + 32 * n + 4 * nc:64 + 32 * n + 5 * nc]
    want = tuple(int((kinds == k).sum()) for k in (ZERO, DATA, UNCHANGED, 3))
    assert (res.n_zero, res.n_data, res.n_unchanged, res.n_packed) == want
    return img, oimg, res


def restore_and_compare(ctx, img, table, **kw):
    targets = [(i, torch.full_like(t, 0x5A) if t.numel() else t.clone()) for i, t in table]
    rc, res = mk.ckpt_restore(ctx, img, targets, opts=mk.make_opts(**kw))
    assert rc == 0, (mk.ckpt_strerror(rc), res.first_bad_chunk)
    torch.cuda.synchronize()
    for (_, a), (_, b) in zip(table, targets):
        assert torch.equal(a, b)
    return res


def test_tiny_image_full_dump_restore(ctx):
    """8 allocations log-uniform in [4 KiB, 4 MiB], 16 MiB, random bytes, 64 KiB chunks."""
    table = workloads.tiny_image(DEV, seed=1)
    img, oimg, res = check_parity(ctx, table, 65536)
    assert res.n_unchanged == 0 and res.n_payload == corc.parse(oimg)[1]["D"]
    restore_and_compare(ctx, img, table)


def _rand_table(rng, gen, n, c, zero_p=0.3, max_chunks=5):
    sizes, table = [], []
    for a in range(n):
        size = int(rng.integers(0, max_chunks * c + 1))
        if rng.random() < 0.2:
            size = int(rng.choice([0, 1, 15, 16, 17, c - 1, c, c + 1, 2 * c, 2 * c + 5]))
        size = max(size, 0)
        t = torch.randint(0, 256, (size,), dtype=torch.uint8, device=DEV, generator=gen)
        for lo in range(0, size, c):
            if rng.random() < zero_p:
                t[lo:lo + c] = 0
        table.append((int(rng.integers(1, 1 << 62)), t))
    return table


@pytest.mark.parametrize("c", [1024, 2048, 4096, 16384, 32768, 65536, 131072, 262144])
def test_chunk_sizes_ragged_tables(ctx, c):
    rng = np.random.default_rng(c)
    gen = torch.Generator(device=DEV).manual_seed(c)
    table = _rand_table(rng, gen, 12, c)
    img, _, _ = check_parity(ctx, table, c)
    restore_and_compare(ctx, img, table)


@pytest.mark.parametrize("c", [16, 32, 64, 128, 256, 512])
def test_bruteforce_tiny_chunk_sizes(ctx, c):
    """Sizes around the chunk edges, contents zero / random / single byte,
    previous image none / same / one byte changed / resized / renamed. The
    previous image is dumped by both sides and must be identical; each side
    then takes the delta against its own previous image. Every image is
    restored: a full one into scratch targets, a delta in place over the
    previous state (resized / renamed previous states share no allocation
    with the new table, so such a delta holds no UNCHANGED chunk and is
    restored into scratch targets)."""
    rng = random.Random(c)
    gen = torch.Generator(device=DEV).manual_seed(c)
    sizes = sorted({0, 1, 15, 16, 17, c - 1, c, c + 1, 2 * c, 2 * c + 5})
    for trial in range(40):
        n = rng.randint(1, 3)
        table = []
        for a in range(n):
            size = rng.choice(sizes)
            kind = rng.choice(["zero", "random", "first", "last"])
            t = torch.zeros(size, dtype=torch.uint8, device=DEV)
            if kind == "random" and size:
                t = torch.randint(0, 256, (size,), dtype=torch.uint8, device=DEV, generator=gen)
            elif kind in ("first", "last") and size:
                t[0 if kind == "first" else size - 1] = rng.randint(1, 255)
            table.append((10 + a, t))
        pk = rng.choice([None, "same", "byte", "resized", "renamed"])
        prev_g = prev_o = pt = None
        if pk is not None:
            pt = []
            for aid, t in table:
                x = t.clone()
                if pk == "byte" and x.numel():
                    x[rng.randrange(x.numel())] ^= 1
                if pk == "resized":
                    x = torch.cat([x, torch.tensor([7], dtype=torch.uint8, device=DEV)])
                pt.append((aid + (1000 if pk == "renamed" else 0), x))
            prev_g, prev_o, _ = check_parity(ctx, pt, c)
        img, oimg, res = check_parity(ctx, table, c, prev_gpu=prev_g, prev_oracle=prev_o)
        if pk in ("same", "byte"):
            # base restored, then the delta applied in place
            targets = [(i, torch.full_like(t, 0x5A) if t.numel() else t.clone()) for i, t in table]
            rc, r = mk.ckpt_restore(ctx, prev_g, targets)
            assert rc == 0, (mk.ckpt_strerror(rc), r.first_bad_chunk)
            rc, r = mk.ckpt_restore(ctx, img, targets)
            assert rc == 0, (mk.ckpt_strerror(rc), r.first_bad_chunk)
            torch.cuda.synchronize()
            for (_, a), (_, b) in zip(table, targets):
                assert torch.equal(a, b), (trial, pk)
            # the oracle applies its delta the same way
            host_t = [(i, x.copy()) for i, x in host(pt)]
            assert corc.restore(prev_o, host_t)[0] == 0
            assert corc.restore(oimg, host_t)[0] == 0
            for (_, a), (_, b) in zip(host(table), host_t):
                assert np.array_equal(a, b)
        else:
            assert res.n_unchanged == 0
            restore_and_compare(ctx, img, table)
        for x in (img, prev_g):
            if x is not None:
                x.free()


@pytest.mark.parametrize("c,kw", [(64, {}), (65536, {}), (65536, {"window_bytes": 4 * 65536}),
                                  (65536, {"flags": mk.OPT_GRAPH}), (16384, {"flags": mk.OPT_PER_ALLOC})])
def test_forced_crc_collision_is_unchanged(ctx, c, kw):
    """A chunk rewritten and then patched in 4 bytes so that its CRC-32C equals
    the base's (solved over GF(2) with the hardware CRC) is UNCHANGED in the
    delta of both the GPU path and the oracle (digest equality is the
    unchanged test); every launch form (two-pass delta in one window,
    single-pass delta over several windows, graph, per-allocation) agrees
    with the oracle byte for byte."""
    rng = np.random.default_rng(c + 7)
    base = [(5, rng.integers(0, 256, 3 * c + 100, dtype=np.uint8)), (6, rng.integers(0, 256, 2 * c, dtype=np.uint8))]
    new = [(i, a.copy()) for i, a in base]
    a1 = new[0][1]
    a1[c + 10] ^= 0xFF                                  # chunk 1 of allocation 5
    patched = crc_collide(base[0][1][c:2 * c].tobytes(), a1[c:2 * c].tobytes(), 20)
    a1[c:2 * c] = np.frombuffer(patched, np.uint8)
    assert not np.array_equal(a1[c:2 * c], base[0][1][c:2 * c])
    new[1][1][5] ^= 1                                   # an ordinary change in allocation 6
    dev_base = [(i, torch.from_numpy(a).to(DEV)) for i, a in base]
    dev_new = [(i, torch.from_numpy(a).to(DEV)) for i, a in new]
    prev_g, prev_o, _ = check_parity(ctx, dev_base, c, **kw)
    img, oimg, res = check_parity(ctx, dev_new, c, prev_gpu=prev_g, prev_oracle=prev_o, **kw)
    kinds = corc_kinds(oimg)
    g6 = -(-(3 * c + 100) // c)                         # first chunk of allocation 6
    assert kinds[1] == UNCHANGED and kinds[g6] == DATA and res.n_unchanged == len(kinds) - 1
    prev_g.free()
    img.free()


def corc_kinds(image):
    """Kind table of a plain-layout image (header fields at their documented
    offsets)."""
    n = int(np.frombuffer(image[20:24].tobytes(), np.uint32)[0])
    nc = int(np.frombuffer(image[24:32].tobytes(), np.uint64)[0])
    o = 64 + 32 * n + 4 * nc
    return [int(x) for x in image[o:o + nc]]


def test_windows_slots_streams_and_shapes_do_not_change_the_image(ctx):
    rng = np.random.default_rng(21)
    gen = torch.Generator(device=DEV).manual_seed(21)
    c = 65536
    table = _rand_table(rng, gen, 20, c, max_chunks=40)
    ref, oimg, _ = check_parity(ctx, table, c)
    variants = [dict(window_bytes=4 * c), dict(window_bytes=c, slots=2), dict(copy_streams=1),
                dict(copy_streams=4, window_bytes=8 * c), dict(flags=mk.OPT_PER_ALLOC),
                dict(wg_threads=1024), dict(wg_threads=256), dict(wg_threads=64)]
    for kw in variants:
        img, _, _ = check_parity(ctx, table, c, **kw)
        restore_and_compare(ctx, img, table, **kw)


def test_large_one_window_dump_and_corrupt_restore(ctx):
    """A ~577 MB table held by one staging window (thousands of work-groups'
    worth of chunks, allocations that end mid-chunk, zero regions, an empty
    allocation): the image is the oracle's at two chunk sizes and restores;
    a flipped byte near the end of the payload gives the oracle's code and
    first bad chunk."""
    gen = torch.Generator(device=DEV).manual_seed(61)
    a = torch.randint(0, 256, ((300 << 20) + 4097,), dtype=torch.uint8, device=DEV, generator=gen)
    a[(5 << 20):(25 << 20)] = 0
    b = torch.randint(0, 256, ((250 << 20) + 33,), dtype=torch.uint8, device=DEV, generator=gen)
    b[:(64 << 20)] = 0
    s = torch.randint(0, 256, (999,), dtype=torch.uint8, device=DEV, generator=gen)
    table = [(1, a), (2, torch.zeros(0, dtype=torch.uint8, device=DEV)), (3, b), (4, s)]
    for c in (65536, 16384):
        img, oimg, res = check_parity(ctx, table, c)
        assert res.windows == 1
        restore_and_compare(ctx, img, table)
        img.free()
    bad = oimg.copy()
    bad[bad.size - 5000] ^= 0x10
    want = corc.restore(bad, [(i, np.zeros(t.numel(), np.uint8)) for i, t in table])
    rc, bimg = mk.ckpt_image_import(bad)
    assert rc == 0
    rc, rres = mk.ckpt_restore(ctx, bimg, [(i, torch.zeros_like(t)) for i, t in table])
    assert (rc, rres.first_bad_chunk) == want and rc == mk.CKPT_ECORRUPT
    bimg.free()


def test_graph_replays_and_per_allocation_launches(ctx):
    """Batched form: the captured graph is replayed on new contents of the same
    table; the per-allocation launch baseline gives the same image."""
    c = 65536
    rng = np.random.default_rng(26)
    gen = torch.Generator(device=DEV).manual_seed(26)
    table = _rand_table(rng, gen, 40, c, max_chunks=6)
    prev_g = prev_o = None
    for rep in range(4):
        if rep:
            workloads.mutate_runs(table, seed=27 + rep, chunk=c, frac=0.2, run_mean=2)
        img, oimg, _ = check_parity(ctx, table, c, prev_gpu=prev_g if rep == 3 else None,
                                    prev_oracle=prev_o if rep == 3 else None, flags=mk.OPT_GRAPH)
        prev_g, prev_o = img, oimg
    check_parity(ctx, table, c, flags=mk.OPT_PER_ALLOC)


def test_autotuned_options_give_the_oracle_image(ctx):
    c_rng = np.random.default_rng(28)
    gen = torch.Generator(device=DEV).manual_seed(28)
    table = _rand_table(c_rng, gen, 30, 65536, max_chunks=12)
    rc, best, gbps = mk.ckpt_autotune(ctx, table, sample_bytes=8 << 20)
    assert rc == 0 and best.chunk_size in (16384, 65536, 262144) and gbps > 0
    check_parity(ctx, table, best.chunk_size, wg_threads=best.wg_threads, copy_streams=best.copy_streams)
    rc2, best2, _ = mk.ckpt_autotune(ctx, table, sample_bytes=8 << 20)     # cached
    assert rc2 == 0 and best2.chunk_size == best.chunk_size


def test_delta_dump_merge_and_in_place_restore(ctx):
    c = 65536
    rng = np.random.default_rng(22)
    gen = torch.Generator(device=DEV).manual_seed(22)
    base = _rand_table(rng, gen, 10, c, max_chunks=30)
    new = [(i, t.clone()) for i, t in base]
    workloads.mutate_runs(new, seed=23, chunk=c, frac=0.2, run_mean=3)
    new[1] = (new[1][0], torch.zeros_like(new[1][1]))
    new[2] = (new[2][0] + 77, new[2][1])               # renamed: no match in the base
    b_img, b_or, _ = check_parity(ctx, base, c)
    d_img, d_or, res = check_parity(ctx, new, c, prev_gpu=b_img, prev_oracle=b_or)
    assert res.n_unchanged > 0
    # the same delta through every launch form: one window (three passes:
    # digests and kinds, offsets, gather), several windows and a captured
    # graph (single pass with look-back), one launch per allocation
    for kw in (dict(window_bytes=4 * c), dict(flags=mk.OPT_GRAPH), dict(flags=mk.OPT_PER_ALLOC),
               dict(flags=mk.OPT_PER_ALLOC, window_bytes=2 * c)):
        check_parity(ctx, new, c, prev_gpu=b_img, prev_oracle=b_or, **kw)
    # other chunk sizes: a streamed tile shape (16 KiB) and several passes per chunk (256 KiB)
    for c2 in (16384, 262144):
        b2, bo2, _ = check_parity(ctx, base, c2)
        check_parity(ctx, new, c2, prev_gpu=b2, prev_oracle=bo2)
        check_parity(ctx, new, c2, prev_gpu=b2, prev_oracle=bo2, window_bytes=4 * c2)
    # same delta when the previous image is not resident (imported copy)
    rc, b_imp = mk.ckpt_image_import(b_img.view())
    assert rc == 0
    check_parity(ctx, new, c, prev_gpu=b_imp, prev_oracle=b_or)
    # merge == full dump (library and oracle)
    rc, merged = mk.ckpt_merge(b_img, d_img)
    assert rc == 0
    rc, full_or = corc.dump(host(new), c)
    assert np.array_equal(merged.view(), full_or)
    # in-place: restore base, then the delta
    targets = [(i, torch.zeros_like(t)) for i, t in new]
    base_targets = [(i, t) for (i, _), (_, t) in zip(base, targets)]
    assert mk.ckpt_restore(ctx, b_img, base_targets)[0] == 0
    rc, r = mk.ckpt_restore(ctx, d_img, targets)
    assert rc == 0, mk.ckpt_strerror(rc)
    torch.cuda.synchronize()
    for (_, a), (_, b) in zip(new, targets):
        assert torch.equal(a, b)


def test_resident_digest_tables_past_capacity(ctx):
    """More images than the context keeps digest tables for (8): evicted
    tables' buffers take later tables of other sizes; deltas against the
    newest images (tables resident) and the oldest (evicted) match the
    oracle, and the newest delta restores in place."""
    c = 4096
    rng = np.random.default_rng(41)
    gen = torch.Generator(device=DEV).manual_seed(41)
    states = []
    for k in range(11):
        table = _rand_table(rng, gen, 2 + k % 4, c, zero_p=0.2, max_chunks=2 + 3 * (k % 3))
        img, oimg, _ = check_parity(ctx, table, c)
        states.append((table, img, oimg))
    for k in (0, 1, 9, 10):
        table, img, oimg = states[k]
        new = [(i, t.clone()) for i, t in table]
        workloads.mutate_runs(new, seed=50 + k, chunk=c, frac=0.3, run_mean=2)
        d_img, _, _ = check_parity(ctx, new, c, prev_gpu=img, prev_oracle=oimg)
    targets = [(i, t.clone()) for i, t in table]
    rc, _ = mk.ckpt_restore(ctx, d_img, targets)
    assert rc == 0
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for (_, a), (_, b) in zip(targets, new))


def test_error_paths_match_the_oracle(ctx):
    c = 4096
    rng = np.random.default_rng(24)
    gen = torch.Generator(device=DEV).manual_seed(24)
    table = _rand_table(rng, gen, 6, c, zero_p=0.2)
    img, oimg, _ = check_parity(ctx, table, c)
    raw = img.tobytes()
    n = len(table)
    nc = corc.parse(oimg)[1]["n_chunks"]
    tl = (32 * n + 5 * nc + 15) & ~15
    spots = [0, 12, 30, 61, 64 + 3, 64 + 32 * n + 2, 64 + 32 * n + 4 * nc]
    if len(raw) > 64 + tl:
        spots += [64 + tl + 1, len(raw) - 1]
    for pos in spots:
        bad = bytearray(raw)
        bad[pos] ^= 0x10
        bad = bytes(bad)
        hosts = [(i, np.zeros(t.numel(), np.uint8)) for i, t in table]
        want = corc.restore(bad, hosts)
        rc, bimg = mk.ckpt_image_import(bad)
        if rc != 0:
            # the import validates header and tables on the host
            assert rc == want[0] == mk.CKPT_ECORRUPT
            continue
        targets = [(i, torch.zeros_like(t)) for i, t in table]
        rc, res = mk.ckpt_restore(ctx, bimg, targets)
        assert (rc, res.first_bad_chunk) == want, pos
    # table mismatch and wrong base
    t2 = [(i + 1, t) for i, t in table]
    assert mk.ckpt_restore(ctx, img, t2)[0] == mk.CKPT_EMISMATCH
    new = [(i, t.clone()) for i, t in table]
    workloads.mutate_runs(new, seed=25, chunk=c, frac=0.3, run_mean=2)
    d_img, d_or, _ = check_parity(ctx, new, c, prev_gpu=img, prev_oracle=oimg)
    wrong = [(i, torch.full_like(t, 3)) for i, t in table]
    rc, res = mk.ckpt_restore(ctx, d_img, wrong)
    want = corc.restore(d_or, [(i, np.full(t.numel(), 3, np.uint8)) for i, t in table])
    assert (rc, res.first_bad_chunk) == want and rc == mk.CKPT_EBASE
    # the base check runs before any chunk is written: the targets are untouched
    torch.cuda.synchronize()
    assert all(bool((t == 3).all()) for _, t in wrong)
    # likewise with the strict re-read, and on the on-demand path (whose
    # base check the host waits for before the first upload)
    rc, res = mk.ckpt_restore(ctx, d_img, wrong, opts=mk.make_opts(strict_verify=1))
    assert (rc, res.first_bad_chunk) == want
    rc, res = mk.ckpt_restore_some(ctx, d_img, wrong)
    assert (rc, res.first_bad_chunk) == want
    torch.cuda.synchronize()
    assert all(bool((t == 3).all()) for _, t in wrong)
    # and the same targets holding the base then take the delta
    good = [(i, t.clone()) for i, t in table]
    rc, _ = mk.ckpt_restore(ctx, d_img, good)
    assert rc == 0
    assert all(torch.equal(g, t) for (_, g), (_, t) in zip(good, new))


def test_pageable_host_images(ctx):
    """Images in pageable host memory (the fallback once the driver's pinned
    memory is used up) dump and restore exactly as pinned ones."""
    c = 65536
    rng = np.random.default_rng(31)
    gen = torch.Generator(device=DEV).manual_seed(31)
    table = _rand_table(rng, gen, 12, c, max_chunks=8)
    os.environ["MICKPT_HOST_PAGEABLE"] = "1"
    try:
        img, oimg, _ = check_parity(ctx, table, c)
        restore_and_compare(ctx, img, table)
        new = [(i, t.clone()) for i, t in table]
        workloads.mutate_runs(new, seed=32, chunk=c, frac=0.3, run_mean=2)
        check_parity(ctx, new, c, prev_gpu=img, prev_oracle=oimg)
        check_parity(ctx, table, c, window_bytes=2 * c)
    finally:
        del os.environ["MICKPT_HOST_PAGEABLE"]


def test_on_demand_restore_of_listed_allocations(ctx):
    """ckpt_restore_some: the listed allocations (any order, by id) get the
    bytes the oracle restores from the same image; unlisted targets are not
    touched; unknown ids, other sizes and repeated ids are rejected."""
    c = 65536
    rng = np.random.default_rng(33)
    gen = torch.Generator(device=DEV).manual_seed(33)
    table = _rand_table(rng, gen, 14, c, max_chunks=10)
    img, oimg, _ = check_parity(ctx, table, c)
    # the oracle's restore of the whole image: the reference bytes
    ref = [(i, np.zeros(t.numel(), np.uint8)) for i, t in table]
    rc, first_bad = corc.restore(oimg, ref)
    assert rc == 0
    targets = [(i, torch.full_like(t, 0xA5) if t.numel() else t.clone()) for i, t in table]
    pick = [5, 0, 11, 3, 8]                      # any order
    for opts in (None, mk.make_opts(window_bytes=2 * c)):
        for _, t in targets:
            t.fill_(0xA5)
        rc, res = mk.ckpt_restore_some(ctx, img, [targets[k] for k in pick], opts=opts)
        assert rc == 0, mk.ckpt_strerror(rc)
        torch.cuda.synchronize()
        for k, ((_, t), (_, r)) in enumerate(zip(targets, ref)):
            got = t.cpu().numpy()
            if k in pick:
                assert np.array_equal(got, r), k
            else:
                assert (got == 0xA5).all(), k         # untouched
        assert res.n_logical == sum(table[k][1].numel() for k in pick)
    # the remaining allocations in a second call complete the restore
    rest = [targets[k] for k in range(len(table)) if k not in pick]
    assert mk.ckpt_restore_some(ctx, img, rest)[0] == 0
    torch.cuda.synchronize()
    for (_, t), (_, r) in zip(targets, ref):
        assert np.array_equal(t.cpu().numpy(), r)
    # errors
    big = [k for k, (_, t) in enumerate(table) if t.numel() > 0][0]
    wrong_size = [(table[big][0], torch.zeros(table[big][1].numel() + 16, dtype=torch.uint8, device=DEV))]
    assert mk.ckpt_restore_some(ctx, img, wrong_size)[0] == mk.CKPT_EMISMATCH
    assert mk.ckpt_restore_some(ctx, img, [(12345, targets[0][1])])[0] == mk.CKPT_EMISMATCH
    assert mk.ckpt_restore_some(ctx, img, [targets[big], targets[big]])[0] == mk.CKPT_EINVAL
    # a delta: the listed allocations must hold the base in their UNCHANGED chunks
    new = [(i, t.clone()) for i, t in table]
    workloads.mutate_runs(new, seed=34, chunk=c, frac=0.3, run_mean=2)
    d_img, _, dres = check_parity(ctx, new, c, prev_gpu=img, prev_oracle=oimg)
    assert dres.n_unchanged > 0
    base_targets = [(i, t.clone()) for i, t in table]
    assert mk.ckpt_restore_some(ctx, d_img, [base_targets[k] for k in pick])[0] == 0
    torch.cuda.synchronize()
    for k in pick:
        assert torch.equal(base_targets[k][1], new[k][1])


def test_image_file_round_trip(ctx, tmp_path):
    """A dumped image (pinned host memory) saved to a file and loaded back is
    byte-identical and restores the state."""
    c = 65536
    rng = np.random.default_rng(35)
    gen = torch.Generator(device=DEV).manual_seed(35)
    table = _rand_table(rng, gen, 10, c, max_chunks=200)
    img, oimg, _ = check_parity(ctx, table, c)
    path = str(tmp_path / "state.img")
    assert mk.ckpt_image_save(img, path, 4) == 0
    rc, back = mk.ckpt_image_load(path, 3)
    assert rc == 0 and np.array_equal(back.view(), oimg)
    restore_and_compare(ctx, back, table)


def test_corrupt_previous_image_is_rejected_like_the_oracle(ctx):
    """A delta dump against a previous image whose header or tables were
    damaged fails with the oracle's code (the previous digest table is
    checked before it is trusted); damage in its payload, which a delta
    dump never reads, leaves both sides' delta images equal."""
    c = 4096
    rng = np.random.default_rng(71)
    gen = torch.Generator(device=DEV).manual_seed(71)
    table = _rand_table(rng, gen, 6, c, max_chunks=8)
    for where in ("header", "records", "crc", "kind", "payload"):
        prev_g, prev_o, _ = check_parity(ctx, table, c)
        v = prev_g.view()           # the library's own image bytes, writable
        n = len(table)
        nc = int(np.frombuffer(prev_o[24:32].tobytes(), np.uint64)[0])
        tl = (32 * n + 5 * nc + 15) & ~15
        pos = {"header": 33, "records": 64 + 8, "crc": 64 + 32 * n + 4 * (nc // 2),
               "kind": 64 + 32 * n + 4 * nc + nc // 2, "payload": 64 + tl + 100}[where]
        v[pos] ^= 0x40
        bad_o = prev_o.copy()
        bad_o[pos] ^= 0x40
        orc, oimg = corc.dump(host(table), c, prev=bad_o)
        rc, img, _ = mk.ckpt_dump(ctx, table, prev=prev_g, opts=mk.make_opts(chunk_size=c))
        assert rc == orc, (where, rc, orc)
        if where == "payload":
            assert rc == 0 and np.array_equal(img.view(), oimg)
            img.free()
        else:
            assert rc == mk.CKPT_ECORRUPT and img is None
        prev_g.free()


def test_fresh_lookback_words_are_cleared():
    """Look-back status words live in device memory that hipMalloc may hand
    back from earlier allocations. Device memory is filled with words that
    read as published inclusive prefixes of the first epoch (value 0, so a
    dump that trusted them would misplace records, not write out of bounds)
    and returned to the runtime; a fresh context's first dumps -- whose
    status buffers may reuse that memory -- still give the oracle's images."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    word = (2 << 62) | (1 << 40)       # inclusive prefix, epoch 1, value 0
    poison = [torch.full((2 << 20,), word - (1 << 64), dtype=torch.int64, device=DEV) for _ in range(64)]
    torch.cuda.synchronize()
    del poison
    torch.cuda.empty_cache()
    c2 = mk.ckpt_ctx_create(0, 64 << 20)
    try:
        gen = torch.Generator(device=DEV).manual_seed(72)
        for c, size in ((64, 8 << 20), (4096, 24 << 20), (65536, 40 << 20)):
            t = torch.randint(0, 256, (size,), dtype=torch.uint8, device=DEV, generator=gen)
            t[size // 3:size // 2] = 0
            img, _, _ = check_parity(c2, [(1, t), (2, t[:size // 5].clone())], c)
            img.free()
    finally:
        mk.ckpt_ctx_destroy(c2)


def test_strict_verify_restores_and_reports_like_the_oracle(ctx):
    """strict_verify = 1: a good image restores byte for byte and the re-read
    stage is timed; a damaged payload gives the oracle's (code, first bad
    chunk), as without strict mode; a delta applied in place with strict mode
    re-reads every chunk, UNCHANGED ones included."""
    c = 16384
    rng = np.random.default_rng(73)
    gen = torch.Generator(device=DEV).manual_seed(73)
    table = _rand_table(rng, gen, 10, c, max_chunks=9)
    img, oimg, _ = check_parity(ctx, table, c)
    res = restore_and_compare(ctx, img, table, strict_verify=1)
    assert res.ns_stage[4] > 0 and res.ns_stage[3] > 0
    plain = restore_and_compare(ctx, img, table)
    assert plain.ns_stage[4] == 0
    bad = oimg.copy()
    bad[bad.size - 3000] ^= 0x08
    want = corc.restore(bad, [(i, np.zeros(t.numel(), np.uint8)) for i, t in table])
    rc, bimg = mk.ckpt_image_import(bad)
    assert rc == 0
    for strict in (0, 1):
        targets = [(i, torch.zeros_like(t)) for i, t in table]
        rc, r = mk.ckpt_restore(ctx, bimg, targets, opts=mk.make_opts(strict_verify=strict))
        assert (rc, r.first_bad_chunk) == want and rc == mk.CKPT_ECORRUPT
    bimg.free()
    # delta in place, strict
    prev = [(i, t.clone()) for i, t in table]
    workloads.mutate_runs(table, seed=74, chunk=c, frac=0.3, run_mean=2)
    delta, odelta, dres = check_parity(ctx, table, c, prev_gpu=img, prev_oracle=oimg)
    assert dres.n_unchanged > 0
    rc, r = mk.ckpt_restore(ctx, delta, prev, opts=mk.make_opts(strict_verify=1))
    assert rc == 0, (mk.ckpt_strerror(rc), r.first_bad_chunk)
    assert r.ns_stage[1] > 0 and r.ns_stage[4] > 0
    torch.cuda.synchronize()
    for (_, a), (_, b) in zip(table, prev):
        assert torch.equal(a, b)
    assert mk.ckpt_restore(ctx, img, table, opts=mk.make_opts(strict_verify=2))[0] == mk.CKPT_EINVAL
    img.free()
    delta.free()


def test_strict_verify_sees_writes_that_did_not_stick(ctx):
    """Two allocations of the table restored into the same device memory: each
    chunk passes the fused check as it is written, but the memory can hold
    only one of the two contents, so the strict re-read fails (the fused
    check alone cannot see it)."""
    c = 65536
    gen = torch.Generator(device=DEV).manual_seed(75)
    a = torch.randint(0, 256, (8 * c + 100,), dtype=torch.uint8, device=DEV, generator=gen)
    b = torch.randint(0, 256, (8 * c + 100,), dtype=torch.uint8, device=DEV, generator=gen)
    img, _, _ = check_parity(ctx, [(1, a), (2, b)], c)
    same = torch.zeros_like(a)
    rc, r = mk.ckpt_restore(ctx, img, [(1, same), (2, same)])
    assert rc == 0
    rc, r = mk.ckpt_restore(ctx, img, [(1, same), (2, same)], opts=mk.make_opts(strict_verify=1))
    assert rc == mk.CKPT_ECORRUPT and r.first_bad_chunk < 18
    img.free()


def test_stage_times_are_reported(ctx):
    """ckpt_result.ns_stage: the stages each call form runs are timed, the
    others are 0, and CKPT_OPT_NO_TIMING leaves only the wall times."""
    c = 65536
    rng = np.random.default_rng(76)
    gen = torch.Generator(device=DEV).manual_seed(76)
    table = _rand_table(rng, gen, 8, c, max_chunks=20)
    img, res = gpu_dump(ctx, table, chunk_size=c)
    st = list(res.ns_stage)
    assert st[0] > 0 and st[1] > 0 and st[2] == 0 and st[3] == 0 and st[4] > 0 and st[5] > 0 and st[7] >= st[4]
    assert st[1] == res.ns_kernel
    workloads.mutate_runs(table, seed=77, chunk=c, frac=0.2, run_mean=3)
    delta, dres = gpu_dump(ctx, table, prev=img, chunk_size=c)
    st = list(dres.ns_stage)
    assert all(x > 0 for x in (st[0], st[1], st[2], st[3], st[5], st[7]))
    rc, r = mk.ckpt_restore(ctx, img, table)
    assert rc == 0
    st = list(r.ns_stage)
    assert st[0] > 0 and st[1] == 0 and st[2] > 0 and st[3] > 0 and st[4] == 0 and st[5] > 0 and st[7] > 0
    rc, r = mk.ckpt_restore(ctx, delta, table, opts=mk.make_opts(flags=mk.OPT_NO_TIMING))
    assert rc == 0
    st = list(r.ns_stage)
    assert st[1] > 0 and st[3] == 0 and st[5] == 0 and st[7] > 0
    img.free()
    delta.free()


def test_graph_restore_replays_and_rejects_corrupt_images(ctx):
    """Batched form, restore side: a full image restores through one captured
    graph, replayed on new images of the same table (strict mode too); an
    image whose tables were damaged is rejected by the graph's own
    validation with the oracle's code and nothing written; a damaged payload
    gives the oracle's (code, first bad chunk)."""
    c = 65536
    rng = np.random.default_rng(78)
    gen = torch.Generator(device=DEV).manual_seed(78)
    table = _rand_table(rng, gen, 30, c, max_chunks=6)
    gopts = dict(flags=mk.OPT_GRAPH)
    for rep in range(3):
        if rep:
            workloads.mutate_runs(table, seed=79 + rep, chunk=c, frac=0.3, run_mean=2)
        img, oimg, _ = check_parity(ctx, table, c, **gopts)
        res = restore_and_compare(ctx, img, table, strict_verify=int(rep == 2), **gopts)
        assert res.windows == 1 and res.ns_stage[3] > 0
        img.free()
    img, oimg, _ = check_parity(ctx, table, c)
    n = len(table)
    nc = int(np.frombuffer(oimg[24:32].tobytes(), np.uint64)[0])
    # damaged crc[] entry: the tables digest no longer matches
    v = img.view()
    pos = 64 + 32 * n + 4 * (nc // 3)
    v[pos] ^= 0x01
    bad_o = oimg.copy()
    bad_o[pos] ^= 0x01
    want = corc.restore(bad_o, [(i, np.zeros(t.numel(), np.uint8)) for i, t in table])
    targets = [(i, torch.full_like(t, 0x5A) if t.numel() else t.clone()) for i, t in table]
    rc, r = mk.ckpt_restore(ctx, img, targets, opts=mk.make_opts(**gopts))
    assert (rc, r.first_bad_chunk) == want and rc == mk.CKPT_ECORRUPT
    torch.cuda.synchronize()
    assert all(bool((t == 0x5A).all()) for _, t in targets if t.numel())    # nothing written
    v[pos] ^= 0x01
    # damaged payload
    v[v.size - 777] ^= 0x20
    bad_o = oimg.copy()
    bad_o[bad_o.size - 777] ^= 0x20
    want = corc.restore(bad_o, [(i, np.zeros(t.numel(), np.uint8)) for i, t in table])
    rc, r = mk.ckpt_restore(ctx, img, targets, opts=mk.make_opts(**gopts))
    assert (rc, r.first_bad_chunk) == want and rc == mk.CKPT_ECORRUPT
    img.free()
