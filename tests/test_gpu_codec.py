"""GPU parity of the byte-plane codec (CKPT_OPT_CODEC): images from the HIP
path are byte-identical to the CPU oracle's codec images, restores of PACKED
records write back exactly the dumped bytes, and corrupt records are reported
at the same chunk as the oracle reports them. Every call goes through the C
ABI."""
import os
import struct
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import oracle as corc  # noqa: E402
from paper_2502_16631_amd import mickpt as mk  # noqa: E402
import workloads  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda"
PACKED = 3


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = mk.ckpt_ctx_create(0, 1 << 30)
    yield c
    mk.ckpt_ctx_destroy(c)


def typed_table(c, seed):
    """Allocations of the number formats a device holds in training and HPC
    jobs, with ragged tails: bf16 N(0, 0.02) weights, fp32 N(0, 1e-3)
    optimizer state, bf16 N(0, 1) activations, fp64 N(0, 1), uniform int32,
    small-integer int32, all-zero and constant regions, random bytes."""
    gen = torch.Generator(device=DEV).manual_seed(seed)
    rng = np.random.default_rng(seed)

    def n_of(width, chunks):
        return (chunks * c + int(rng.integers(0, c))) // width

    t = []
    t.append((torch.randn(n_of(2, 7), generator=gen, device=DEV) * 0.02).to(torch.bfloat16))
    t.append(torch.randn(n_of(4, 5), generator=gen, device=DEV) * 1e-3)
    t.append(torch.randn(n_of(2, 4), generator=gen, device=DEV).to(torch.bfloat16))
    t.append(torch.randn(n_of(8, 4), generator=gen, device=DEV, dtype=torch.float64))
    t.append(torch.randint(-2 ** 31, 2 ** 31 - 1, (n_of(4, 3),), generator=gen, device=DEV, dtype=torch.int32))
    t.append(torch.randint(0, 9, (n_of(4, 3),), generator=gen, device=DEV, dtype=torch.int32))
    z = torch.zeros(3 * c + 40, dtype=torch.uint8, device=DEV)
    z[c:2 * c] = 7                                   # one constant chunk between zero ones
    t.append(z)
    t.append(torch.randint(0, 256, (2 * c + 5,), generator=gen, device=DEV, dtype=torch.uint8))
    t.append(torch.zeros(0, dtype=torch.uint8, device=DEV))
    return [(5000 + i, x.view(torch.uint8).reshape(-1)) for i, x in enumerate(t)]


def host(table):
    return workloads.host_copy(table)


def codec_parity(ctx, table, c, prev_gpu=None, prev_oracle=None, **kw):
    flags = kw.pop("flags", 0) | mk.OPT_CODEC
    rc, img, res = mk.ckpt_dump(ctx, table, prev=prev_gpu, opts=mk.make_opts(chunk_size=c, flags=flags, **kw))
    assert rc == 0, mk.ckpt_strerror(rc)
    rc, oimg = corc.dump(host(table), c, prev=prev_oracle, codec=True)
    assert rc == 0
    got = img.view()
    assert got.size == oimg.size, (got.size, oimg.size)
    if not np.array_equal(got, oimg):
        diff = np.nonzero(got != oimg)[0]
        raise AssertionError("image differs at %d bytes, first at %d" % (diff.size, diff[0]))
    return img, oimg, res


def restore_check(ctx, img, table, **kw):
    targets = [(i, torch.full_like(t, 0x5A) if t.numel() else t.clone()) for i, t in table]
    rc, res = mk.ckpt_restore(ctx, img, targets, opts=mk.make_opts(**kw))
    assert rc == 0, (mk.ckpt_strerror(rc), res.first_bad_chunk)
    torch.cuda.synchronize()
    for (_, a), (_, b) in zip(table, targets):
        assert torch.equal(a, b)
    return res


@pytest.mark.parametrize("c", [4096, 8192, 16384, 32768, 65536])
def test_codec_images_match_the_oracle(ctx, c):
    table = typed_table(c, seed=c)
    img, oimg, res = codec_parity(ctx, table, c)
    assert res.n_packed > 0 and res.n_payload < res.n_logical
    assert res.n_zero + res.n_data + res.n_packed == res.n_chunks
    r = restore_check(ctx, img, table)
    assert r.n_packed == res.n_packed
    # several restore windows
    restore_check(ctx, img, table, window_bytes=2 * c)
    # the oracle's image restores through the device decode too
    rc, oi = mk.ckpt_image_import(oimg.tobytes())
    assert rc == 0
    restore_check(ctx, oi, table)


def test_codec_delta_merge_and_on_demand_restore(ctx):
    c = 65536
    base = typed_table(c, seed=41)
    new = [(i, t.clone()) for i, t in base]
    workloads.mutate_runs(new, seed=42, chunk=c, frac=0.3, run_mean=2)
    new[6] = (new[6][0], torch.zeros_like(new[6][1]))
    b_img, b_or, _ = codec_parity(ctx, base, c)
    d_img, d_or, res = codec_parity(ctx, new, c, prev_gpu=b_img, prev_oracle=b_or)
    assert res.n_unchanged > 0
    # a codec delta against a plain base, and a plain delta against a codec base
    rc, p_img, _ = mk.ckpt_dump(ctx, base, opts=mk.make_opts(chunk_size=c))
    rc, p_or = corc.dump(host(base), c)
    codec_parity(ctx, new, c, prev_gpu=p_img, prev_oracle=p_or)
    rc, pd, _ = mk.ckpt_dump(ctx, new, prev=b_img, opts=mk.make_opts(chunk_size=c))
    rc, pd_or = corc.dump(host(new), c, prev=b_or)
    assert rc == 0 and np.array_equal(pd.view(), pd_or)
    # merge == full codec dump (library and oracle)
    rc, merged = mk.ckpt_merge(b_img, d_img)
    assert rc == 0
    rc, full_or = corc.dump(host(new), c, codec=True)
    assert np.array_equal(merged.view(), full_or)
    rc, m_or = corc.merge(b_or, d_or)
    assert np.array_equal(m_or, full_or)
    # in-place delta restore over the base
    targets = [(i, t.clone()) for i, t in base]
    rc, r = mk.ckpt_restore(ctx, d_img, targets)
    assert rc == 0, mk.ckpt_strerror(rc)
    torch.cuda.synchronize()
    for (_, a), (_, b) in zip(new, targets):
        assert torch.equal(a, b)
    # on-demand restore of some allocations of a codec image
    targets = [(i, torch.full_like(t, 0xA5) if t.numel() else t.clone()) for i, t in new]
    pick = [3, 0, 5]
    rc, _ = mk.ckpt_restore_some(ctx, merged, [targets[k] for k in pick])
    assert rc == 0, mk.ckpt_strerror(rc)
    torch.cuda.synchronize()
    for k, ((_, t), (_, ref)) in enumerate(zip(targets, new)):
        if k in pick:
            assert torch.equal(t, ref), k
        elif t.numel():
            assert bool((t == 0xA5).all()), k


def _packed_record(oimg):
    """(chunk index, payload offset, length, record bytes) of a PACKED chunk
    whose record has a DICT plane with escapes, and the tables length."""
    p = corc.parse(oimg)[1]
    n, nc = p["n_allocs"], p["n_chunks"]
    tl = (32 * n + 9 * nc + 15) & ~15
    rl = np.frombuffer(oimg[64 + 32 * n + 4 * nc: 64 + 32 * n + 8 * nc].tobytes(), np.uint32)
    kinds = oimg[64 + 32 * n + 8 * nc: 64 + 32 * n + 9 * nc]
    pos = 0
    for g in range(nc):
        if kinds[g] == PACKED:
            rec = oimg[64 + tl + pos: 64 + tl + pos + rl[g]].tobytes()
            escs = struct.unpack_from("<8I", rec, 8)
            if any(rec[q] == 2 and escs[q] > 0 for q in range(8)):
                return g, 64 + tl + pos, int(rl[g]), rec
        pos += int(rl[g])
    raise AssertionError("no PACKED record with escapes")


def test_corrupt_records_match_the_oracle(ctx):
    c = 16384
    table = typed_table(c, seed=43)
    img, oimg, _ = codec_parity(ctx, table, c)
    g, at, rl, rec = _packed_record(oimg)
    q = next(q for q in range(8) if rec[q] == 2 and struct.unpack_from("<8I", rec, 8)[q] > 0)
    L = c // 8
    sec = 48 + sum(16 if rec[p] == 1 else L if rec[p] == 0 else
                   16 + L // 2 + ((struct.unpack_from("<8I", rec, 8)[p] + 15) & ~15) for p in range(q))
    spots = {
        "mode": at + 0,
        "escape count": at + 8 + 4 * q,
        "reserved": at + 45,
        "dictionary entry": at + sec + 1,
        "code byte": at + sec + 16 + 3,
        "escape byte": at + sec + 16 + L // 2,
        "raw or last byte": at + rl - 1,
    }
    for name, pos in spots.items():
        bad = oimg.copy()
        bad[pos] ^= 0x21
        want = corc.restore(bad, [(i, np.zeros(t.numel(), np.uint8)) for i, t in table])
        rc, bimg = mk.ckpt_image_import(bad.tobytes())
        assert rc == 0, name                    # payload bytes are not covered by the tables digest
        targets = [(i, torch.zeros_like(t)) for i, t in table]
        rc, res = mk.ckpt_restore(ctx, bimg, targets)
        assert (rc, res.first_bad_chunk) == want, name
        if name in ("mode", "escape count", "reserved", "code byte", "escape byte"):
            assert want == (mk.CKPT_ECORRUPT, g), name


def test_codec_option_errors(ctx):
    table = typed_table(4096, seed=44)
    for kw in (dict(chunk_size=2048, flags=mk.OPT_CODEC),
               dict(chunk_size=131072, flags=mk.OPT_CODEC),
               dict(chunk_size=4096, flags=mk.OPT_CODEC | mk.OPT_PER_ALLOC),
               dict(chunk_size=4096, flags=mk.OPT_CODEC | mk.OPT_GRAPH)):
        rc, img, _ = mk.ckpt_dump(ctx, table, opts=mk.make_opts(**kw))
        assert rc == mk.CKPT_EINVAL and img is None, kw
    # the context still works afterwards
    img, _, _ = codec_parity(ctx, table, 4096)
    restore_check(ctx, img, table)


@pytest.mark.parametrize("c,win_chunks", [(4096, 4), (16384, 7), (65536, 3)])
def test_codec_dump_over_several_staging_windows(ctx, c, win_chunks):
    """A codec dump whose payload spans several staging windows (pieces on
    the slot ring) gives the oracle's image, also as a delta and with
    three slots; it restores."""
    table = typed_table(c, seed=c + 7)
    img, oimg, res = codec_parity(ctx, table, c, window_bytes=win_chunks * c)
    assert res.windows > 2
    codec_parity(ctx, table, c, window_bytes=win_chunks * c, slots=3)
    restore_check(ctx, img, table)
    new = [(i, t.clone()) for i, t in table]
    workloads.mutate_runs(new, seed=c + 8, chunk=c, frac=0.3, run_mean=2)
    codec_parity(ctx, new, c, prev_gpu=img, prev_oracle=oimg, window_bytes=win_chunks * c)


def test_served_loop_rejects_codec_images_and_takes_plain_ones(ctx):
    """The served request loop restores the plain layout only: a codec image
    ends with CKPT_EINVAL, the plain image of the same state restores, and a
    served delta dump against a codec base gives the oracle's plain delta."""
    import time
    c = 65536
    table = typed_table(c, seed=45)
    img, oimg, _ = codec_parity(ctx, table, c)
    rc, plain, _ = mk.ckpt_dump(ctx, table, opts=mk.make_opts(chunk_size=c))
    assert rc == 0
    srv = mk.ckpt_serve_create(ctx, 4, 1 << 30)
    try:
        targets = [(i, torch.zeros_like(t)) for i, t in table]
        rc1, t1 = mk.ckpt_serve_submit(srv, mk.REQ_RESTORE, targets, img=img)
        rc2, t2 = mk.ckpt_serve_submit(srv, mk.REQ_RESTORE, targets, img=plain)
        new = [(i, t.clone()) for i, t in table]
        workloads.mutate_runs(new, seed=46, chunk=c, frac=0.3, run_mean=2)
        rc3, t3 = mk.ckpt_serve_submit(srv, mk.REQ_DUMP, new, prev=img)
        assert rc1 == rc2 == rc3 == 0
        got = {}
        t0 = time.time()
        while len(got) < 3:
            for k, tk in (("codec", t1), ("plain", t2), ("delta", t3)):
                if k not in got:
                    done, rc, out, lat = mk.ckpt_serve_poll(srv, tk)
                    if done:
                        got[k] = (rc, out)
            assert time.time() - t0 < 120, "serving requests did not complete"
            time.sleep(0.001)
        assert got["codec"][0] == mk.CKPT_EINVAL
        assert got["plain"][0] == 0
        torch.cuda.synchronize()
        for (_, a), (_, b) in zip(table, targets):
            assert torch.equal(a, b)
        assert got["delta"][0] == 0
        rc, want = corc.dump(workloads.host_copy(new), c, prev=oimg)
        assert rc == 0 and np.array_equal(got["delta"][1].view(), want)
    finally:
        mk.ckpt_serve_destroy(srv)
