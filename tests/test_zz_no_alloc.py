"""ckpt_dump_into: the dump into fixed buffers (the caller's host buffer and
the library's per-GPU device array) gives the same image bytes as ckpt_dump
for the same arguments, on calls in a row whose inputs shrink, grow past one
staging slot and carry a previous image, allocates no device memory, and
rejects what does not fit. Every call goes through the C ABI."""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2502_16631_amd import mickpt as mk  # noqa: E402
import workloads  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _table(gen, sizes, zero_every=3, c=65536):
    out = []
    for i, s in enumerate(sizes):
        t = torch.randint(0, 256, (s,), dtype=torch.uint8, device=DEV, generator=gen)
        for k, lo in enumerate(range(0, s, c)):
            if k % zero_every == 1:
                t[lo:lo + c] = 0
        out.append((1000 + i, t))
    return out


def _same_as_dump(ctx, table, out, prev=None, **kw):
    """ckpt_dump_into's image equals ckpt_dump's for the same arguments."""
    opts = mk.make_opts(**kw)
    rc, img, res = mk.ckpt_dump(ctx, table, prev=prev, opts=opts)
    assert rc == 0, mk.ckpt_strerror(rc)
    want = img.view().copy()
    img.free()
    out[:] = 0xEE
    rc, n, r = mk.ckpt_dump_into(ctx, table, out, prev=prev, opts=opts)
    assert rc == 0, mk.ckpt_strerror(rc)
    assert n == want.size and r.n_payload == res.n_payload and r.n_chunks == res.n_chunks
    assert np.array_equal(out[:n], want), "first difference at byte %d" % int(np.nonzero(out[:n] != want)[0][0])
    return n, r


def test_dump_into_matches_dump_on_calls_in_a_row():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = mk.ckpt_ctx_create(0, 1 << 30)
    try:
        gen = torch.Generator(device=DEV).manual_seed(91)
        out = np.zeros(300 << 20, dtype=np.uint8)
        big = _table(gen, [40 << 20, 3 << 20, 77, 0, (20 << 20) + 5])                 # ~63 MiB: one window
        small = _table(gen, [1 << 20, 4096 + 3, 65536])                              # then a smaller input
        several = _table(gen, [100 << 20, 64 << 20, 12345])                          # > one slot: windows on two slots
        print("dump_into: one window, 63 MiB", flush=True)
        _same_as_dump(ctx, big, out)
        print("dump_into: smaller input", flush=True)
        _same_as_dump(ctx, small, out)
        print("dump_into: several windows", flush=True)
        n, r = _same_as_dump(ctx, several, out)
        assert r.windows >= 3
        print("dump_into: 16 KiB chunks, 256 threads", flush=True)
        _same_as_dump(ctx, small, out, chunk_size=16384, wg_threads=256)
        # a delta against an image of ckpt_dump
        rc, base, _ = mk.ckpt_dump(ctx, big, opts=mk.make_opts())
        assert rc == 0
        workloads.mutate_runs(big, seed=92, chunk=65536, frac=0.1, run_mean=3)
        torch.cuda.synchronize()
        print("dump_into: delta", flush=True)
        n, r = _same_as_dump(ctx, big, out, prev=base)
        assert r.n_unchanged > 0
        base.free()
        # no device memory is allocated by a call (its buffers are the array)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        for tab in (several, small):
            rc, n, _ = mk.ckpt_dump_into(ctx, tab, out)
            assert rc == 0
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
    finally:
        mk.ckpt_ctx_destroy(ctx)


def test_dump_into_limits():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = mk.ckpt_ctx_create(0, 1 << 30)
    try:
        gen = torch.Generator(device=DEV).manual_seed(93)
        table = _table(gen, [5 << 20, 1000])
        tiny = np.zeros(4096, dtype=np.uint8)
        rc, n, _ = mk.ckpt_dump_into(ctx, table, tiny)
        assert rc == mk.CKPT_ENOMEM and n == 0
        out = np.zeros(16 << 20, dtype=np.uint8)
        # more allocations than the array's descriptors hold
        many = [(i, 0, 0) for i in range(16385)]
        rc, n, _ = mk.ckpt_dump_into(ctx, many, out)
        assert rc == mk.CKPT_ELIMIT and n == 0
        # more chunks than its tables hold (2^20 + 1 chunks of 16 bytes)
        t = torch.zeros((1 << 24) + 16, dtype=torch.uint8, device=DEV)
        rc, n, _ = mk.ckpt_dump_into(ctx, [(1, t)], out, opts=mk.make_opts(chunk_size=16))
        assert rc == mk.CKPT_ELIMIT and n == 0
        # a chunk larger than a staging slot
        rc, n, _ = mk.ckpt_dump_into(ctx, [(1, t)], out, opts=mk.make_opts(chunk_size=1 << 26))
        assert rc == mk.CKPT_ELIMIT and n == 0
        # forms that allocate are refused
        rc, n, _ = mk.ckpt_dump_into(ctx, table, out, opts=mk.make_opts(flags=mk.OPT_GRAPH))
        assert rc == mk.CKPT_EINVAL
        # the array still works after the refusals
        rc, img, _ = mk.ckpt_dump(ctx, table)
        assert rc == 0
        rc, n, _ = mk.ckpt_dump_into(ctx, table, out)
        assert rc == 0 and np.array_equal(out[:n], img.view())
        img.free()
    finally:
        mk.ckpt_ctx_destroy(ctx)
