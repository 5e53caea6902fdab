"""GPU tests of concurrent use from host threads: several threads calling
dump and restore on one shared context (its lock serializes the calls) or on
contexts of their own (which run side by side on the device) get the
oracle's images -- plain, codec and delta -- and restore exactly the dumped
bytes, round after round."""
import os
import sys
import threading

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
C = 65536
THREADS = 4


def make_table(seed):
    """~24 MB: random bytes with a 1 MiB zero region in the larger
    allocations, bf16 weights (PACKED under the codec), one empty
    allocation, ragged sizes."""
    gen = torch.Generator(device=DEV).manual_seed(seed)
    sizes = [(8 << 20) + 13 * seed, 3 << 20, 5 * C, 0, (12 << 20) + 1]
    out = []
    for k, n in enumerate(sizes):
        if k == 1:
            t = (torch.randn(n // 2, generator=gen, device=DEV) * 0.02).to(torch.bfloat16).view(torch.uint8)
        else:
            t = torch.randint(0, 256, (n,), dtype=torch.uint8, device=DEV, generator=gen) if n else \
                torch.zeros(0, dtype=torch.uint8, device=DEV)
        if n > (1 << 20):
            t[n // 3:n // 3 + (1 << 20)] = 0
        out.append((100 * seed + k, t))
    return out


def worker(ctx, table, want, errors):
    """Round after round: a full dump (plain, codec, plain), its restore, and
    at the end a delta dump of a changed copy of the state against the last
    image."""
    try:
        img = None
        for r, codec in enumerate((False, True, False)):
            if img is not None:
                img.free()
            opts = mk.make_opts(chunk_size=C, flags=mk.OPT_CODEC if codec else 0)
            rc, img, res = mk.ckpt_dump(ctx, table, opts=opts)
            assert rc == 0, mk.ckpt_strerror(rc)
            assert np.array_equal(img.view(), want["codec" if codec else "plain"])
            assert (res.n_packed > 0) == codec
            targets = [(i, torch.full_like(t, 0x5A) if t.numel() else t.clone()) for i, t in table]
            torch.cuda.synchronize()
            rc, rres = mk.ckpt_restore(ctx, img, targets)
            assert rc == 0, (mk.ckpt_strerror(rc), rres.first_bad_chunk)
            torch.cuda.synchronize()
            for (_, a), (_, b) in zip(table, targets):
                assert torch.equal(a, b)
        rc, dimg, dres = mk.ckpt_dump(ctx, want["changed"], prev=img, opts=mk.make_opts(chunk_size=C))
        assert rc == 0 and dres.n_unchanged > 0, mk.ckpt_strerror(rc)
        assert np.array_equal(dimg.view(), want["delta"])
        dimg.free()
        img.free()
    except BaseException as e:   # reported by the main thread
        errors.append(e)


def run_threads(ctxs):
    tables = [make_table(s) for s in range(1, THREADS + 1)]
    wants = []
    for s, t in enumerate(tables):
        changed = [(i, x.clone()) for i, x in t]
        workloads.mutate_runs(changed, seed=50 + s, chunk=C, frac=0.1, run_mean=4)
        torch.cuda.synchronize()
        h = workloads.host_copy(t)
        rc, plain = corc.dump(h, C)
        rc2, codec = corc.dump(h, C, codec=True)
        rc3, delta = corc.dump(workloads.host_copy(changed), C, prev=plain)
        assert rc == rc2 == rc3 == 0
        wants.append({"plain": plain, "codec": codec, "changed": changed, "delta": delta})
    errors = []
    ths = [threading.Thread(target=worker, args=(ctxs[k % len(ctxs)], tables[k], wants[k], errors))
           for k in range(THREADS)]
    for th in ths:
        th.start()
    for th in ths:
        th.join(timeout=300)
    assert not any(th.is_alive() for th in ths)
    if errors:
        raise errors[0]


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_threads_share_one_context(gpu):
    c = mk.ckpt_ctx_create(0, 1 << 30)
    try:
        run_threads([c])
    finally:
        mk.ckpt_ctx_destroy(c)


def test_threads_with_contexts_of_their_own(gpu):
    cs = [mk.ckpt_ctx_create(0, 256 << 20) for _ in range(THREADS)]
    try:
        run_threads(cs)
    finally:
        for c in cs:
            mk.ckpt_ctx_destroy(c)
