"""Served form on the GPU: requests submitted together (and so batched into
shared launches) give the same results as each request alone, byte for
byte, and as the CPU oracle."""
import os
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

pytestmark = pytest.mark.gpu
DEV = "cuda"
C = 65536


def _tenant_table(seed, n, max_chunks):
    rng = np.random.default_rng(seed)
    gen = torch.Generator(device=DEV).manual_seed(seed)
    table = []
    for a in range(n):
        size = int(rng.integers(0, max_chunks * C)) if rng.random() > 0.1 else int(rng.integers(0, 100))
        t = torch.randint(0, 256, (size,), dtype=torch.uint8, device=DEV, generator=gen)
        for lo in range(0, size, C):
            if rng.random() < 0.3:
                t[lo:lo + C] = 0
        table.append((seed * 1000 + a, t))
    return table


def _wait(srv, tickets, timeout=120):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for k, tk in tickets.items():
            if k in out:
                continue
            done, rc, img, lat = mk.ckpt_serve_poll(srv, tk)
            if done:
                out[k] = (rc, img, lat)
        assert time.time() - t0 < timeout, "serving requests did not complete"
        time.sleep(0.001)
    return out


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = mk.ckpt_ctx_create(0, 1 << 30)
    yield c
    mk.ckpt_ctx_destroy(c)


def test_mixed_requests_equal_each_request_alone(ctx):
    os.environ["MICKPT_SERVE_WINDOW"] = str(1 << 20)     # 16 chunks per window: many merged launches
    tenants = {k: _tenant_table(10 + k, 6 + k, 12 + 6 * k) for k in range(6)}
    opts = mk.make_opts(chunk_size=C)
    # alone: plain-path base images, then new states and their plain full / delta images
    base = {}
    for k, tab in tenants.items():
        rc, img, _ = mk.ckpt_dump(ctx, tab, opts=opts)
        assert rc == 0
        base[k] = img
    for k, tab in tenants.items():
        workloads.mutate_runs(tab, seed=50 + k, chunk=C, frac=0.1, run_mean=2)
    alone_full, alone_delta = {}, {}
    for k, tab in tenants.items():
        alone_full[k] = mk.ckpt_dump(ctx, tab, opts=opts)[1]
        alone_delta[k] = mk.ckpt_dump(ctx, tab, prev=base[k], opts=opts)[1]
    # restore targets: fresh buffers for the base images
    targets = {k: [(i, torch.full_like(t, 0x33)) for i, t in tab] for k, tab in tenants.items()}

    srv = mk.ckpt_serve_create(ctx, max_active=8, budget=1 << 30)
    try:
        tickets = {}
        for k, tab in tenants.items():
            tickets[("full", k)] = mk.ckpt_serve_submit(srv, mk.REQ_DUMP, tab, tenant=k)[1]
            tickets[("delta", k)] = mk.ckpt_serve_submit(srv, mk.REQ_DUMP, tab, prev=base[k], tenant=k)[1]
            tickets[("restore", k)] = mk.ckpt_serve_submit(srv, mk.REQ_RESTORE, targets[k], img=base[k], tenant=k)[1]
        res = _wait(srv, tickets)
        st = mk.ckpt_serve_stats(srv)
    finally:
        mk.ckpt_serve_destroy(srv)
    assert st.completed == len(tickets) and st.failed == 0
    assert st.max_batch >= 2, "requests never shared a launch"
    for k, tab in tenants.items():
        rc, img, _ = res[("full", k)]
        assert rc == 0 and np.array_equal(img.view(), alone_full[k].view())
        rc, oimg = corc.dump(workloads.host_copy(tab), C)
        assert np.array_equal(img.view(), oimg)
        rc, img, _ = res[("delta", k)]
        assert rc == 0 and np.array_equal(img.view(), alone_delta[k].view())
        rc, _, _ = res[("restore", k)]
        assert rc == 0
    # restored buffers hold the base states: re-dump them and compare with the base images
    torch.cuda.synchronize()
    for k in tenants:
        rc, img, _ = mk.ckpt_dump(ctx, targets[k], opts=opts)
        assert rc == 0 and np.array_equal(img.view(), base[k].view())


def test_serving_errors_and_deadline(ctx):
    os.environ["MICKPT_SERVE_WINDOW"] = str(1 << 20)
    tab = _tenant_table(77, 4, 8)
    rc, img, _ = mk.ckpt_dump(ctx, tab, opts=mk.make_opts(chunk_size=C))
    assert rc == 0
    srv = mk.ckpt_serve_create(ctx, max_active=2, budget=1 << 30)
    try:
        wrong = [(i + 1, t) for i, t in tab]
        t1 = mk.ckpt_serve_submit(srv, mk.REQ_RESTORE, wrong, img=img)[1]
        past = time.clock_gettime_ns(time.CLOCK_MONOTONIC) - 1
        t2 = mk.ckpt_serve_submit(srv, mk.REQ_DUMP, tab, deadline_ns=past)[1]
        res = _wait(srv, {"mismatch": t1, "late": t2})
    finally:
        mk.ckpt_serve_destroy(srv)
    assert res["mismatch"][0] == mk.CKPT_EMISMATCH
    assert res["late"][0] == mk.CKPT_ETIMEOUT


def test_pageable_images_through_host_workers(ctx):
    """Every image in pageable host memory (MICKPT_HOST_PAGEABLE): the served
    loop moves payload windows between the device and those images on its
    host worker threads (dumps of several windows reuse each staging slot
    only once the worker has copied it out; restores launch a window only
    once its payload is up). Images equal the plain path's byte for byte and
    restores write back the base states."""
    os.environ["MICKPT_SERVE_WINDOW"] = str(1 << 20)
    os.environ["MICKPT_HOST_PAGEABLE"] = "1"
    try:
        tenants = {k: _tenant_table(40 + k, 4 + k, 20 + 8 * k) for k in range(4)}
        opts = mk.make_opts(chunk_size=C)
        base = {k: mk.ckpt_dump(ctx, tab, opts=opts)[1] for k, tab in tenants.items()}
        for k, tab in tenants.items():
            workloads.mutate_runs(tab, seed=60 + k, chunk=C, frac=0.2, run_mean=3)
        alone_full = {k: mk.ckpt_dump(ctx, tab, opts=opts)[1] for k, tab in tenants.items()}
        alone_delta = {k: mk.ckpt_dump(ctx, tab, prev=base[k], opts=opts)[1] for k, tab in tenants.items()}
        targets = {k: [(i, torch.full_like(t, 0x44)) for i, t in tab] for k, tab in tenants.items()}
        srv = mk.ckpt_serve_create(ctx, max_active=6, budget=1 << 30)
        try:
            tickets = {}
            for k, tab in tenants.items():
                tickets[("full", k)] = mk.ckpt_serve_submit(srv, mk.REQ_DUMP, tab, tenant=k)[1]
                tickets[("delta", k)] = mk.ckpt_serve_submit(srv, mk.REQ_DUMP, tab, prev=base[k], tenant=k)[1]
                tickets[("restore", k)] = mk.ckpt_serve_submit(srv, mk.REQ_RESTORE, targets[k], img=base[k],
                                                               tenant=k)[1]
            res = _wait(srv, tickets)
            st = mk.ckpt_serve_stats(srv)
        finally:
            mk.ckpt_serve_destroy(srv)
        assert st.completed == len(tickets) and st.failed == 0 and st.host_copies > 0
        for k in tenants:
            for kind, want in (("full", alone_full[k]), ("delta", alone_delta[k])):
                rc, img, _ = res[(kind, k)]
                assert rc == 0 and np.array_equal(img.view(), want.view()), (kind, k)
            assert res[("restore", k)][0] == 0
        torch.cuda.synchronize()
        for k in tenants:
            rc, img, _ = mk.ckpt_dump(ctx, targets[k], opts=opts)
            assert rc == 0 and np.array_equal(img.view(), base[k].view())
    finally:
        del os.environ["MICKPT_HOST_PAGEABLE"]
