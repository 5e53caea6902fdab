"""The batched, incremental and served forms of the benchmark (bench.py
--form ...). Each returns one JSON-ready dict. Inputs come from workloads.py
(seeded, synthetic, on the device)."""
import hashlib
import sys
import time

import numpy as np

import workloads

C = 65536


def _pct(xs, q):
    xs = sorted(xs)
    return xs[min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))] if xs else None


def _nbytes(table):
    return sum(t.numel() * t.element_size() for _, t in table)


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def piece_sha256(a, piece=256 << 20, threads=16):
    """SHA-256 over the SHA-256 digests of consecutive 256 MiB pieces of a
    uint8 array (pieces hashed on a thread pool: hashlib releases the GIL)."""
    from concurrent.futures import ThreadPoolExecutor
    spans = [(lo, min(a.size, lo + piece)) for lo in range(0, a.size, piece)] or [(0, 0)]
    with ThreadPoolExecutor(threads) as ex:
        parts = list(ex.map(lambda s: hashlib.sha256(memoryview(a[s[0]:s[1]])).digest(), spans))
    return hashlib.sha256(b"".join(parts)).hexdigest()


def incremental(args, torch, mk, link):
    """HPC image (512 fp64/int32 allocations, 40 GB, ~60 % zero chunks): a base
    dump, then 5 % of chunks rewritten in clustered runs; timed: the delta
    dump against the base, the restore of the base and the in-place restore
    of the delta."""
    total = int(40e9 * args.scale)
    table, masks = workloads.hpc_state("cuda", seed=3, total=total)
    torch.cuda.synchronize()
    N = _nbytes(table)
    ctx = mk.ckpt_ctx_create(0, max(args.budget, N + (1 << 30)))
    opts = mk.make_opts(chunk_size=C)
    rc, base, bres = mk.ckpt_dump(ctx, table, opts=opts)
    assert rc == 0
    dirty = workloads.mutate_runs(table, seed=33, chunk=C, frac=0.05, run_mean=16)
    torch.cuda.synchronize()
    t_delta, t_base, t_apply, kern = [], [], [], []
    st_delta, st_apply = [], []   # ckpt_result.ns_stage of the timed delta dumps and applies
    D = 0
    for k in range(args.warmup + args.steps):
        t0 = time.perf_counter()
        rc, delta, dres = mk.ckpt_dump(ctx, table, prev=base, opts=opts)
        t1 = time.perf_counter()
        assert rc == 0
        rc, r1 = mk.ckpt_restore(ctx, base, table, opts=opts)           # back to the base state
        t2 = time.perf_counter()
        assert rc == 0, mk.ckpt_strerror(rc)
        rc, r2 = mk.ckpt_restore(ctx, delta, table, opts=opts)          # base + delta, in place
        t3 = time.perf_counter()
        assert rc == 0, mk.ckpt_strerror(rc)
        if k >= args.warmup:
            t_delta.append(t1 - t0)
            t_base.append(t2 - t1)
            t_apply.append(t3 - t2)
            kern.append(dres.ns_kernel)
            st_delta.append(list(dres.ns_stage))
            st_apply.append(list(r2.ns_stage))
            D = dres.n_payload
            info = dres.as_dict()
        delta.free()
        _log("step %d: delta dump %.3f s, base restore %.3f s, delta apply %.3f s" % (k, t1 - t0, t2 - t1, t3 - t2))
    mk.ckpt_ctx_destroy(ctx)
    nc = info["n_chunks"]
    k_avg = sum(kern) / len(kern) / 1e9
    alg = N + D + 9 * nc
    td = sum(t_delta) / len(t_delta)
    return {
        "metric": "incremental dump / base+delta restore GB/s at 1 GPU", "form": "incremental",
        "value": round(N / td / 1e9, 3), "unit": "GB/s (logical N per delta-dump second)",
        "config": {"workload": "HPC image: %d fp64/int32 allocations, %.1f GB, %.1f%% zero chunks, %d of %d chunks "
                               "rewritten in runs (mean 16)" % (len(table), N / 1e9, 100.0 * info["n_zero"] / nc, dirty, nc),
                   "chunk": C, "N_bytes": N, "base_D_bytes": bres.n_payload, "delta_D_bytes": D,
                   "unchanged_chunks": info["n_unchanged"]},
        "delta_dump_ms_p50": round(_pct(t_delta, 50) * 1e3, 2),
        "base_restore_ms_p50": round(_pct(t_base, 50) * 1e3, 2),
        "delta_apply_ms_p50": round(_pct(t_apply, 50) * 1e3, 2),
        # medians of ckpt_result.ns_stage (ms): delta dump set-up, digest + kind
        # passes, offsets scans, gathers, host link, finalize, -, whole call;
        # delta apply validate, base check, host link, scatter + verify, -,
        # finalize, -, whole call
        "delta_dump_stage_ms_p50": [round(_pct([x[i] for x in st_delta], 50) / 1e6, 3) for i in range(8)],
        "delta_apply_stage_ms_p50": [round(_pct([x[i] for x in st_apply], 50) / 1e6, 3) for i in range(8)],
        "delta_link_GBps": round(info["link_bytes"] / td / 1e9, 2),
        "link_measured_GBps": {k: round(v, 2) for k, v in link.items()},
        "roofline": {"bound": "hbm", "achieved": round(alg / k_avg / 1e9, 1), "peak": 8000.0, "unit": "GB/s",
                     "frac": round(alg / k_avg / 1e9 / 8000.0, 4),
                     "kernel": "delta dump stage: digest+kind pass, offsets scan, gather (one window)"},
    }


def batched(args, torch, mk, link):
    """10,000 allocations log-uniform in [256 B, 256 MiB] (60 GB, ~30 % zero
    chunks): autotuned options, the graph-captured single-launch form and the
    per-allocation launch form, dump + restore each."""
    total = int(60e9 * args.scale)
    table = workloads.fragmented_state("cuda", seed=4, total=total)
    torch.cuda.synchronize()
    N = _nbytes(table)
    ctx = mk.ckpt_ctx_create(0, max(args.budget, N + (4 << 30)))
    t0 = time.perf_counter()
    rc, best, tuned_gbps = mk.ckpt_autotune(ctx, table, sample_bytes=int(4e9), flags=mk.OPT_GRAPH)
    t_tune = time.perf_counter() - t0
    assert rc == 0
    _log("autotune: chunk %d, threads %d, streams %d (%.1f GB/s on the sample, %.1f s)"
         % (best.chunk_size, best.wg_threads, best.copy_streams, tuned_gbps, t_tune))
    forms = {
        "batched": mk.make_opts(chunk_size=best.chunk_size, wg_threads=best.wg_threads,
                                copy_streams=best.copy_streams, flags=mk.OPT_GRAPH),
        "per_alloc": mk.make_opts(chunk_size=best.chunk_size, wg_threads=best.wg_threads,
                                  copy_streams=best.copy_streams, flags=mk.OPT_PER_ALLOC),
    }
    out = {}
    shas = {}
    for name, opts in forms.items():
        td, tr, kern = [], [], []
        for k in range(args.warmup + args.steps):
            t0 = time.perf_counter()
            rc, img, res = mk.ckpt_dump(ctx, table, opts=opts)
            t1 = time.perf_counter()
            assert rc == 0
            rc, rres = mk.ckpt_restore(ctx, img, table, opts=opts)
            t2 = time.perf_counter()
            assert rc == 0, mk.ckpt_strerror(rc)
            if k >= args.warmup:
                td.append(t1 - t0)
                tr.append(t2 - t1)
                kern.append(res.ns_kernel)
                info = res.as_dict()
            if k == 0:
                shas[name] = piece_sha256(img.view())   # outside the timed steps (warm-up)
            img.free()
            _log("%s step %d: dump %.3f s restore %.3f s" % (name, k, t1 - t0, t2 - t1))
        out[name] = {"dump_GBps": round(N / (sum(td) / len(td)) / 1e9, 3),
                     "restore_GBps": round(N / (sum(tr) / len(tr)) / 1e9, 3),
                     "dump_p50_ms": round(_pct(td, 50) * 1e3, 2), "dump_p99_ms": round(_pct(td, 99) * 1e3, 2),
                     "launches_per_dump": info["windows"]}
    mk.ckpt_ctx_destroy(ctx)
    b, p = out["batched"], out["per_alloc"]
    return {
        "metric": "batched dump/restore GB/s at 1 GPU vs per-allocation launches", "form": "batched",
        "value": round(2 * N / (N / b["dump_GBps"] / 1e9 + N / b["restore_GBps"] / 1e9) / 1e9, 3), "unit": "GB/s",
        "config": {"workload": "fragmented: %d allocations, %.1f GB, %d chunks (%d zero)"
                               % (len(table), N / 1e9, info["n_chunks"], info["n_zero"]),
                   "chunk": best.chunk_size, "wg_threads": best.wg_threads, "copy_streams": best.copy_streams,
                   "autotune_s": round(t_tune, 2)},
        "batched": b, "per_alloc": p,
        "dump_speedup_vs_per_alloc": round(b["dump_GBps"] / p["dump_GBps"], 3),
        "restore_speedup_vs_per_alloc": round(b["restore_GBps"] / p["restore_GBps"], 3),
        "link_measured_GBps": {k: round(v, 2) for k, v in link.items()},
        "images_sha256_identical": len(set(shas.values())) == 1, "image_sha256": shas["batched"][:16],
    }


def _rss_gb():
    """Resident host memory of this process (pinned image memory included)."""
    try:
        with open("/proc/self/status") as fh:
            for line in fh:
                if line.startswith("VmRSS:"):
                    return int(line.split()[1]) * 1024 / 1e9
    except OSError:
        pass
    return float("nan")


def _hip_last_error():
    """hipGetLastError of the calling thread (and clears it): 0 when no HIP call
    of this thread has left an error behind."""
    import ctypes
    return int(ctypes.CDLL("libamdhip64.so").hipGetLastError())


def _dev_gb(torch):
    """Free device memory and what torch holds, GB."""
    free, total = torch.cuda.mem_get_info()
    return "device free %.1f of %.1f GB, torch reserved %.1f GB" % (free / 1e9, total / 1e9,
                                                                   torch.cuda.memory_reserved() / 1e9)


def _tenant_states(torch, n_t, total, seed=5):
    """32 tenant device states, sizes log-uniform in [100 MB, 40 GB] rescaled
    to `total` bytes (the c5 draw), kinds cycling DL-like (bf16 weights
    N(0, 0.02) and fp32 optimizer state N(0, 1e-3)), HPC-like (the HPC
    image's zero-run process) and fragmented-like (random bytes with zero
    blocks)."""
    sizes = workloads.loguniform_sizes(n_t, 100 * 10**6, 40 * 10**9, int(total), 1 << 20, seed=seed)
    tenants = []
    for t, size in enumerate(sizes):
        kind = t % 3
        if kind == 0:       # per parameter a bf16 weight (2 bytes) and fp32 state (4 bytes): size / 6 of each
            gen = torch.Generator(device="cuda").manual_seed(100 + t)
            w = torch.empty(size // 6, dtype=torch.bfloat16, device="cuda").normal_(0, 0.02, generator=gen)
            m = torch.empty(size // 6, dtype=torch.float32, device="cuda").normal_(0, 1e-3, generator=gen)
            table = [(0, w), (1, m)]
        elif kind == 1:     # allocations as in the HPC image (512 for 40 GB, 1 MiB - 1 GiB)
            n = max(8, int(round(512 * size / 40e9)))
            table, _ = workloads.hpc_state("cuda", seed=100 + t, total=size, n=n, chunk=C)
        else:               # allocations as in the fragmented state (10,000 for 60 GB, 256 B - 256 MiB)
            n = max(16, int(round(10000 * size / 60e9)))
            table = workloads.fragmented_state("cuda", seed=100 + t, total=size, n=n)
        # two clustered dirty sets (5 % of chunks, runs of mean 16), used in turn
        plans = [workloads.dirty_chunks(table, seed=1000 * t + k, chunk=C, frac=0.05, run_mean=16) for k in range(2)]
        tenants.append({"table": table, "N": _nbytes(table), "kind": ("DL", "HPC", "fragmented")[kind],
                        "plans": plans, "mut": 0})
    return tenants


def _trace(rate, duration, n_t, seed=5):
    """Poisson arrivals (aggregate rate), uniform tenant; 50 % restores of the
    tenant's last image, 25 % full dumps, 25 % delta dumps (after 5 % of the
    tenant's chunks are rewritten)."""
    rng = np.random.default_rng(seed)
    out, tt = [], 0.0
    while True:
        tt += rng.exponential(1.0 / rate)
        if tt > duration:
            return out
        r = rng.random()
        out.append((tt, int(rng.integers(0, n_t)), "restore" if r < 0.5 else ("delta" if r < 0.75 else "full")))


def _lat_summary(lat):
    return {"p50_ms": round(_pct(lat, 50) * 1e3, 2) if lat else None,
            "p99_ms": round(_pct(lat, 99) * 1e3, 2) if lat else None,
            "max_ms": round(max(lat) * 1e3, 2) if lat else None}


def serve(args, torch, mk, link):
    """The served form on config c5: 32 tenants whose device states are drawn
    log-uniform in [100 MB, 40 GB] and rescaled to --serve-state bytes in
    total (host memory for the tenants' last images bounds the scale: the
    draw totals ~213 GB), a Poisson trace of --rate requests per second for
    --duration seconds. --serve-leg served: the trace through the request
    loop (16 lanes, 64 GB staging budget); baseline: the same trace through
    plain calls with per-allocation launches, one request at a time in
    arrival order (the plain per-allocation path), stopped 25 % past the
    trace's end (requests not done by then are counted at their latency
    so far, a lower bound). A tenant's requests run one at a time in both.
    Latency is arrival to completion."""
    n_t = 32
    leg = args.serve_leg
    tenants = _tenant_states(torch, n_t, args.serve_state)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()     # the generators' temporaries back to the device
    N_all = sum(t["N"] for t in tenants)
    _log("tenant states: %.1f GB; %s" % (N_all / 1e9, _dev_gb(torch)))
    # the context's own staging (base dumps, the baseline's plain calls): 8 GiB, windows of 2 GiB
    # for the large tenants; the served loop admits against its own 64 GB budget
    ctx = mk.ckpt_ctx_create(0, 8 << 30)
    opts = mk.make_opts(chunk_size=C)
    t0 = time.perf_counter()
    for t in tenants:
        rc, img, _ = mk.ckpt_dump(ctx, t["table"], opts=opts)
        assert rc == 0, mk.ckpt_strerror(rc)
        t["last"] = img
    _log("tenants ready: %.1f GB of state in %d tenants, base images %.1f GB (%.1f s), host RSS %.1f GB; %s"
         % (N_all / 1e9, n_t, sum(t["last"].nbytes() for t in tenants) / 1e9, time.perf_counter() - t0, _rss_gb(),
            _dev_gb(torch)))
    arrivals = _trace(args.rate, args.duration, n_t)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    _log("sticky HIP error of this thread after the base dumps: %d" % _hip_last_error())

    def mutate(ten):
        with torch.cuda.stream(stream):
            workloads.apply_dirty(ten["table"], ten["plans"][ten["mut"] % 2], chunk=C)
        ten["mut"] += 1
        stream.synchronize()

    lat, by_kind, fails = [], {"restore": 0, "delta": 0, "full": 0}, {}
    done_bytes, link_bytes = 0, 0
    t_start = time.perf_counter()
    last_log = t_start
    st = None
    if leg == "served":
        srv = mk.ckpt_serve_create(ctx, 16, 64 << 30)
        busy, backlog, inflight = [None] * n_t, [[] for _ in range(n_t)], {}
        ai = 0

        def submit(tid, kind, t_arr):
            ten = tenants[tid]
            if ten.get("stale"):
                kind = "full"
            if kind == "restore":
                rc, tk = mk.ckpt_serve_submit(srv, mk.REQ_RESTORE, ten["table"], img=ten["last"], tenant=tid)
            else:
                prev = None
                if kind == "delta":
                    mutate(ten)
                    prev = ten["last"]
                rc, tk = mk.ckpt_serve_submit(srv, mk.REQ_DUMP, ten["table"], prev=prev, tenant=tid)
            assert rc == 0
            busy[tid] = tk
            inflight[tk] = (tid, kind, t_arr)

        while ai < len(arrivals) or inflight:
            now = time.perf_counter() - t_start
            while ai < len(arrivals) and arrivals[ai][0] <= now:
                t_arr, tid, kind = arrivals[ai]
                ai += 1
                if busy[tid] is None:
                    submit(tid, kind, t_arr)
                else:
                    backlog[tid].append((kind, t_arr))
            for tk in list(inflight):
                done, rc, img, _ = mk.ckpt_serve_poll(srv, tk)
                if not done:
                    continue
                tid, kind, t_arr = inflight.pop(tk)
                ten = tenants[tid]
                busy[tid] = None
                lat.append(time.perf_counter() - t_start - t_arr)
                if rc != 0:
                    fails[mk.ckpt_strerror(rc)] = fails.get(mk.ckpt_strerror(rc), 0) + 1
                    if kind != "restore":
                        ten["stale"] = True
                else:
                    by_kind[kind] += 1
                    done_bytes += ten["N"]
                    if img is not None:
                        link_bytes += img.nbytes()
                        ten["last"] = img     # the old image is freed with its last reference
                        ten["stale"] = False
                    else:
                        link_bytes += ten["last"].nbytes()
                if backlog[tid]:
                    k2, ta2 = backlog[tid].pop(0)
                    submit(tid, k2, ta2)
            if time.perf_counter() - last_log > 30:
                last_log = time.perf_counter()
                _log("served: t=%.0f s, %d of %d arrived, %d done, %d in flight, host RSS %.1f GB" % (
                    now, ai, len(arrivals), len(lat), len(inflight), _rss_gb()))
            time.sleep(0.0005)
        wall = time.perf_counter() - t_start
        st = mk.ckpt_serve_stats(srv)
        mk.ckpt_serve_destroy(srv)
        unfinished = 0
    else:
        popts = mk.make_opts(chunk_size=C, flags=mk.OPT_PER_ALLOC)
        t_stop = args.duration * 1.25
        unfinished = 0
        free_at = [0.0] * n_t      # a tenant's requests one at a time (all of them are, here)
        for t_arr, tid, kind in arrivals:
            now = time.perf_counter() - t_start
            if now > t_stop:
                lat.append(now - t_arr)    # not done by the stop: latency so far (a lower bound)
                unfinished += 1
                continue
            if t_arr > now:
                time.sleep(t_arr - now)
            ten = tenants[tid]
            if ten.get("stale"):
                kind = "full"
            if kind == "restore":
                rc, _ = mk.ckpt_restore(ctx, ten["last"], ten["table"], opts=popts)
                img = None
            else:
                prev = None
                if kind == "delta":
                    mutate(ten)
                    prev = ten["last"]
                rc, img, _ = mk.ckpt_dump(ctx, ten["table"], prev=prev, opts=popts)
            lat.append(time.perf_counter() - t_start - t_arr)
            if rc != 0:
                fails[mk.ckpt_strerror(rc)] = fails.get(mk.ckpt_strerror(rc), 0) + 1
                if kind != "restore":
                    ten["stale"] = True
                continue
            by_kind[kind] += 1
            done_bytes += ten["N"]
            if img is not None:
                link_bytes += img.nbytes()
                ten["last"] = img
                ten["stale"] = False
            else:
                link_bytes += ten["last"].nbytes()
            if time.perf_counter() - last_log > 30:
                last_log = time.perf_counter()
                _log("baseline: t=%.0f s, %d of %d done, host RSS %.1f GB" % (
                    time.perf_counter() - t_start, len(lat), len(arrivals), _rss_gb()))
        wall = time.perf_counter() - t_start
    mk.ckpt_ctx_destroy(ctx)
    offered = sum(tenants[tid]["last"].nbytes() for _, tid, _ in arrivals) / max(args.duration, 1e-9)
    out = {
        "metric": "served dump/restore throughput and p50/p99 latency at 1 GPU", "form": "serve", "leg": leg,
        "value": round(done_bytes / wall / 1e9, 3), "unit": "GB/s (logical state of completed requests)",
        "config": {"workload": "%d tenants, %.1f GB of device state (log-uniform [100 MB, 40 GB] rescaled), "
                               "Poisson %.1f req/s for %.0f s" % (n_t, N_all / 1e9, args.rate, args.duration),
                   "tenant_GB": [round(t["N"] / 1e9, 2) for t in tenants], "chunk": C,
                   "staging_budget": 64 << 30, "context_staging": 8 << 30, "max_active": 16},
        "requests": len(arrivals), "completed_ok": sum(by_kind.values()), "failed": sum(fails.values()),
        "fail_codes": fails, "unfinished_at_stop": unfinished, "by_kind": by_kind,
        "latency": _lat_summary(lat), "link_GBps": round(link_bytes / wall / 1e9, 3),
        "offered_link_GBps_approx": round(offered / 1e9, 2),
        "link_measured_GBps": {k: round(v, 2) for k, v in link.items()}, "wall_s": round(wall, 2),
    }
    if st is not None:
        out["server"] = {"p50_ms": round(st.p50_ns / 1e6, 2), "p99_ms": round(st.p99_ns / 1e6, 2),
                         "mean_wait_ms": round(st.mean_wait_ns / 1e6, 2), "max_wait_ms": round(st.max_wait_ns / 1e6, 2),
                         "merged_launches": st.launches, "max_batch": st.max_batch,
                         "host_copies": st.host_copies, "host_copy_GB": round(st.host_copy_bytes / 1e9, 2)}
    return out


def ondemand(args, torch, mk, link):
    """On-demand restore on the training state (1.3B decoder, 303
    allocations, ~27 GB): the 292 bf16 parameter tensors are restored first
    (what an inference or resumed forward pass needs), the optimizer state
    and activations after; against one full restore."""
    table = workloads.training_state("cuda", seed=2)
    torch.cuda.synchronize()
    N = _nbytes(table)
    params = table[:292]
    rest = table[292:]
    ctx = mk.ckpt_ctx_create(0, max(args.budget, N + (1 << 30)))
    opts = mk.make_opts(chunk_size=C)
    rc, img, _ = mk.ckpt_dump(ctx, table, opts=opts)
    assert rc == 0
    t_full, t_params, t_rest = [], [], []
    for k in range(args.warmup + args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, _ = mk.ckpt_restore(ctx, img, table, opts=opts)
        t1 = time.perf_counter()
        assert rc == 0, mk.ckpt_strerror(rc)
        rc, rp = mk.ckpt_restore_some(ctx, img, params, opts=opts)
        t2 = time.perf_counter()
        assert rc == 0, mk.ckpt_strerror(rc)
        rc, rr = mk.ckpt_restore_some(ctx, img, rest, opts=opts)
        t3 = time.perf_counter()
        assert rc == 0, mk.ckpt_strerror(rc)
        if k >= args.warmup:
            t_full.append(t1 - t0)
            t_params.append(t2 - t1)
            t_rest.append(t3 - t2)
        _log("step %d: full %.3f s, parameters first %.3f s, rest %.3f s" % (k, t1 - t0, t2 - t1, t3 - t2))
    mk.ckpt_ctx_destroy(ctx)
    Np = _nbytes(params)
    tp = _pct(t_params, 50)
    return {
        "metric": "on-demand restore: time until the parameters are usable, at 1 GPU", "form": "ondemand",
        "value": round(tp * 1e3, 2), "unit": "ms", "higher_is_better": False,
        "config": {"workload": "decoder-1.3B training state (303 allocations)", "chunk": C, "N_bytes": N,
                   "parameter_bytes": Np, "parameter_allocations": len(params)},
        "full_restore_ms_p50": round(_pct(t_full, 50) * 1e3, 2),
        "parameters_first_ms_p50": round(tp * 1e3, 2),
        "rest_after_ms_p50": round(_pct(t_rest, 50) * 1e3, 2),
        "parameters_GBps": round(Np / tp / 1e9, 2),
        "speedup_to_parameters": round(_pct(t_full, 50) / tp, 2),
        "link_measured_GBps": {k: round(v, 2) for k, v in link.items()},
    }


def storage(args, torch, mk, link):
    """Storage leg on the training state (~27 GB). Sequential: dump, then the
    image to a file (synced); the file back into an image, then restore.
    Overlapped: ckpt_dump_file (the file written while the image is copied
    out) and ckpt_restore_file (windows uploaded while the file loads).
    Times each; the file is removed afterwards."""
    import os
    table = workloads.training_state("cuda", seed=2)
    torch.cuda.synchronize()
    N = _nbytes(table)
    ctx = mk.ckpt_ctx_create(0, max(args.budget, N + (1 << 30)))
    opts = mk.make_opts(chunk_size=C)
    path = args.path
    t = {k: [] for k in ("dump", "save", "load", "restore", "dump_file", "restore_file")}
    size = 0
    try:
        for k in range(args.warmup + args.steps):
            row = {}
            t0 = time.perf_counter()
            rc, img, _ = mk.ckpt_dump(ctx, table, opts=opts)
            t1 = time.perf_counter()
            assert rc == 0
            rc = mk.ckpt_image_save(img, path, args.io_threads)
            t2 = time.perf_counter()
            assert rc == 0, mk.ckpt_strerror(rc)
            size = img.nbytes()
            img.free()
            rc, img2 = mk.ckpt_image_load(path, args.io_threads)
            t3 = time.perf_counter()
            assert rc == 0, mk.ckpt_strerror(rc)
            rc, _ = mk.ckpt_restore(ctx, img2, table, opts=opts)
            t4 = time.perf_counter()
            assert rc == 0, mk.ckpt_strerror(rc)
            img2.free()
            os.remove(path)
            row.update(dump=t1 - t0, save=t2 - t1, load=t3 - t2, restore=t4 - t3)
            t0 = time.perf_counter()
            rc, _, _ = mk.ckpt_dump_file(ctx, table, path, opts=opts, io_threads=args.io_threads)
            t1 = time.perf_counter()
            assert rc == 0, mk.ckpt_strerror(rc)
            rc, _ = mk.ckpt_restore_file(ctx, path, table, opts=opts, io_threads=args.io_threads)
            t2 = time.perf_counter()
            assert rc == 0, mk.ckpt_strerror(rc)
            os.remove(path)
            row.update(dump_file=t1 - t0, restore_file=t2 - t1)
            if k >= args.warmup:
                for key, v in row.items():
                    t[key].append(v)
            _log("step %d: " % k + ", ".join("%s %.3f s" % (key, v) for key, v in row.items()))
    finally:
        if os.path.exists(path):
            os.remove(path)
        mk.ckpt_ctx_destroy(ctx)
    md = {key: _pct(v, 50) for key, v in t.items()}
    dump_save = md["dump"] + md["save"]
    load_restore = md["load"] + md["restore"]
    return {
        "metric": "dump-to-file and restore-from-file GB/s at 1 GPU", "form": "storage",
        "value": round(2 * N / (md["dump_file"] + md["restore_file"]) / 1e9, 3),
        "unit": "GB/s (logical, dump to file + restore from file, overlapped)",
        "config": {"workload": "decoder-1.3B training state (303 allocations)", "chunk": C, "N_bytes": N,
                   "image_bytes": size, "io_threads": args.io_threads, "path": path},
        "sequential": {"dump_ms_p50": round(md["dump"] * 1e3, 1), "save_ms_p50": round(md["save"] * 1e3, 1),
                       "load_ms_p50": round(md["load"] * 1e3, 1), "restore_ms_p50": round(md["restore"] * 1e3, 1),
                       "dump_and_save_GBps": round(N / dump_save / 1e9, 3),
                       "load_and_restore_GBps": round(N / load_restore / 1e9, 3)},
        "overlapped": {"dump_file_ms_p50": round(md["dump_file"] * 1e3, 1),
                       "restore_file_ms_p50": round(md["restore_file"] * 1e3, 1),
                       "dump_file_GBps": round(N / md["dump_file"] / 1e9, 3),
                       "restore_file_GBps": round(N / md["restore_file"] / 1e9, 3)},
        "file_write_GBps": round(size / md["save"] / 1e9, 3), "file_read_GBps": round(size / md["load"] / 1e9, 3),
        "link_measured_GBps": {k: round(v, 2) for k, v in link.items()},
    }


def codec(args, torch, mk, link):
    """Byte-plane codec on the training state (~27 GB: bf16 parameters and
    activations, fp32 master weights and moments): plain and codec dumps and
    restores of the same state, timed end to end (device stage + host link),
    with the payload each moves over the link."""
    table = workloads.training_state("cuda", seed=2)
    torch.cuda.synchronize()
    N = _nbytes(table)
    ctx = mk.ckpt_ctx_create(0, max(args.budget, N + (1 << 30)))
    plain = mk.make_opts(chunk_size=C)
    packed = mk.make_opts(chunk_size=C, flags=mk.OPT_CODEC)
    t = {k: [] for k in ("dump_plain", "dump_codec", "restore_plain", "restore_codec",
                         "kernel_dump_codec", "kernel_restore_codec", "kernel_dump_plain", "kernel_restore_plain")}
    D = {}
    n_packed = 0
    for k in range(args.warmup + args.steps):
        row = {}
        for name, opts in (("plain", plain), ("codec", packed)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, img, res = mk.ckpt_dump(ctx, table, opts=opts)
            t1 = time.perf_counter()
            assert rc == 0, mk.ckpt_strerror(rc)
            D[name] = res.n_payload
            if name == "codec":
                n_packed = res.n_packed
            row["dump_" + name] = t1 - t0
            row["kernel_dump_" + name] = res.ns_kernel * 1e-9
            rc, rres = mk.ckpt_restore(ctx, img, table, opts=opts)
            t2 = time.perf_counter()
            assert rc == 0, mk.ckpt_strerror(rc)
            row["restore_" + name] = t2 - t1
            row["kernel_restore_" + name] = rres.ns_kernel * 1e-9
            img.free()
        if k >= args.warmup:
            for key, v in row.items():
                t[key].append(v)
        _log("step %d: " % k + ", ".join("%s %.3f s" % (key, v) for key, v in row.items()))
    mk.ckpt_ctx_destroy(ctx)
    md = {key: _pct(v, 50) for key, v in t.items()}
    return {
        "metric": "dump and restore GB/s with the byte-plane codec at 1 GPU", "form": "codec",
        "value": round(2 * N / (md["dump_codec"] + md["restore_codec"]) / 1e9, 3),
        "unit": "GB/s (logical, dump + restore)",
        "config": {"workload": "decoder-1.3B training state (303 allocations)", "chunk": C, "N_bytes": N},
        "payload_plain_bytes": D["plain"], "payload_codec_bytes": D["codec"],
        "link_bytes_ratio": round(D["codec"] / D["plain"], 4), "packed_chunks": n_packed,
        "dump_ms_p50": {"plain": round(md["dump_plain"] * 1e3, 1), "codec": round(md["dump_codec"] * 1e3, 1)},
        "restore_ms_p50": {"plain": round(md["restore_plain"] * 1e3, 1), "codec": round(md["restore_codec"] * 1e3, 1)},
        "device_stage_ms_p50": {"dump_plain": round(md["kernel_dump_plain"] * 1e3, 2),
                                "dump_codec": round(md["kernel_dump_codec"] * 1e3, 2),
                                "restore_plain": round(md["kernel_restore_plain"] * 1e3, 2),
                                "restore_codec": round(md["kernel_restore_codec"] * 1e3, 2)},
        "plain_GBps": round(2 * N / (md["dump_plain"] + md["restore_plain"]) / 1e9, 3),
        "link_measured_GBps": {k: round(v, 2) for k, v in link.items()},
    }


def summary(args, torch, mk, link):
    """Compact results of the incremental, batched and served forms for the
    default bench line (one warm-up and three timed steps each; the served
    form for 20 s of arrivals per leg); a failure of one is reported in its
    entry and never stops the others."""
    import copy
    a = copy.copy(args)
    a.steps, a.warmup, a.scale = 3, 1, 1.0
    a.serve_state, a.rate, a.duration = 180e9, 20.0, 20.0
    out = {}
    for name, fn in (("incremental", incremental), ("batched", batched), ("serve", None)):
        t0 = time.perf_counter()
        try:
            if name == "serve":
                # the served configuration (32 tenants, 180 GB) for 20 s of arrivals, through the
                # request loop and through per-allocation calls one request at a time
                legs = {}
                for leg in ("served", "baseline"):
                    a.serve_leg = leg
                    r = serve(a, torch, mk, link)
                    legs[leg] = {"GBps": r["value"], "requests": r["requests"], "completed_ok": r["completed_ok"],
                                 "failed": r["failed"], "unfinished_at_stop": r["unfinished_at_stop"],
                                 "latency": r["latency"], "link_GBps": r["link_GBps"]}
                    if leg == "served":
                        legs[leg]["mean_wait_ms"] = r["server"]["mean_wait_ms"]
                        legs[leg]["max_batch"] = r["server"]["max_batch"]
                    torch.cuda.synchronize()
                    torch.cuda.empty_cache()
                out[name] = {"workload": r["config"]["workload"], **legs}
                out[name]["wall_s"] = round(time.perf_counter() - t0, 1)
                continue
            r = fn(a, torch, mk, link)
            if name == "incremental":
                out[name] = {"workload": r["config"]["workload"], "delta_D_bytes": r["config"]["delta_D_bytes"],
                             "delta_dump_ms_p50": r["delta_dump_ms_p50"],
                             "delta_link_frac": round(r["delta_link_GBps"] / link["d2h"], 4),
                             "base_restore_ms_p50": r["base_restore_ms_p50"],
                             "delta_apply_ms_p50": r["delta_apply_ms_p50"],
                             "delta_dump_stage_ms_p50": r["delta_dump_stage_ms_p50"],
                             "delta_apply_stage_ms_p50": r["delta_apply_stage_ms_p50"],
                             "dump_stage_hbm_frac": r["roofline"]["frac"]}
            else:
                out[name] = {"workload": r["config"]["workload"], "chunk": r["config"]["chunk"],
                             "batched_dump_GBps": r["batched"]["dump_GBps"],
                             "batched_restore_GBps": r["batched"]["restore_GBps"],
                             "per_alloc_dump_GBps": r["per_alloc"]["dump_GBps"],
                             "per_alloc_restore_GBps": r["per_alloc"]["restore_GBps"],
                             "dump_speedup_vs_per_alloc": r["dump_speedup_vs_per_alloc"],
                             "restore_speedup_vs_per_alloc": r["restore_speedup_vs_per_alloc"],
                             "images_sha256_identical": r["images_sha256_identical"]}
        except Exception as e:   # reported, never fatal to the headline
            out[name] = {"error": "%s: %s" % (type(e).__name__, e)}
        out[name]["wall_s"] = round(time.perf_counter() - t0, 1)
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return out
