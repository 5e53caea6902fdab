"""Benchmark: dump + restore of a synthetic device state on one MI355X.

A step is one pass of the whole hot path over the workload: a full dump of
every allocation into a verified image in pinned host memory (chunk digests,
zero detection, look-back compaction, gather, D2H ring), then a restore of
that image back into the allocations (H2D ring, scatter, verification).

Default workload: the training state of a 1.3B-parameter decoder (bf16
parameters, fp32 master weights and Adam moments, 8 GiB of bf16
activations; 303 allocations, ~27 GB), 64 KiB chunks.

Prints one JSON line. `value` = logical bytes dumped plus restored per second
of the timed steps (GB/s, 1e9). `roofline` is the dump-mode chunk kernel
against the HBM peak on its algorithmic bytes (read N, write D, 9 bytes of
tables per chunk), timed by HIP events on the stream it runs on.
`cpu_baseline` is the CPU oracle on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "dump/restore GB/s at 1 GPU (% of HBM & host-link peak); p50/p99 ckpt latency"


def pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[k]


def link_baseline(torch, nbytes=4 << 30, reps=3):
    """Pinned hipMemcpy bandwidth, D2H and H2D, measured in this run."""
    d = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    h = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
    out = {}
    for name, fn in (("d2h", lambda: h.copy_(d, non_blocking=True)), ("h2d", lambda: d.copy_(h, non_blocking=True))):
        best = 0.0
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            best = max(best, nbytes / (time.perf_counter() - t0) / 1e9)
        out[name] = best
    del d, h
    return out


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "dump_kernel_traffic_training.json")
KERNEL_SOURCES = ("paper_2502_16631_amd/csrc/kernels.hip", "paper_2502_16631_amd/csrc/kernels.h",
                  "paper_2502_16631_amd/csrc/common.h")
BUILD_SCRIPT = "paper_2502_16631_amd/build.sh"


def kernel_source_hash():
    """SHA-256 over the kernel sources and the kernels' compile flags (the
    FLAGS / KFLAGS arrays of the build script)."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    flags, inside = [], False
    with open(os.path.join(ROOT, BUILD_SCRIPT)) as fh:
        for line in fh:
            if line.startswith(("FLAGS=(", "KFLAGS=(")):
                inside = True
            if inside:
                flags.append(line)
                if line.rstrip().endswith(")"):
                    inside = False
    h.update("".join(flags).encode())
    return h.hexdigest()


def measured_traffic(workload, chunk, n_chunks):
    """HBM bytes per dump launch (FETCH_SIZE + WRITE_SIZE, each scaled by what
    the counter reads for a 1 GiB elementwise copy) from the committed
    rocprofv3 counter runs -- only if they were taken on this kernel source
    and this workload; otherwise None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    if (rec.get("kernel_source_sha256") != kernel_source_hash() or rec.get("workload") != workload
            or rec.get("chunk") != chunk or rec.get("n_chunks") != n_chunks):
        return None
    return rec.get("traffic_bytes_per_launch")


def copy_kernel_rate(torch, nbytes=4 << 30, reps=5):
    """Read + write GB/s of a plain elementwise pass (torch.bitwise_not over
    nbytes into another buffer), median of reps: the measured copy-kernel
    ceiling the dump kernel is compared with."""
    src = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    torch.bitwise_not(src, out=dst)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        torch.bitwise_not(src, out=dst)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3)
    del src, dst
    torch.cuda.synchronize()
    return 2.0 * nbytes / sorted(ts)[len(ts) // 2] / 1e9


def copy_kernel_ceiling(torch, nbytes=4 << 30, reps=3):
    """Read + write GB/s of the hand-written 128-bit copy kernels
    (csrc/copyprobe.hip: contiguous tiles per work-group with four or eight
    blocks in flight per thread, or 64 KiB chunks taken by ticket as the
    dump kernel takes them), best over a sweep of grid sizes (from one
    work-group per CU up), work-group widths, loads in flight and plain /
    non-temporal stores: the measured copy ceiling of this GPU."""
    import ctypes
    so = os.path.join(ROOT, "paper_2502_16631_amd", "libmkcopy.so")
    L = ctypes.CDLL(so)
    L.mkcopy_run.restype = ctypes.c_int
    L.mkcopy_run.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                             ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_float)]
    src = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    shapes = [(blocks, threads, nt) for blocks in (256, 512, 1024, 2048, 4096, 8192, 16384)
              for threads in (256, 512, 1024) for nt in (0, 1, 2, 3)]
    shapes += [(blocks, 512, nt) for blocks in (256, 512, 768, 1024) for nt in (4, 5)]
    best = None
    for blocks, threads, nt in shapes:
        ms = ctypes.c_float(0)
        rc = L.mkcopy_run(dst.data_ptr(), src.data_ptr(), nbytes, blocks, threads, nt, reps, ctypes.byref(ms))
        if rc != 0:
            raise RuntimeError("copy kernel: hip error %d" % rc)
        gbs = 2.0 * nbytes / (ms.value * 1e-3) / 1e9
        if best is None or gbs > best["GBps"]:
            best = {"GBps": round(gbs, 1), "pattern": "chunk tickets" if nt & 4 else "tiles", "blocks": blocks,
                    "threads": threads, "nt_stores": bool(nt & 1), "loads_in_flight": 8 if nt & 6 else 4}
    del src, dst
    torch.cuda.synchronize()
    return best


def build_workload(name, torch):
    import workloads
    if name == "training":
        return workloads.training_state("cuda", seed=2), 65536, "decoder-1.3B training state (303 allocations)"
    if name == "tiny":
        return workloads.tiny_image("cuda", seed=1), 65536, "tiny image (8 allocations, 16 MiB)"
    if name == "hpc":
        t, _ = workloads.hpc_state("cuda", seed=3)
        return t, 65536, "HPC image (512 fp64/int32 allocations, 40 GB, 60% zero chunks)"
    if name == "fragmented":
        return workloads.fragmented_state("cuda", seed=4), 65536, "fragmented (10,000 allocations, 60 GB)"
    raise SystemExit("unknown workload " + name)


def host_cpu():
    """CPU model and the number of host cores this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": len(os.sched_getaffinity(0)), "cpu_count": os.cpu_count()}


def cpu_baseline(table, chunk, budget_bytes, mk):
    """The CPU oracle (plain C, Sarwate CRC) on the first allocations of the
    workload up to budget_bytes; device bytes are copied to the host first
    (not timed). The same sample is then dumped on the GPU and the two
    images are compared: SHA-256 (over 256 MiB pieces) of the whole image,
    the full crc[] and kind[] tables."""
    import numpy as np
    from oracle import oracle
    import workloads
    from bench_forms import piece_sha256
    sample, total = [], 0
    for i, t in table:
        nb = t.numel() * t.element_size()
        if total and total + nb > budget_bytes:
            continue
        sample.append((i, t))
        total += nb
        if total >= budget_bytes:
            break
    host = workloads.host_copy(sample)
    threads = oracle.default_threads()
    t0 = time.perf_counter()
    rc, img = oracle.dump(host, chunk, threads=threads)
    dt = time.perf_counter() - t0
    assert rc == 0
    # one thread, on the first allocations up to 1 GB of the same sample
    one, n1 = [], 0
    for i, a in host:
        if n1 and n1 + a.size > 1e9:
            break
        one.append((i, a))
        n1 += a.size
    t1 = time.perf_counter()
    rc, _ = oracle.dump(one, chunk, threads=1)
    d1 = time.perf_counter() - t1
    assert rc == 0
    del host, one
    # the GPU image of the same sample, compared with the oracle's
    ctx = mk.ckpt_ctx_create(0, total + (1 << 30))
    rc, gimg, _ = mk.ckpt_dump(ctx, sample, opts=mk.make_opts(chunk_size=chunk))
    assert rc == 0, mk.ckpt_strerror(rc)
    g = gimg.view()
    n, nc = len(sample), int(np.frombuffer(img[24:32].tobytes(), np.uint64)[0])
    o_crc, o_kind = 64 + 32 * n, 64 + 32 * n + 4 * nc
    sha_o, sha_g = piece_sha256(img), piece_sha256(g)
    parity = {"sha256_equal": sha_o == sha_g and g.size == img.size, "image_bytes": int(img.size),
              "crc_equal": bool(np.array_equal(g[o_crc:o_kind], img[o_crc:o_kind])),
              "kind_equal": bool(np.array_equal(g[o_kind:o_kind + nc], img[o_kind:o_kind + nc])),
              "n_chunks": nc, "sha256": sha_o[:16]}
    gimg.free()
    mk.ckpt_ctx_destroy(ctx)
    del img
    out = {"value": round(total / dt / 1e9, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
           "sample": "full dump of %d of the workload's allocations (%.2f GB), %d threads, %.1f s"
                     % (len(sample), total / 1e9, threads, dt),
           "single_thread_GBps": round(n1 / d1 / 1e9, 3), "parity": parity}
    out.update(host_cpu())
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="training", choices=["training", "tiny", "hpc", "fragmented"])
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--budget", type=int, default=64 << 30,
                    help="device staging budget in bytes (default: one staging window for the whole image, so "
                         "the dump kernel never shares the GPU with its own host-link copies)")
    ap.add_argument("--window", type=int, default=0)
    ap.add_argument("--cpu-sample", type=float, default=16e9, help="bytes of the oracle sample (0 = skip); ~10-15 s of CPU work")
    ap.add_argument("--check", action="store_true", help="verify restored bytes after each step")
    ap.add_argument("--form", default="plain",
                    choices=["plain", "incremental", "batched", "serve", "ondemand", "storage", "codec"],
                    help="plain: full dump + restore (default); incremental: 40 GB HPC image, delta dump and "
                         "base + delta restore; batched: 10,000 allocations, graph-captured single launch vs "
                         "per-allocation launches, autotuned; serve: multi-tenant Poisson trace, p50/p99; "
                         "ondemand: parameters restored first vs one full restore; "
                         "storage: dump + image to file, file + restore; codec: plain vs byte-plane codec "
                         "dump + restore of the training state")
    ap.add_argument("--path", default="/tmp/mickpt_bench.img", help="storage: image file (removed afterwards)")
    ap.add_argument("--io-threads", type=int, default=8, help="storage: file I/O threads")
    ap.add_argument("--scale", type=float, default=1.0, help="scale the total bytes of the non-plain forms")
    ap.add_argument("--duration", type=float, default=600.0, help="serve: seconds of arrivals (10 minutes)")
    ap.add_argument("--rate", type=float, default=20.0, help="serve: aggregate requests per second")
    ap.add_argument("--serve-state", type=float, default=180e9,
                    help="serve: total bytes of the 32 tenants' device states (the log-uniform draw is rescaled "
                         "to it; the tenants' last images must fit host memory)")
    ap.add_argument("--serve-leg", default="served", choices=["served", "baseline"],
                    help="serve: the request loop, or the same trace through plain per-allocation calls one "
                         "request at a time")
    ap.add_argument("--forms", type=int, default=1,
                    help="plain form: also run the incremental and batched forms (compact, 1 + 3 steps each) and "
                         "the served form (180 GB, 20 s of arrivals, served and baseline legs) and report them "
                         "under 'forms' (0 = skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU; the library has no multi-GPU path (each GPU's allocations form an "
              "independent image), so --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2502_16631_amd import mickpt as mk

    # a plain elementwise pass over 1 GiB (reads 1 GiB, writes 1 GiB): the
    # reference that scales the HBM byte counters of a profiled run
    src = torch.zeros(1 << 30, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    torch.bitwise_not(src, out=dst)
    torch.cuda.synchronize()
    del src, dst
    torch.cuda.empty_cache()

    if args.form != "plain":
        import bench_forms
        line = {"incremental": bench_forms.incremental, "batched": bench_forms.batched,
                "serve": bench_forms.serve, "ondemand": bench_forms.ondemand,
                "storage": bench_forms.storage, "codec": bench_forms.codec}[args.form](
                    args, torch, mk, link_baseline(torch))
        print(json.dumps(line), flush=True)
        return

    link = link_baseline(torch)
    copy_gbs = copy_kernel_rate(torch)
    copy_hw = copy_kernel_ceiling(torch)
    table, chunk, wdesc = build_workload(args.workload, torch)
    if args.chunk:
        chunk = args.chunk
    torch.cuda.synchronize()
    N = sum(t.numel() * t.element_size() for _, t in table)
    ctx = mk.ckpt_ctx_create(0, args.budget)
    opts = mk.make_opts(chunk_size=chunk, window_bytes=args.window)
    ref = [(i, t.clone()) for i, t in table] if args.check else None

    dump_s, rest_s, kern_ns, kern_launches, rest_kern_ns = [], [], [], [], []
    dump_st, rest_st = [], []   # ckpt_result.ns_stage of each timed step
    info = {}

    def step(timed):
        t0 = time.perf_counter()
        rc, img, res = mk.ckpt_dump(ctx, table, opts=opts)
        t1 = time.perf_counter()
        assert rc == 0, mk.ckpt_strerror(rc)
        rc, rres = mk.ckpt_restore(ctx, img, table, opts=opts)
        t2 = time.perf_counter()
        assert rc == 0, (mk.ckpt_strerror(rc), rres.first_bad_chunk)
        if timed:
            dump_s.append(t1 - t0)
            rest_s.append(t2 - t1)
            kern_ns.append(res.ns_kernel)
            kern_launches.append(res.windows)
            rest_kern_ns.append(rres.ns_kernel)
            dump_st.append(list(res.ns_stage))
            rest_st.append(list(rres.ns_stage))
            info.update(D=res.n_payload, n_chunks=res.n_chunks, windows=res.windows, zero=res.n_zero,
                        link_bytes=res.link_bytes)
        img.free()
        if ref is not None:
            torch.cuda.synchronize()
            for (_, a), (_, b) in zip(ref, table):
                assert torch.equal(a, b)

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(True)
        print("step %d: dump %.3f s restore %.3f s" % (k, dump_s[-1], rest_s[-1]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    mk.ckpt_ctx_destroy(ctx)

    D, nc = info["D"], info["n_chunks"]
    value = 2.0 * N * args.steps / elapsed / 1e9
    dump_gbs = N / (sum(dump_s) / len(dump_s)) / 1e9
    rest_gbs = N / (sum(rest_s) / len(rest_s)) / 1e9
    alg = N + D + 9 * nc
    k_avg = sum(kern_ns) / len(kern_ns) / 1e9                     # per dump, summed over its launches
    achieved = alg / k_avg / 1e9
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": wdesc, "n_allocs": len(table), "N_bytes": N, "D_bytes": D, "chunk": chunk,
                   "n_chunks": nc, "windows": info["windows"], "staging_budget": args.budget},
        "dump_GBps": round(dump_gbs, 3),
        "restore_GBps": round(rest_gbs, 3),
        "dump_p50_ms": round(pct(dump_s, 50) * 1e3, 3),
        "dump_p99_ms": round(pct(dump_s, 99) * 1e3, 3),
        "restore_p50_ms": round(pct(rest_s, 50) * 1e3, 3),
        "restore_p99_ms": round(pct(rest_s, 99) * 1e3, 3),
        # p50 over the timed steps of each stage (ms): dump set-up, chunk
        # kernels, -, -, host link, finalize, -, whole call; restore validate,
        # base check, host link, scatter + verify, strict re-read, finalize, -,
        # whole call
        "dump_stage_ms_p50": [round(pct([st[i] for st in dump_st], 50) / 1e6, 3) for i in range(8)],
        "restore_stage_ms_p50": [round(pct([st[i] for st in rest_st], 50) / 1e6, 3) for i in range(8)],
        "link_measured_GBps": {k: round(v, 2) for k, v in link.items()},
        "dump_frac_of_link": round((info["link_bytes"] / (sum(dump_s) / len(dump_s)) / 1e9) / link["d2h"], 4),
        "restore_frac_of_link": round((info["link_bytes"] / (sum(rest_s) / len(rest_s)) / 1e9) / link["h2d"], 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(wdesc, chunk, nc),
                     "kernel": "dump-mode chunk kernel", "launches_per_dump": info["windows"],
                     "avg_launch_ms": round(k_avg / max(1, info["windows"]) * 1e3, 4),
                     "copy_kernel_GBps": copy_hw["GBps"], "copy_kernel": copy_hw,
                     "frac_of_copy_kernel": round(achieved / copy_hw["GBps"], 4),
                     "torch_bitwise_not_GBps": round(copy_gbs, 1),
                     "restore_kernel_GBps": round((D + N) / (sum(rest_kern_ns) / len(rest_kern_ns) / 1e9) / 1e9, 1)},
    }
    if args.cpu_sample > 0:
        line["cpu_baseline"] = cpu_baseline(table, chunk, args.cpu_sample, mk)
    if args.forms and args.workload == "training":
        # the incremental (HPC image) and batched (fragmented) forms, compact
        import bench_forms
        del table, ref
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        line["forms"] = bench_forms.summary(args, torch, mk, link)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
