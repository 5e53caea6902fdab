"""Seeded synthetic device states shaped like the paper's workloads.

Input generators only: this module holds none of the checkpoint arithmetic
and is shared by the tests (GPU path and oracle see the same bytes) and the
benchmark. The paper's own workloads (GPT-2 / Llama / BERT training state,
ROCm HPC micro-benchmarks; section 5, "Workloads and micro-benchmarks") are
not available, so these stand in for them with the shapes of its Tables 4
and 5: training state dominated by parameters, optimizer state and
activations; HPC images of many fp64 / int32 arrays with large zero regions.

Every generator returns a list of (id, tensor) on the given device.
"""
import math

import numpy as np
import torch


def loguniform_sizes(n, lo, hi, total, granule, seed):
    """Sizes drawn log-uniform in [lo, hi], rescaled to sum to `total`:
    repeat s <- clamp(s * total / sum(s), lo, hi) until within 0.1 %, then
    round down to a multiple of `granule` (never below lo)."""
    rng = np.random.default_rng(seed)
    s = np.exp(rng.uniform(math.log(lo), math.log(hi), n))
    for _ in range(1000):
        if abs(s.sum() - total) / total < 1e-3:
            break
        s = np.clip(s * total / s.sum(), lo, hi)
    s = np.maximum((s // granule) * granule, lo)
    return [int(x) for x in s]


def _bytes_uniform(n, gen, device):
    return torch.randint(0, 256, (n,), dtype=torch.uint8, device=device, generator=gen)


def tiny_image(device="cuda", seed=1, total=16 << 20, n=8):
    """8 uint8 allocations, sizes log-uniform in [4 KiB, 4 MiB] rescaled to
    16 MiB, uniform random bytes."""
    sizes = loguniform_sizes(n, 4 << 10, 4 << 20, total, 256, seed)
    gen = torch.Generator(device=device).manual_seed(seed)
    return [(1000 + i, _bytes_uniform(s, gen, device)) for i, s in enumerate(sizes)]


def decoder_param_shapes(layers=24, d=2048, ffn=8192, vocab=50257, ctx=2048):
    """Parameter tensors of a GPT-style decoder: token and position
    embeddings, per layer qkv / out / up / down projections with biases and
    two layer norms, final layer norm."""
    shapes = [("wte", (vocab, d)), ("wpe", (ctx, d))]
    for i in range(layers):
        shapes += [("h%d.qkv_w" % i, (3 * d, d)), ("h%d.qkv_b" % i, (3 * d,)),
                   ("h%d.o_w" % i, (d, d)), ("h%d.o_b" % i, (d,)),
                   ("h%d.up_w" % i, (ffn, d)), ("h%d.up_b" % i, (ffn,)),
                   ("h%d.down_w" % i, (d, ffn)), ("h%d.down_b" % i, (d,)),
                   ("h%d.ln1_w" % i, (d,)), ("h%d.ln1_b" % i, (d,)),
                   ("h%d.ln2_w" % i, (d,)), ("h%d.ln2_b" % i, (d,))]
    shapes += [("lnf_w", (d,)), ("lnf_b", (d,))]
    return shapes


def training_state(device="cuda", seed=2, layers=24, d=2048, ffn=8192, vocab=50257, ctx=2048,
                   act_buffers=8, act_bytes=1 << 30):
    """Training state of a 1.3B-parameter decoder (Table 4's GPU share):
    bf16 parameters N(0, 0.02); three flat fp32 buffers -- master weights
    (the same draws in fp32), Adam m and v ~ N(0, 1e-3); 8 x 1 GiB bf16
    activation buffers N(0, 1). 292 + 3 + 8 = 303 allocations."""
    gen = torch.Generator(device=device).manual_seed(seed)
    shapes = decoder_param_shapes(layers, d, ffn, vocab, ctx)
    n_params = sum(int(np.prod(s)) for _, s in shapes)
    master = torch.empty(n_params, dtype=torch.float32, device=device)
    master.normal_(0.0, 0.02, generator=gen)
    out = []
    off = 0
    for i, (_, s) in enumerate(shapes):
        k = int(np.prod(s))
        out.append((i, master[off:off + k].to(torch.bfloat16).view(s).clone()))
        off += k
    m = torch.empty_like(master).normal_(0.0, 1e-3, generator=gen)
    v = torch.empty_like(master).normal_(0.0, 1e-3, generator=gen)
    out += [(len(shapes), master), (len(shapes) + 1, m), (len(shapes) + 2, v)]
    for j in range(act_buffers):
        a = torch.empty(act_bytes // 2, dtype=torch.bfloat16, device=device)
        a.normal_(0.0, 1.0, generator=gen)
        out.append((len(shapes) + 3 + j, a))
    return out


def _geom(rng, mean):
    return int(rng.geometric(1.0 / mean))


def hpc_state(device="cuda", seed=3, total=40 * 10**9, n=512, chunk=65536, zero_run=24, data_run=16):
    """HPC-style state (Table 5): n fp64 / int32 allocations (coin p = 0.5),
    sizes log-uniform in [1 MiB, 1 GiB] rescaled to `total`; at chunk
    granularity a two-state run process makes zero runs (geometric, mean 24)
    and data runs (mean 16): about 60 % of chunks are all zero. Returns the
    table and, per allocation, the boolean data-chunk mask."""
    sizes = loguniform_sizes(n, 1 << 20, 1 << 30, total, 8, seed)
    rng = np.random.default_rng(seed)
    gen = torch.Generator(device=device).manual_seed(seed)
    out, masks = [], []
    zero_state = bool(rng.random() < 0.6)
    left = _geom(rng, zero_run if zero_state else data_run)
    for i, size in enumerate(sizes):
        is_f64 = bool(rng.random() < 0.5)
        nk = (size + chunk - 1) // chunk
        mask = np.zeros(nk, dtype=bool)
        for k in range(nk):
            if left == 0:
                zero_state = not zero_state
                left = _geom(rng, zero_run if zero_state else data_run)
            mask[k] = not zero_state
            left -= 1
        buf = torch.zeros(size, dtype=torch.uint8, device=device)
        _fill_chunks(buf, mask, chunk, is_f64, gen)
        out.append((i, buf))
        masks.append(mask)
    return out, masks


def _fill_chunks(buf, mask, chunk, is_f64, gen):
    """Fresh values of the allocation's dtype in the chunks selected by mask
    (runs of chunks are filled with one call each)."""
    nk = mask.size
    k = 0
    while k < nk:
        if not mask[k]:
            k += 1
            continue
        j = k
        while j < nk and mask[j]:
            j += 1
        lo, hi = k * chunk, min(j * chunk, buf.numel())
        view = buf[lo:hi]
        if is_f64:
            n8 = (hi - lo) // 8
            if n8:
                view[:n8 * 8].view(torch.float64).normal_(0.0, 1.0, generator=gen)
            if (hi - lo) % 8:
                view[n8 * 8:].copy_(torch.randint(1, 256, ((hi - lo) % 8,), dtype=torch.uint8,
                                                  device=buf.device, generator=gen))
        else:
            n4 = (hi - lo) // 4
            if n4:
                view[:n4 * 4].view(torch.int32).random_(generator=gen)
            if (hi - lo) % 4:
                view[n4 * 4:].copy_(torch.randint(1, 256, ((hi - lo) % 4,), dtype=torch.uint8,
                                                  device=buf.device, generator=gen))
        k = j


def mutate_runs(table, seed=33, chunk=65536, frac=0.05, run_mean=16):
    """In place: pick run starts uniformly over all chunks and modify runs of
    geometric length (mean 16) with fresh bytes until `frac` of the chunks
    are modified. Returns the number of modified chunks."""
    rng = np.random.default_rng(seed)
    gen = torch.Generator(device=table[0][1].device).manual_seed(seed)
    counts = [(t.numel() * t.element_size() + chunk - 1) // chunk for _, t in table]
    starts = np.cumsum([0] + counts)
    total = int(starts[-1])
    dirty = np.zeros(total, dtype=bool)
    target = int(frac * total)
    while dirty.sum() < target:
        s = int(rng.integers(0, total))
        L = _geom(rng, run_mean)
        dirty[s:min(total, s + L)] = True
    for a, (_, t) in enumerate(table):
        b = t.view(-1).view(torch.uint8) if t.dtype != torch.uint8 else t.view(-1)
        m = dirty[starts[a]:starts[a + 1]]
        k = 0
        while k < m.size:
            if not m[k]:
                k += 1
                continue
            j = k
            while j < m.size and m[j]:
                j += 1
            lo, hi = k * chunk, min(j * chunk, b.numel())
            b[lo:hi] = torch.randint(0, 256, (hi - lo,), dtype=torch.uint8, device=b.device, generator=gen)
            k = j
    return int(dirty.sum())


def dirty_chunks(table, seed, chunk=65536, frac=0.05, run_mean=16):
    """Chunks to rewrite, as in mutate_runs (run starts uniform over all
    chunks, geometric run lengths, until `frac` of the chunks are covered),
    restricted to full-length chunks: per allocation a list of runs
    (first chunk, end chunk) for apply_dirty."""
    rng = np.random.default_rng(seed)
    counts = [(t.numel() * t.element_size() + chunk - 1) // chunk for _, t in table]
    starts = np.cumsum([0] + counts)
    total = int(starts[-1])
    dirty = np.zeros(total, dtype=bool)
    target, covered = int(frac * total), 0
    while covered < target:
        s = int(rng.integers(0, total))
        e = min(total, s + _geom(rng, run_mean))
        covered += int((~dirty[s:e]).sum())
        dirty[s:e] = True
    out = []
    for a, (_, t) in enumerate(table):
        nfull = (t.numel() * t.element_size()) // chunk
        m = np.concatenate([[False], dirty[starts[a]:starts[a] + nfull], [False]]).astype(np.int8)
        edges = np.flatnonzero(np.diff(m))
        out.append([(int(lo), int(hi)) for lo, hi in zip(edges[0::2], edges[1::2])])
    return out


def apply_dirty(table, plan, chunk=65536):
    """Rewrite the planned runs of chunks in place: every byte of each is
    incremented (mod 256), so each planned chunk changes (one elementwise
    operation per run, issued on the current stream)."""
    for (_, t), runs in zip(table, plan):
        if not runs:
            continue
        b = t.view(-1).view(torch.uint8) if t.dtype != torch.uint8 else t.view(-1)
        for lo, hi in runs:
            b[lo * chunk:hi * chunk] += 1


def fragmented_state(device="cuda", seed=4, total=60 * 10**9, n=10000, zero_block=256 << 10, zero_p=0.3):
    """Allocator-like fragmentation: n allocations, sizes log-uniform in
    [256 B, 256 MiB] rescaled to `total`, random bytes, zero regions as
    256 KiB-aligned blocks with probability 0.3 (whole allocation when it is
    smaller than a block)."""
    sizes = loguniform_sizes(n, 256, 256 << 20, total, 256, seed)
    rng = np.random.default_rng(seed)
    gen = torch.Generator(device=device).manual_seed(seed)
    out = []
    for i, size in enumerate(sizes):
        buf = _bytes_uniform(size, gen, device)
        if size < zero_block:
            if rng.random() < zero_p:
                buf.zero_()
        else:
            nb = (size + zero_block - 1) // zero_block
            z = np.nonzero(rng.random(nb) < zero_p)[0]
            for b in z:
                buf[b * zero_block:min(size, (b + 1) * zero_block)] = 0
        out.append((i, buf))
    return out


def host_copy(table):
    """(id, numpy uint8 array) copies of a device table, for the oracle."""
    out = []
    for i, t in table:
        b = t.reshape(-1).view(torch.uint8) if t.numel() else torch.zeros(0, dtype=torch.uint8)
        out.append((i, b.cpu().numpy()))
    return out
