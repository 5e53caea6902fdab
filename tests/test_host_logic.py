"""CPU tests of the GPU library's host side: the exported C ABI, and the
CRC decomposition the kernels use (emulated on the CPU with the library's own
constant builder) against the SSE4.2 hardware CRC-32C."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from testlib import golden_lines, decode_input, hw_crc32c

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2502_16631_amd", "csrc")
LIB = os.path.join(ROOT, "paper_2502_16631_amd", "libmickpt.so")
EMU_SRC = os.path.join(ROOT, "tests", "emu", "engine_emu.cpp")
EMU = os.path.join(ROOT, "tests", "emu", "libengine_emu.so")


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "mickpt.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ckpt_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def mklib():
    if not os.path.exists(LIB):
        subprocess.check_call(["bash", os.path.join(ROOT, "paper_2502_16631_amd", "build.sh")])
    return ctypes.CDLL(LIB)


def test_library_exports_every_declared_function(mklib):
    names = _declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(mklib, name), name


def test_strerror_and_host_crc(mklib):
    mklib.ckpt_strerror.restype = ctypes.c_char_p
    assert mklib.ckpt_strerror(0) == b"ok"
    assert mklib.ckpt_strerror(-4).startswith(b"image corrupt")
    mklib.ckpt_crc32c.restype = ctypes.c_uint32
    mklib.ckpt_crc32c.argtypes = [ctypes.c_char_p, ctypes.c_uint64]
    for _, inp, want in golden_lines("crc32c_vectors.txt"):
        data = decode_input(inp)
        assert mklib.ckpt_crc32c(data, len(data)) == int(want, 16)


@pytest.fixture(scope="module")
def emu():
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-msse4.2", "-shared", "-fPIC", "-I", CSRC,
                           "-o", EMU, EMU_SRC, os.path.join(CSRC, "hostmath.cpp")])
    L = ctypes.CDLL(EMU)
    L.emu_chunk_crc.restype = ctypes.c_uint32
    L.emu_chunk_crc.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, ctypes.c_int]
    L.emu_alloc_crc.restype = ctypes.c_uint32
    L.emu_alloc_crc.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int]
    L.emu_combine.restype = ctypes.c_uint32
    L.emu_combine.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64]
    L.emu_codec_crc.restype = ctypes.c_uint32
    L.emu_codec_crc.argtypes = [ctypes.c_void_p, ctypes.c_uint32]
    return L


# (C, T, K): every shape family the kernels compile, including several passes
SHAPES = [(16, 1, 1), (32, 2, 1), (64, 4, 1), (512, 32, 1), (1024, 64, 1), (2048, 64, 1), (4096, 64, 4),
          (16384, 256, 4), (32768, 256, 8), (65536, 512, 8), (65536, 1024, 4), (131072, 1024, 8),
          (262144, 1024, 8)]


@pytest.mark.parametrize("c,t,k", SHAPES)
def test_engine_decomposition_equals_crc32c(emu, c, t, k):
    rng = np.random.default_rng(c + t + k)
    for ln in sorted({c, c - 1, c - 15, c // 2 + 3, 17, 16, 15, 1}):
        if ln <= 0 or ln > c:
            continue
        data = rng.integers(0, 256, ln, dtype=np.uint8)
        assert emu.emu_chunk_crc(data.ctypes.data, ln, c, t, k) == hw_crc32c(data), (c, t, k, ln)


@pytest.mark.parametrize("c", [4096, 8192, 16384, 32768, 65536])
def test_codec_decode_digest_equals_crc32c(emu, c):
    """The codec decode kernel's digest (per-lane slice-by-16 over consecutive
    rows, lane constants, preset term; the library's own constant builder)
    is CRC-32C: checked against the hardware instruction."""
    rng = np.random.default_rng(c)
    for data in (rng.integers(0, 256, c, dtype=np.uint8), np.zeros(c, np.uint8),
                 (rng.standard_normal(c // 4) * 0.02).astype(np.float32).view(np.uint8)):
        assert emu.emu_codec_crc(data.ctypes.data, c) == hw_crc32c(data), c


def test_combine_reproduces_whole_allocation_crc(emu):
    rng = np.random.default_rng(5)
    for c in (16, 64, 4096):
        for size in (1, c - 1, c, c + 1, 5 * c + 7, 300 * c + 3):
            data = rng.integers(0, 256, size, dtype=np.uint8)
            crcs = np.array([hw_crc32c(data[i:i + c]) for i in range(0, size, c)], dtype=np.uint32)
            for threads in (1, 3, 256):
                assert emu.emu_alloc_crc(crcs.ctypes.data, size, c, threads) == hw_crc32c(data)
    a, b = b"hello ", b"world"
    assert emu.emu_combine(hw_crc32c(a), hw_crc32c(b), len(b)) == hw_crc32c(a + b)


def test_image_save_load_round_trip(mklib, tmp_path):
    """Image files: save writes exactly the image's bytes, load reads them
    back and validates them; corrupt, truncated and missing files are
    rejected. Images come from the CPU oracle (on a machine without a GPU the
    library keeps them in pageable memory). Sizes cross several 64 MiB I/O
    pieces and leave an unaligned tail."""
    import sys
    sys.path.insert(0, ROOT)
    from oracle import oracle as corc
    rng = np.random.default_rng(5)
    sizes = [0, 1, 5000, 65536, 70_000_001, 80 << 20]
    allocs = [(i + 1, rng.integers(0, 256, size=s, dtype=np.uint8)) for i, s in enumerate(sizes)]
    allocs[3][1][:] = 0
    rc, img = corc.dump(allocs, 65536)
    assert rc == 0 and img.size > (128 << 20) and img.size % 4096
    vp = ctypes.c_void_p
    mklib.ckpt_image_import.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(vp)]
    mklib.ckpt_image_save.argtypes = [vp, ctypes.c_char_p, ctypes.c_uint32]
    mklib.ckpt_image_load.argtypes = [ctypes.c_char_p, ctypes.c_uint32, ctypes.POINTER(vp)]
    mklib.ckpt_image_bytes.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_uint64)]
    mklib.ckpt_image_free.argtypes = [vp]
    h = vp()
    assert mklib.ckpt_image_import(img.ctypes.data, img.size, ctypes.byref(h)) == 0
    path = str(tmp_path / "state.img").encode()
    assert mklib.ckpt_image_save(h, path, 3) == 0
    with open(path, "rb") as f:
        assert f.read() == img.tobytes()
    h2 = vp()
    assert mklib.ckpt_image_load(path, 2, ctypes.byref(h2)) == 0
    p, n = vp(), ctypes.c_uint64()
    assert mklib.ckpt_image_bytes(h2, ctypes.byref(p), ctypes.byref(n)) == 0
    assert ctypes.string_at(p.value, n.value) == img.tobytes()
    mklib.ckpt_image_free(h2)
    # a flipped header byte, a flipped tables byte, a truncated file, no file
    raw = bytearray(img.tobytes())
    for pos in (20, 64 + 3):
        bad = bytearray(raw)
        bad[pos] ^= 0x40
        with open(path, "wb") as f:
            f.write(bad)
        h3 = vp()
        assert mklib.ckpt_image_load(path, 4, ctypes.byref(h3)) == -4 and not h3.value
    with open(path, "wb") as f:
        f.write(raw[:len(raw) // 2])
    h3 = vp()
    assert mklib.ckpt_image_load(path, 4, ctypes.byref(h3)) == -4
    assert mklib.ckpt_image_load(str(tmp_path / "missing.img").encode(), 4, ctypes.byref(h3)) == -8
    assert mklib.ckpt_image_save(h, str(tmp_path / "no" / "dir.img").encode(), 2) == -8
    mklib.ckpt_image_free(h)


def test_codec_images_import_and_merge_on_the_host(mklib):
    """The library's host-side image handling of the codec layout: import
    validates oracle-made codec images (and rejects table corruptions the
    oracle rejects), and ckpt_merge of codec / plain bases and deltas is
    byte-identical to the oracle's merge."""
    import sys
    sys.path.insert(0, ROOT)
    from oracle import oracle as corc
    vp = ctypes.c_void_p
    mklib.ckpt_image_import.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(vp)]
    mklib.ckpt_image_bytes.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_uint64)]
    mklib.ckpt_image_free.argtypes = [vp]
    mklib.ckpt_merge.argtypes = [vp, vp, ctypes.POINTER(vp)]

    def imp(a):
        h = vp()
        rc = mklib.ckpt_image_import(a.ctypes.data, a.size, ctypes.byref(h))
        return rc, h

    def bytes_of(h):
        p, n = vp(), ctypes.c_uint64()
        assert mklib.ckpt_image_bytes(h, ctypes.byref(p), ctypes.byref(n)) == 0
        return ctypes.string_at(p, n.value)

    c = 4096
    rng = np.random.default_rng(9)
    bf16 = ((rng.standard_normal(20 * c) * 0.02).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    base = [(1, bf16.view(np.uint8).copy()),
            (2, (rng.standard_normal(3 * c) * 1e-3).astype(np.float32).view(np.uint8)),
            (3, rng.integers(0, 256, 2 * c + 7, dtype=np.uint8)),
            (4, np.zeros(3 * c, np.uint8))]
    new = [(i, a.copy()) for i, a in base]
    new[0][1][3 * c:5 * c] = rng.integers(0, 256, 2 * c, dtype=np.uint8)
    new[3][1][c:2 * c] = 9
    for base_codec in (True, False):
        rc, b = corc.dump(base, c, codec=base_codec)
        rc, d = corc.dump(new, c, prev=b, codec=True)
        rc, want = corc.merge(b, d)
        assert rc == 0
        rcb, hb = imp(b)
        rcd, hd = imp(d)
        assert rcb == 0 and rcd == 0
        hm = vp()
        assert mklib.ckpt_merge(hb, hd, ctypes.byref(hm)) == 0
        assert bytes_of(hm) == want.tobytes()
        for h in (hb, hd, hm):
            mklib.ckpt_image_free(h)
    # table corruptions of a codec image: a record length, a kind, the flag
    rc, img = corc.dump(base, c, codec=True)
    n, nc = 4, sum((a.size + c - 1) // c for _, a in base)
    for pos in (64 + 32 * n + 4 * nc + 4, 64 + 32 * n + 8 * nc + 1, 12):
        bad = img.copy()
        bad[pos] ^= 0x04
        want = corc.parse(bad)[0]
        rc, h = imp(bad)
        assert rc == want == -4, pos


def test_pinned_digest_tables_are_never_evicted():
    """Eviction of resident digest tables (the library's own rule, compiled
    for the CPU): the victim is the least recently used table no request has
    pinned; with every table pinned nothing is evicted."""
    so = os.path.join(ROOT, "tests", "emu", "libdigest_policy.so")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-D__HIP_PLATFORM_AMD__",
                           "-I/opt/rocm/include", "-I", CSRC, "-o", so,
                           os.path.join(ROOT, "tests", "emu", "digest_policy.cpp")])
    L = ctypes.CDLL(so)
    L.emu_digest_victim.restype = ctypes.c_uint64
    L.emu_digest_victim.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int]
    rng = np.random.default_rng(40)
    for trial in range(300):
        n = int(rng.integers(1, 40))
        uids = rng.choice(np.arange(1, 10**6, dtype=np.uint64), n, replace=False)
        last = rng.permutation(n).astype(np.uint64) + 1
        pins = (rng.random(n) < rng.random()).astype(np.uint32) * rng.integers(1, 4, n).astype(np.uint32)
        v = L.emu_digest_victim(uids.ctypes.data, last.ctypes.data, pins.ctypes.data, n)
        free = pins == 0
        if not free.any():
            assert v == 0
        else:
            i = int(np.nonzero(uids == v)[0][0])
            assert pins[i] == 0 and last[i] == last[free].min()


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: asked for more, it exits with status 2 and
    says why, before touching any device."""
    import sys
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and "--gpus 2" in p.stderr
    assert p.stdout == ""
