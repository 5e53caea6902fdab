"""ctypes wrapper of the plain-C oracle (ckpt_oracle.c).

TEST INFRASTRUCTURE ONLY. Only tests/, __graft_entry__.smoke() and bench.py's
CPU-baseline leg may import this module; the product path never does. It
imports nothing from the GPU package, and the GPU package imports nothing
from here.

Images and allocations are numpy uint8 arrays (or bytes). Return codes are
those of the image format: 0 OK, -1 EINVAL, -2 ENOMEM, -4 ECORRUPT,
-5 EMISMATCH, -6 EBASE.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ckpt_oracle.c")
# CKPT_ORACLE_LIB names another build of the same source (the tests load an
# AddressSanitizer / UndefinedBehaviorSanitizer build this way)
LIB = os.environ.get("CKPT_ORACLE_LIB") or os.path.join(HERE, "libckpt_oracle.so")
NO_CHUNK = (1 << 64) - 1

_u8p = ctypes.POINTER(ctypes.c_uint8)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_lib = None


def build():
    """Compile the oracle with the host C compiler (no GPU code involved)."""
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-Wall", "-shared", "-fPIC",
                           "-pthread", "-o", LIB, SRC])


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        L.orc_crc32c.restype = ctypes.c_uint32
        L.orc_crc32c.argtypes = [_u8p, ctypes.c_uint64]
        L.orc_image_bound.restype = ctypes.c_uint64
        L.orc_image_bound.argtypes = [ctypes.c_uint32, _u64p, ctypes.c_uint32]
        L.orc_dump.restype = ctypes.c_int
        L.orc_dump.argtypes = [ctypes.c_uint32, _u64p, _u64p, ctypes.POINTER(_u8p), ctypes.c_uint32,
                               ctypes.c_int, _u8p, ctypes.c_uint64, ctypes.c_int, _u8p, ctypes.c_uint64, _u64p]
        L.orc_restore.restype = ctypes.c_int
        L.orc_restore.argtypes = [_u8p, ctypes.c_uint64, ctypes.c_uint32, _u64p, _u64p,
                                  ctypes.POINTER(_u8p), ctypes.c_int, _u64p]
        L.orc_merge.restype = ctypes.c_int
        L.orc_merge.argtypes = [_u8p, ctypes.c_uint64, _u8p, ctypes.c_uint64, _u8p, ctypes.c_uint64, _u64p]
        L.orc_parse.restype = ctypes.c_int
        L.orc_parse.argtypes = [_u8p, ctypes.c_uint64, _u64p]
        _lib = L
    return _lib


def _as_u8(x):
    if isinstance(x, np.ndarray):
        return np.ascontiguousarray(x).view(np.uint8).reshape(-1)
    return np.frombuffer(bytes(x), dtype=np.uint8)


def _ptr(a):
    if a.size == 0:
        a = np.zeros(1, np.uint8)      # keep a valid address for empty buffers
    return a.ctypes.data_as(_u8p), a


def default_threads():
    return max(1, min(16, os.cpu_count() or 1))


def crc32c(data):
    a = _as_u8(data)
    p, keep = _ptr(a)
    return int(lib().orc_crc32c(p, a.size))


def _table(allocs):
    n = len(allocs)
    ids = np.array([int(i) for i, _ in allocs], dtype=np.uint64)
    arrs = [_as_u8(b) for _, b in allocs]
    sizes = np.array([a.size for a in arrs], dtype=np.uint64)
    ptrs = (_u8p * max(n, 1))()
    keep = []
    for k, a in enumerate(arrs):
        p, kk = _ptr(a)
        ptrs[k] = p
        keep.append(kk)
    return n, ids, sizes, ptrs, keep


def dump(allocs, c, prev=None, threads=None, codec=False):
    """allocs: list of (id, array) in table order. Returns (rc, image array or None).
    codec: store full DATA chunks as byte-plane records where shorter."""
    n, ids, sizes, ptrs, keep = _table(allocs)
    cap = 80
    if n:
        cap = max(cap, int(lib().orc_image_bound(n, sizes.ctypes.data_as(_u64p), c)))
    out = np.empty(cap, dtype=np.uint8)
    olen = ctypes.c_uint64(0)
    if prev is not None:
        pv = _as_u8(prev)
        pp, pkeep = _ptr(pv)
        plen = pv.size
    else:
        pp, plen = None, 0
    rc = lib().orc_dump(n, ids.ctypes.data_as(_u64p), sizes.ctypes.data_as(_u64p), ptrs, c, int(bool(codec)),
                        pp, plen, threads or default_threads(),
                        out.ctypes.data_as(_u8p), out.size, ctypes.byref(olen))
    if rc != 0:
        return rc, None
    return 0, out[:olen.value]


def restore(image, allocs, threads=None):
    """allocs: list of (id, writable uint8 array) in table order; written in place.
    Returns (rc, first_bad_chunk)."""
    img = _as_u8(image)
    ip, ikeep = _ptr(img)
    n = len(allocs)
    ids = np.array([int(i) for i, _ in allocs], dtype=np.uint64)
    sizes = np.array([b.size for _, b in allocs], dtype=np.uint64)
    ptrs = (_u8p * max(n, 1))()
    keep = []
    for k, (_, b) in enumerate(allocs):
        assert isinstance(b, np.ndarray) and b.dtype == np.uint8 and b.flags.c_contiguous
        p, kk = _ptr(b)
        ptrs[k] = p
        keep.append(kk)
    bad = ctypes.c_uint64(0)
    rc = lib().orc_restore(ip, img.size, n, ids.ctypes.data_as(_u64p), sizes.ctypes.data_as(_u64p),
                           ptrs, threads or default_threads(), ctypes.byref(bad))
    return rc, bad.value


def merge(base, delta):
    b = _as_u8(base)
    d = _as_u8(delta)
    bp, bk = _ptr(b)
    dp, dk = _ptr(d)
    cap = b.size + d.size + 64
    out = np.empty(cap, dtype=np.uint8)
    olen = ctypes.c_uint64(0)
    rc = lib().orc_merge(bp, b.size, dp, d.size, out.ctypes.data_as(_u8p), cap, ctypes.byref(olen))
    if rc != 0:
        return rc, None
    return 0, out[:olen.value]


def parse(image):
    img = _as_u8(image)
    ip, keep = _ptr(img)
    f = np.zeros(8, dtype=np.uint64)
    rc = lib().orc_parse(ip, img.size, f.ctypes.data_as(_u64p))
    if rc != 0:
        return rc, None
    keys = ["flags", "C", "n_allocs", "n_chunks", "D", "base_state", "N", "state_digest"]
    return 0, {k: int(v) for k, v in zip(keys, f)}
