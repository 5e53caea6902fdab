"""Run by tests/test_lib_sanitized.py in a child process that loads an
AddressSanitizer / UndefinedBehaviorSanitizer build of the library (host
code) and calls its host-only entry points through the C ABI on images the
oracle wrote: valid, with a byte flipped at a stride of positions, cut short
at many lengths; merges of matching and mismatched pairs; image files saved,
loaded, truncated and missing. Any out-of-bounds access or undefined
behaviour aborts the process. Return codes are also checked against the
oracle's parse of the same bytes."""
import ctypes
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from oracle import oracle as o  # noqa: E402

with open("/proc/self/maps") as fh:
    assert "libclang_rt.asan" in fh.read(), "the sanitizer runtime is not loaded"

L = ctypes.CDLL(os.environ["MICKPT_SAN_LIB"])
vp = ctypes.c_void_p
L.ckpt_image_import.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(vp)]
L.ckpt_image_bytes.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_uint64)]
L.ckpt_image_free.argtypes = [vp]
L.ckpt_image_free.restype = None
L.ckpt_merge.argtypes = [vp, vp, ctypes.POINTER(vp)]
L.ckpt_image_save.argtypes = [vp, ctypes.c_char_p, ctypes.c_uint32]
L.ckpt_image_load.argtypes = [ctypes.c_char_p, ctypes.c_uint32, ctypes.POINTER(vp)]
L.ckpt_strerror.restype = ctypes.c_char_p
L.ckpt_crc32c.argtypes = [vp, ctypes.c_uint64]
L.ckpt_crc32c.restype = ctypes.c_uint32
tmp = os.environ["MICKPT_SAN_DIR"]


def imp(a):
    a = np.ascontiguousarray(a)
    h = vp()
    rc = L.ckpt_image_import(a.ctypes.data if a.size else None, a.size, ctypes.byref(h))
    return rc, h


def content(h):
    p, n = vp(), ctypes.c_uint64()
    assert L.ckpt_image_bytes(h, ctypes.byref(p), ctypes.byref(n)) == 0
    return np.ctypeslib.as_array((ctypes.c_uint8 * n.value).from_address(p.value)).copy() if n.value else \
        np.zeros(0, np.uint8)


def table(seed):
    r = np.random.default_rng(seed)
    out = []
    for k, n in enumerate([0, 1, 15, 17, 1000, 4096, 5000, 9000]):
        a = r.integers(0, 256, n, dtype=np.uint8)
        if n > 100:
            a[10:60] = 0
        out.append((k + 1, a))
    out.append((99, (r.standard_normal(2048) * 0.02).astype(np.float32).view(np.uint8).copy()))
    return out


for code in range(-10, 2):
    assert L.ckpt_strerror(code)
r = np.random.default_rng(5)
for n in (0, 1, 7, 16, 1000, 65537):
    b = r.integers(0, 256, n, dtype=np.uint8)
    assert L.ckpt_crc32c(b.ctypes.data if n else None, n) == o.crc32c(b)

for C in (256, 4096):
    t = table(C)
    for codec in (False, True):
        rc, base = o.dump(t, C, codec=codec, threads=1)
        assert rc == 0
        t2 = [(i, a.copy()) for i, a in t]
        t2[4][1][3] ^= 1
        t2[8][1][100] ^= 7
        rc, delta = o.dump(t2, C, prev=base, codec=codec, threads=1)
        assert rc == 0
        rc, merged = o.merge(base, delta)
        assert rc == 0
        hb = imp(base)
        hd = imp(delta)
        assert hb[0] == 0 and hd[0] == 0
        assert np.array_equal(content(hb[1]), base)
        hm = vp()
        assert L.ckpt_merge(hb[1], hd[1], ctypes.byref(hm)) == 0
        assert np.array_equal(content(hm), merged)
        L.ckpt_image_free(hm)
        bad = vp()
        assert L.ckpt_merge(hd[1], hb[1], ctypes.byref(bad)) != 0      # roles swapped
        assert L.ckpt_merge(hb[1], hb[1], ctypes.byref(bad)) != 0      # a full image is no delta
        for im in (base, delta, merged):
            for pos in range(0, im.size, 7):
                b = im.copy()
                b[pos] ^= 0x41
                rc, h = imp(b)
                want = o.parse(b)[0]
                assert (rc == 0) == (want == 0), (pos, rc, want)
                if rc == 0:
                    L.ckpt_image_free(h)
            for cut in range(0, im.size, 53):
                rc, h = imp(im[:cut].copy())
                assert rc != 0
        path = os.path.join(tmp, "img_%d_%d.bin" % (C, codec)).encode()
        assert L.ckpt_image_save(hd[1], path, 3) == 0
        h2 = vp()
        assert L.ckpt_image_load(path, 2, ctypes.byref(h2)) == 0
        assert np.array_equal(content(h2), delta)
        L.ckpt_image_free(h2)
        with open(path, "r+b") as fh:
            fh.truncate(delta.size - 9)
        assert L.ckpt_image_load(path, 2, ctypes.byref(h2)) != 0
        assert L.ckpt_image_load(path + b".missing", 2, ctypes.byref(h2)) != 0
        os.remove(path)
        L.ckpt_image_free(hb[1])
        L.ckpt_image_free(hd[1])
print("sanitized library ok")
