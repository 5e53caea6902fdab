"""Run by tests/test_oracle_sanitized.py in a child process whose C oracle is
an AddressSanitizer / UndefinedBehaviorSanitizer build: dumps (plain, codec,
delta), merges, parses and restores over ragged tables, then images with a
byte flipped at many positions and images cut short at many lengths. Any
out-of-bounds access or undefined behaviour aborts the process."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from oracle import oracle as o  # noqa: E402

with open("/proc/self/maps") as fh:
    assert "libasan" in fh.read(), "the sanitizer runtime is not loaded"


def table(seed):
    r = np.random.default_rng(seed)
    out = []
    for k, n in enumerate([0, 1, 15, 17, 1000, 4096, 5000, 9000]):
        a = r.integers(0, 256, n, dtype=np.uint8)
        if n > 100:
            a[10:60] = 0
        if k == 5:
            a[:] = 0
        out.append((k + 1, a))
    w = (r.standard_normal(2048) * 0.02).astype(np.float32).view(np.uint8)   # PACKED under the codec
    out.append((99, w.copy()))
    return out


def zeros(t):
    return [(i, np.zeros(a.size, np.uint8)) for i, a in t]


for C in (256, 512, 4096):
    t = table(C)
    for codec in (False, True):
        rc, img = o.dump(t, C, codec=codec, threads=1)
        assert rc == 0
        t2 = [(i, a.copy()) for i, a in t]
        t2[4][1][3] ^= 1
        t2[8][1][100] ^= 7
        rc, d = o.dump(t2, C, prev=img, codec=codec, threads=1)
        assert rc == 0
        rc, m = o.merge(img, d)
        assert rc == 0
        for im in (img, d, m):
            o.parse(im)
            for pos in range(0, im.size, 11):
                b = im.copy()
                b[pos] ^= 0x41
                o.restore(b, zeros(t), threads=1)
            for cut in range(0, im.size, 131):
                o.restore(im[:cut].copy(), zeros(t), threads=1)
                o.parse(im[:cut].copy())
        for th in (1, 4):
            tgt = zeros(t)
            assert o.restore(img, tgt, threads=th)[0] == 0
            assert all(np.array_equal(a, b) for (_, a), (_, b) in zip(t, tgt))
print("sanitized oracle ok")
