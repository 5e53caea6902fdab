"""Shared helpers for the tests: golden-fixture parsing and the hardware
CRC-32C cross-check (x86 SSE4.2), which shares nothing with the oracle."""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")
_hw = None


def hw_crc32c(data):
    """CRC-32C computed by the SSE4.2 crc32 instruction."""
    global _hw
    if _hw is None:
        so = os.path.join(HERE, "hwcrc", "libhwcrc.so")
        if not os.path.exists(so):
            subprocess.check_call(["gcc", "-O2", "-msse4.2", "-shared", "-fPIC", "-o", so,
                                   os.path.join(HERE, "hwcrc", "hw_crc32c.c")])
        _hw = ctypes.CDLL(so)
        _hw.hw_crc32c.restype = ctypes.c_uint32
        _hw.hw_crc32c.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
    if isinstance(data, np.ndarray):
        a = np.ascontiguousarray(data).view(np.uint8).reshape(-1)
    else:
        a = np.frombuffer(bytes(data), dtype=np.uint8)
    if a.size == 0:
        return 0
    return int(_hw.hw_crc32c(a.ctypes.data, a.size))


def decode_input(spec):
    """Inputs of the golden files: ascii:<text>, fill:<hex>x<n>, inc:<hex>x<n>,
    dec:<hex>x<n>, empty."""
    if spec == "empty":
        return b""
    kind, _, arg = spec.partition(":")
    if kind == "ascii":
        return arg.encode()
    start, _, count = arg.partition("x")
    start, count = int(start, 16), int(count)
    if kind == "fill":
        return bytes([start]) * count
    if kind == "inc":
        return bytes((start + i) & 0xFF for i in range(count))
    if kind == "dec":
        return bytes((start - i) & 0xFF for i in range(count))
    raise ValueError(spec)


def golden_lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line.split()


def _raw_crc(data):
    """Raw CRC-32C (no preset, no complement) from the hardware CRC: CRC is affine,
    so raw(M) = CRC(M) xor CRC(0^|M|)."""
    return hw_crc32c(data) ^ hw_crc32c(bytes(len(data)))


def crc_collide(orig, modified, pos):
    """Patch 4 bytes of `modified` at `pos` so that its CRC-32C equals orig's
    (CRC is affine in the message: the 32 single-bit flips of those bytes span
    the raw CRC's 32-bit space, so the system over GF(2) has a solution).
    Built on the hardware CRC only, so it shares nothing with the oracle or
    the GPU library."""
    n = len(orig)
    target = _raw_crc(bytes(a ^ b for a, b in zip(orig, modified)))
    cols = []
    for bit in range(32):
        e = bytearray(n)
        e[pos + bit // 8] = 1 << (bit % 8)
        cols.append(_raw_crc(bytes(e)))
    # solve sum(w_i * cols_i) = target over GF(2)
    basis = {}
    for v, m in ((cols[i], 1 << i) for i in range(32)):
        for b in range(31, -1, -1):
            if not (v >> b) & 1:
                continue
            if b in basis:
                v ^= basis[b][0]
                m ^= basis[b][1]
            else:
                basis[b] = (v, m)
                break
    v, m = target, 0
    for b in range(31, -1, -1):
        if (v >> b) & 1:
            v ^= basis[b][0]
            m ^= basis[b][1]
    assert v == 0
    out = bytearray(modified)
    for i in range(4):
        out[pos + i] ^= (m >> (8 * i)) & 0xFF
    return bytes(out)
