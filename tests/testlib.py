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
