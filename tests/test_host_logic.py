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
