"""The library's host-only paths built with AddressSanitizer and
UndefinedBehaviorSanitizer (host code only; the kernels are the ordinary
build) run without a finding in a child process on the CPU: image import
(valid, every byte flipped at a stride, cut short at many lengths), bytes,
merge (valid and mismatched pairs), save / load (round trip, truncated and
missing files), strerror and the host CRC-32C. Images come from the plain-C
oracle; no GPU is involved."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2502_16631_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_2502_16631_amd", "_build")


def _clang_asan():
    base = "/opt/rocm/llvm/lib/clang"
    if not os.path.isdir(base):
        return None
    for v in sorted(os.listdir(base), reverse=True):
        p = os.path.join(base, v, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(p):
            return p
    return None


def test_sanitized_library_host_paths(tmp_path):
    asan = _clang_asan()
    if asan is None:
        pytest.skip("no clang AddressSanitizer runtime")
    for o in ("kernels.o", "codec.o", "gather.o"):
        if not os.path.exists(os.path.join(BUILD, o)):
            subprocess.check_call(["bash", os.path.join(ROOT, "paper_2502_16631_amd", "build.sh")])
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    objs = []
    for src in ("runtime.hip", "serve.hip"):
        obj = str(tmp_path / (src + ".o"))
        subprocess.check_call(["hipcc"] + flags + san + ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in ("hostmath.cpp", "storage.cpp"):
        obj = str(tmp_path / (src + ".o"))
        subprocess.check_call(["/opt/rocm/llvm/bin/clang++", "-O1", "-g", "-std=c++17", "-fPIC", "-msse4.2",
                               "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-fsanitize=address,undefined",
                               "-fno-omit-frame-pointer", "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    lib = str(tmp_path / "libmickpt_san.so")
    subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC"] + san + ["-o", lib] + objs +
                          [os.path.join(BUILD, o) for o in ("kernels.o", "codec.o", "gather.o")] + ["-lpthread"])
    env = dict(os.environ, LD_PRELOAD=asan, MICKPT_SAN_LIB=lib, MICKPT_SAN_DIR=str(tmp_path),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:protect_shadow_gap=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    p = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "lib_sanitized_case.py")],
                       env=env, capture_output=True, text=True, timeout=600)
    assert p.returncode == 0 and "sanitized library ok" in p.stdout, (p.stdout[-2000:], p.stderr[-4000:])
