"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only) runs its dump, merge, parse and restore paths --
including corrupt and truncated images -- without a finding. The oracle is
the reference every GPU result is compared with, so its own memory safety
is checked here."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    p = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_sanitized_oracle(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("no AddressSanitizer runtime for gcc")
    lib = str(tmp_path / "libckpt_oracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=gnu11", "-Wall", "-fsanitize=address,undefined",
                           "-fno-omit-frame-pointer", "-shared", "-fPIC", "-pthread", "-o", lib,
                           os.path.join(ROOT, "oracle", "ckpt_oracle.c")])
    env = dict(os.environ, LD_PRELOAD=asan, CKPT_ORACLE_LIB=lib,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    p = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "oracle_sanitized_case.py")],
                       env=env, capture_output=True, text=True, timeout=300)
    assert p.returncode == 0 and "sanitized oracle ok" in p.stdout, (p.stdout[-2000:], p.stderr[-4000:])
