"""The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code only; gcc), driven through every entry point by
tests/oracle_sanitize_driver.c: a heap overflow, use after free, leak,
signed overflow, misaligned or out-of-bounds access in the oracle aborts the
run and fails the test."""
from __future__ import annotations

import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_behaviour_sanitizers():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "oracle_sanitize")
        subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp",
                               "-ffp-contract=off", "-fsanitize=address,undefined",
                               "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                               "-o", exe, os.path.join(HERE, "oracle_sanitize_driver.c"), "-lm"])
        env = dict(os.environ, OMP_NUM_THREADS="4",
                   ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "all checks passed" in r.stdout
        assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
