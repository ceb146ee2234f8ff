"""The CPU oracle under the address and undefined-behaviour sanitizers.

A small C driver (tests/oracle_sanitize_driver.c) calls every oracle entry
point on small grids (direct and smoothed coarse solves, graded spacing,
a one-level and a one-cell-column case); it is compiled with gcc
-fsanitize=address,undefined and run on the CPU.  Any out-of-bounds access,
use after free, leak or undefined operation ends it with a report."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_sanitize"
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(HERE, "oracle_sanitize_driver.c"), "-o", str(exe), "-lm"]
    subprocess.check_call(cmd)
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([str(exe)], env=env, capture_output=True, text=True, timeout=600)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert "oracle sanitize driver: ok" in out
