"""The CPU oracle and the all-cores baseline built with AddressSanitizer and
UndefinedBehaviorSanitizer (gcc, host code only) and driven over edge cases
by tests/native/oracle_sanitize.c: no out-of-bounds access, leak or
undefined behaviour, and the expected results on the tiny cases."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = os.path.join(tmp_path, "oracle_sanitize")
    cmd = ["gcc", "-std=c11", "-g", "-O1", "-fsanitize=address,undefined",
           "-fno-omit-frame-pointer", "-fno-sanitize-recover=all", "-fopenmp", "-o", exe,
           os.path.join(HERE, "native", "oracle_sanitize.c"), os.path.join(ROOT, "oracle", "oracle.c"),
           os.path.join(ROOT, "oracle", "oracle_omp.c"), "-lm"]
    b = subprocess.run(cmd, capture_output=True, text=True)
    if b.returncode != 0 and "asan" in (b.stderr + b.stdout).lower():
        pytest.skip("this gcc has no sanitizer runtime")
    assert b.returncode == 0, b.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="4")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout + r.stderr[-4000:]
