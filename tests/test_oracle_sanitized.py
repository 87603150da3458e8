"""The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle's C source and a driver that calls every entry point (seeded
populations, coincident and collinear agents, n = 0, 1, 2, error paths, one
and four threads) are built with gcc -fsanitize=address,undefined as one host
program and run; any invalid access, leak or undefined operation aborts it.
Host code only: nothing here is built for or run on the GPU.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "orc_sanitized"
    src = [os.path.join(ROOT, "tests", "oracle_sanitize_driver.c"), os.path.join(ROOT, "oracle", "mech_oracle.c")]
    subprocess.run(["gcc", "-O1", "-g", "-std=c99", "-fopenmp", "-ffp-contract=off",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", *src, "-o", str(exe), "-lm"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "all ok" in r.stdout
