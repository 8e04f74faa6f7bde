"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a
standalone driver (oracle/sanitize_driver.cpp) built with both sanitizers
sets up every preconditioner form on a small coupled system, solves,
applies, inspects the hierarchies and calls the building blocks; any
out-of-bounds access, use after free, leak or undefined operation aborts
it with a report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    cmd = ["g++", "-std=c++17", "-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-static-libasan", os.path.join(ROOT, "oracle", "oracle.cpp"),
           os.path.join(ROOT, "oracle", "sanitize_driver.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=600)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout
