"""The CPU oracle built under AddressSanitizer and UndefinedBehaviorSanitizer
(gcc) runs every one of its entry points on small grids without a report:
out-of-bounds accesses, use after free, leaks, signed overflow, misaligned
or null accesses abort the driver."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    subprocess.check_call([
        "gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer",
        "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
        "-I", os.path.join(ROOT, "oracle"), "-o", exe,
        os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
        os.path.join(ROOT, "oracle", "hmg_oracle.c"), "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "oracle driver done" in r.stdout
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-4000:]
