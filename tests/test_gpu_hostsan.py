"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
on the GPU: a copy of the library whose host pass carries both sanitizers
(device code unchanged) runs a C driver through the C-ABI -- grids of both
precisions and all variants, solves with and without an initial guess, a
batch, the ray-corrected cycle solver, the request server with admission,
grid reuse and cancellation, and argument checks.  Any invalid host access
or undefined behaviour aborts the driver with a report.  Leak checking is
off: the ROCm runtime keeps allocations until the process ends."""
import os
import subprocess

import pytest

from paper_1312_2880_amd import build as hb

pytestmark = pytest.mark.gpu


def test_host_code_clean_under_asan_and_ubsan():
    if not os.path.exists(hb.SAN_EXE):
        pytest.fail("host-sanitized driver not built (paper_1312_2880_amd.build --hostsan)")
    print("case host sanitizer driver", flush=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([hb.SAN_EXE], env=env, capture_output=True, text=True, timeout=200)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    assert "host driver done" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-6000:]
