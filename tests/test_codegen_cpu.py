"""Code-generation checks on the gfx950 device assembly of every kernel
source (CPU only: hipcc cross-compiles).

The library writes device memory only through vector memory instructions:
no scalar-cache stores, scalar atomics or scalar-cache write-back/discard
may appear in the generated code, and no kernel may spill to scratch.
"""
import glob
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1312_2880_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FORBIDDEN = re.compile(r"^\s*(s_store_|s_atomic_|s_buffer_store|s_buffer_atomic|s_scratch_store|"
                       r"s_dcache_wb|s_dcache_discard)", re.M)


def device_asm(src, tmp_path):
    out = tmp_path / (os.path.basename(src) + ".s")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "--offload-device-only", "-S", "-o",
           str(out), src]
    res = subprocess.run(cmd, capture_output=True, text=True, cwd=CSRC)
    assert res.returncode == 0, res.stderr[-2000:]
    return out.read_text()


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="hipcc not available")
@pytest.mark.parametrize("src", sorted(glob.glob(os.path.join(CSRC, "*.hip"))), ids=os.path.basename)
def test_device_code_uses_vector_stores_only(src, tmp_path):
    asm = device_asm(src, tmp_path)
    bad = FORBIDDEN.findall(asm)
    assert not bad, f"scalar-cache writes in {os.path.basename(src)}: {sorted(set(bad))}"
    scratch = [int(x) for x in re.findall(r"\.private_segment_fixed_size:\s+(\d+)", asm)]
    assert all(x == 0 for x in scratch), f"scratch use in {os.path.basename(src)}: {scratch}"
