"""Build libhmg.so for gfx950 with hipcc (in-tree, next to this file).

    python -m paper_1312_2880_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["hmg_kernels.hip", "hmg_fused.hip", "hmg_lex.hip", "hmg_ray.hip", "hmg_api.hip", "hmg_solve.hip"]
OUT = os.path.join(HERE, "libhmg.so")
# a copy of the library whose host code carries AddressSanitizer and
# UndefinedBehaviorSanitizer (device code as usual), and the driver that
# exercises it through the C-ABI
SAN_DIR = os.path.join(HERE, "hostsan")
SAN_LIB = os.path.join(SAN_DIR, "libhmg_hostsan.so")
SAN_EXE = os.path.join(SAN_DIR, "hmg_host_driver")
ARCH = os.environ.get("HMG_OFFLOAD_ARCH", "gfx950")


def _run(cmd, verbose):
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    msgs = "\n".join(l for l in (res.stdout + res.stderr).splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError(f"{cmd[0]} failed:\n" + msgs)
    if verbose and msgs.strip():
        print(msgs, file=sys.stderr)


def _hipcc_cmd(opt, extra):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    return [hipcc, f"--offload-arch={ARCH}", opt, "-std=c++17", "-fPIC", "-shared",
            "-Wall", "-Wno-unused-function",
            # keep the compiler from forming packed FP32 instructions
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC] + extra + \
        [os.path.join(CSRC, s) for s in SOURCES] + \
        ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]


def build(verbose: bool = False) -> str:
    tmp = OUT + ".tmp%d" % os.getpid()
    _run(_hipcc_cmd("-O3", []) + ["-o", tmp], verbose)
    os.replace(tmp, OUT)
    return OUT


def build_hostsan(verbose: bool = False) -> str:
    """The host-sanitized library and its driver (tests/sanitize/host_driver.c).
    Only host code is instrumented: each -fsanitize= applies to the host pass."""
    os.makedirs(SAN_DIR, exist_ok=True)
    san = []
    for flag in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all",
                 "-fno-omit-frame-pointer", "-g"):
        san += ["-Xarch_host", flag]
    tmp = SAN_LIB + ".tmp%d" % os.getpid()
    _run(_hipcc_cmd("-O1", san) + ["-o", tmp], verbose)
    os.replace(tmp, SAN_LIB)
    clang = os.environ.get("HMG_CLANG", "/opt/rocm/llvm/bin/clang")
    tmp = SAN_EXE + ".tmp%d" % os.getpid()
    _run([clang, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"),
          os.path.join(ROOT, "tests", "sanitize", "host_driver.c"), "-o", tmp,
          "-L", SAN_DIR, "-lhmg_hostsan", "-Wl,-rpath,$ORIGIN"], verbose)
    os.replace(tmp, SAN_EXE)
    return SAN_EXE


if __name__ == "__main__":
    print(build(verbose=True))
    if "--hostsan" in sys.argv:
        print(build_hostsan(verbose=True))
