"""CPU-side checks of the C-ABI library: it loads, exports every function
that include/hmg.h declares, and rejects bad arguments before touching a
device.  No kernel runs here."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hmg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(hmg_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for required in ("hmg_grid_create", "hmg_vcycle", "hmg_solve", "hmg_solve_batch",
                     "hmg_submit", "hmg_poll", "hmg_cancel"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1312_2880_amd import hmg
    lib = ctypes.CDLL(hmg.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared_functions()) == set(hmg.EXPORTED)


def test_oracle_is_not_linked_into_the_library():
    from paper_1312_2880_amd import hmg
    lib = ctypes.CDLL(hmg.LIB_PATH)
    assert not hasattr(lib, "orc_vcycle")
    src = os.path.join(ROOT, "paper_1312_2880_amd")
    for dirpath, _, files in os.walk(src):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in text and "hmg_oracle" not in text, fn


def test_defaults_are_the_papers_constants():
    from paper_1312_2880_amd import hmg
    o = hmg.opts()
    assert o.beta == 0.5                      # eq:mh, beta = 0.5
    assert (o.nu_pre, o.nu_post) == (1, 1)    # V(1,1) smoothing
    assert (o.kacz_pre, o.kacz_post) == (4, 4)
    assert o.variant == hmg.HYB and o.coarsest_n == 7
    # schedule defaults: fused kernels, tuned Kaczmarz tiles, dense bottom cycle
    assert (o.one_pass_kernels, o.autotune, o.bottom_dense, o.use_graph) == (0, 1, 1, 1)


def _header_fields(typedef_name):
    """Field names of a `typedef struct { ... } name;` of the public header."""
    import re
    hdr = open(os.path.join(ROOT, "include", "hmg.h")).read()
    end = hdr.index("} %s;" % typedef_name)
    body = hdr[hdr.rindex("typedef struct {", 0, end) + len("typedef struct {"):end]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        for part in decl.split(None, 1)[1].split(","):
            names.append(part.strip().split("[")[0])
    return names


def test_opts_struct_matches_the_header():
    """The ctypes mirror of hmg_opts has the header's field order."""
    from paper_1312_2880_amd import hmg
    assert [f for f, _ in hmg.Opts._fields_] == _header_fields("hmg_opts")


def test_info_and_result_structs_match_the_header():
    from paper_1312_2880_amd import hmg
    assert [f for f, _ in hmg.SolveInfo._fields_] == _header_fields("hmg_solve_info")
    assert [f for f, _ in hmg.Result._fields_] == _header_fields("hmg_result")
    assert [f for f, _ in hmg.Plan._fields_] == _header_fields("hmg_plan")


def test_null_arguments_are_rejected():
    from paper_1312_2880_amd import hmg
    lib = hmg._lib
    out = ctypes.c_void_p()
    k = np.ones((9, 9))
    assert lib.hmg_grid_create(None, 7, 0.125, hmg._ptr(k), None, 1, None,
                               ctypes.byref(out)) == hmg.ERR_INVALID
    assert lib.hmg_vcycle(None, None, None) == hmg.ERR_INVALID
    assert lib.hmg_solve(None, None, None, 1e-6, 10, None) == hmg.ERR_INVALID
    assert lib.hmg_poll(None, 1, None, None) == hmg.ERR_INVALID
    assert b"null" in lib.hmg_last_error()


def test_input_generators_do_not_depend_on_thread_count():
    """The seeded media are the same bits whatever the number of BLAS/OpenMP
    threads (the oracle's stored counts and the GPU runs on another host use
    the same problem)."""
    import hashlib
    import subprocess
    import sys
    code = ("import hashlib, sys; sys.path.insert(0, %r); "
            "from paper_1312_2880_amd import inputs; "
            "h, k, f = inputs.layered_problem(255, 2, 50.0); "
            "w = inputs.wedge_problem(127); "
            "print(hashlib.sha256(k.tobytes() + f.tobytes() + w[1].tobytes()).hexdigest())" % ROOT)
    out = set()
    for threads in ("1", "3", "8"):
        env = dict(os.environ, OMP_NUM_THREADS=threads, OPENBLAS_NUM_THREADS=threads)
        out.add(subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                               check=True).stdout.strip())
    assert len(out) == 1, out
