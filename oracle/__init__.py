"""FP64 CPU oracle for the multigrid-preconditioned Helmholtz solver of
Livshits, arXiv:1312.2880 (Sections 1, 4, 5 and 6).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and
by the CPU-baseline leg of the benchmark, never by the GPU library.  It shares
no code with the HIP path.  The arithmetic lives in ``hmg_oracle.c`` (plain
C99, FP64, no contraction); this module only marshals numpy arrays.

Array conventions: a grid with ``n`` interior nodes per side has
``(n+2) x (n+2)`` nodes, stored as numpy arrays of shape ``(n+2, n+2)``
indexed ``[j, i]`` (x fastest); complex arrays are ``complex128``; ``k`` is
the real wavenumber per node.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hmg_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libhmg_oracle.so")

SL, HLM, HYB = 0, 1, 2
SM_GS, SM_KACZ, SM_LU = 0, 1, 2
ORDER_COLOUR, ORDER_LEX = 0, 1
PREC_NONE, PREC_VCYCLE, PREC_EXACT = 0, 1, 2
MIX_OFF, MIX_FUSED, MIX_ONEPASS = 0, 1, 2
OK, NOT_CONVERGED, BREAKDOWN = 0, 4, 5
MAX_LEVELS = 24


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, -ffp-contract=off)."""
    if force or not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-std=c99", "-O2", "-fno-fast-math", "-ffp-contract=off",
            "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Opts(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int), ("beta", ctypes.c_double),
                ("nu_pre", ctypes.c_int), ("nu_post", ctypes.c_int),
                ("kacz_pre", ctypes.c_int), ("kacz_post", ctypes.c_int),
                ("kacz_band", ctypes.c_int), ("coarsest_n", ctypes.c_int),
                ("gs_order", ctypes.c_int), ("kacz_order", ctypes.c_int),
                ("hyb_mid", ctypes.c_int)]


class _Plan(ctypes.Structure):
    L = MAX_LEVELS
    _fields_ = [("nlev", ctypes.c_int), ("n", ctypes.c_int * L),
                ("H", ctypes.c_double * L), ("kHmin", ctypes.c_double * L),
                ("kHmax", ctypes.c_double * L), ("smoother", ctypes.c_int * L),
                ("sigma_relax", ctypes.c_double * L),
                ("sigma_resid", ctypes.c_double * L),
                ("pre", ctypes.c_int * L), ("post", ctypes.c_int * L)]


class _Info(ctypes.Structure):
    _fields_ = [("halfsteps", ctypes.c_int), ("rel_res", ctypes.c_double),
                ("restarts", ctypes.c_int), ("status", ctypes.c_int),
                ("vcycles", ctypes.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        i, d = ctypes.c_int, ctypes.c_double
        sig = {
            "orc_apply": [i, d, P, d, P, P],
            "orc_residual": [i, d, P, d, P, P, P],
            "orc_dense": [i, d, P, d, P],
            "orc_gs_lex": [i, d, P, d, P, P],
            "orc_gs_rb": [i, d, P, d, P, P],
            "orc_kacz_lex": [i, d, P, d, P, P],
            "orc_kacz_5c": [i, d, P, d, P, P],
            "orc_restrict_fw": [i, P, P],
            "orc_prolong_add": [i, P, P],
            "orc_inject_k": [i, P, P],
            "orc_lu_factor": [i, P, P],
            "orc_lu_solve": [i, P, P, P],
            "orc_opts_default": [P],
            "orc_grid_create": [i, d, P, P],
            "orc_grid_destroy": [P],
            "orc_grid_plan": [P, P],
            "orc_vcycle": [P, P, P],
            "orc_bicgstab": [P, P, P, d, i, i, P, P, i],
            "orc_bicgstab_ex": [P, P, P, d, i, i, P, P, i, i],
            "orc_bicgstab_ex2": [P, P, P, d, i, i, P, P, i, i, i, i],
            "orc_grid_override_level": [P, i, i, d, d, i, i],
            "orc_grid_set_mixed": [P, i, i, i, i],
            "orc_grid_set_mixed_ex": [P, i, i, i, i, i],
            "orc_grid_set_ray": [P, i],
            "orc_ray_correct": [P, P, P],
            "orc_cycles": [P, P, P, d, i, P],
            "orc_grid_set_study": [P, i, i],
            "orc_set_boundary_row_scale": [i],
        }
        for name, args in sig.items():
            fn = getattr(_lib, name)
            fn.argtypes = args
            fn.restype = None
        _lib.orc_grid_create.restype = P
        _lib.orc_lu_factor.restype = i
        _lib.orc_bicgstab.restype = i
        _lib.orc_bicgstab_ex.restype = i
        _lib.orc_bicgstab_ex2.restype = i
        _lib.orc_grid_set_ray.restype = i
        _lib.orc_cycles.restype = i
        _lib.orc_grid_override_level.restype = i
    return _lib


def set_boundary_row_scale(on: bool) -> None:
    """Study reading (process-wide): rows with b boundary faces multiplied by
    2^-b in every operator of the oracle; the caller scales right-hand sides
    the same way.  Leave it off outside a study."""
    lib().orc_set_boundary_row_scale(int(bool(on)))


def set_threads(n: int) -> None:
    """Number of OpenMP threads the oracle's parallel loops use (results do
    not depend on it: every reduction is sequential)."""
    fn = lib().omp_set_num_threads
    fn.argtypes = [ctypes.c_int]
    fn.restype = None
    fn(int(n))


def _c(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def _n_of(a) -> int:
    a = np.asarray(a)
    assert a.ndim == 2 and a.shape[0] == a.shape[1], a.shape
    return a.shape[0] - 2


# ---- single-level operations ----------------------------------------------

def apply(h, k, sigma, u):
    """A_sigma u (L for sigma = 0, M = L + i sigma k^2 otherwise)."""
    n = _n_of(k)
    k, kp = _c(k, np.float64)
    u, up = _c(u, np.complex128)
    out = np.empty_like(u)
    lib().orc_apply(n, h, kp, sigma, up, out.ctypes.data_as(ctypes.c_void_p))
    return out


def residual(h, k, sigma, f, u):
    n = _n_of(k)
    k, kp = _c(k, np.float64)
    f, fp = _c(f, np.complex128)
    u, up = _c(u, np.complex128)
    out = np.empty_like(u)
    lib().orc_residual(n, h, kp, sigma, fp, up, out.ctypes.data_as(ctypes.c_void_p))
    return out


def dense(h, k, sigma):
    n = _n_of(k)
    m = (n + 2) ** 2
    k, kp = _c(k, np.float64)
    A = np.empty((m, m), np.complex128)
    lib().orc_dense(n, h, kp, sigma, A.ctypes.data_as(ctypes.c_void_p))
    return A


def _sweep(name, h, k, sigma, f, u):
    n = _n_of(k)
    k, kp = _c(k, np.float64)
    f, fp = _c(f, np.complex128)
    u = np.array(u, dtype=np.complex128, order="C", copy=True)
    getattr(lib(), name)(n, h, kp, sigma, fp, u.ctypes.data_as(ctypes.c_void_p))
    return u


def gs_lex(h, k, sigma, f, u):
    """One lexicographic Gauss-Seidel sweep; returns the new iterate."""
    return _sweep("orc_gs_lex", h, k, sigma, f, u)


def gs_rb(h, k, sigma, f, u):
    """One red-black Gauss-Seidel sweep (red = (i+j) even first)."""
    return _sweep("orc_gs_rb", h, k, sigma, f, u)


def kacz_lex(h, k, sigma, f, u):
    """One lexicographic Kaczmarz (row-action) sweep."""
    return _sweep("orc_kacz_lex", h, k, sigma, f, u)


def kacz_5c(h, k, sigma, f, u):
    """One 5-colour Kaczmarz sweep, colours (i+2j) mod 5 = 0..4."""
    return _sweep("orc_kacz_5c", h, k, sigma, f, u)


def restrict_fw(r):
    n = _n_of(r)
    nc = (n - 1) // 2
    r, rp = _c(r, np.complex128)
    fc = np.empty((nc + 2, nc + 2), np.complex128)
    lib().orc_restrict_fw(n, rp, fc.ctypes.data_as(ctypes.c_void_p))
    return fc


def prolong_add(ec, u):
    nc = _n_of(ec)
    ec, ep = _c(ec, np.complex128)
    u = np.array(u, dtype=np.complex128, order="C", copy=True)
    assert u.shape == (2 * nc + 3, 2 * nc + 3)
    lib().orc_prolong_add(nc, ep, u.ctypes.data_as(ctypes.c_void_p))
    return u


def inject_k(k):
    n = _n_of(k)
    nc = (n - 1) // 2
    k, kp = _c(k, np.float64)
    kc = np.empty((nc + 2, nc + 2), np.float64)
    lib().orc_inject_k(n, kp, kc.ctypes.data_as(ctypes.c_void_p))
    return kc


def lu_solve_dense(A, b):
    """Oracle's own LU with partial pivoting applied to a dense matrix."""
    m = A.shape[0]
    LU = np.array(A, dtype=np.complex128, order="C", copy=True)
    piv = np.zeros(m, np.int32)
    rc = lib().orc_lu_factor(m, LU.ctypes.data_as(ctypes.c_void_p),
                             piv.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise ZeroDivisionError("singular matrix")
    x = np.array(b, dtype=np.complex128, order="C", copy=True)
    lib().orc_lu_solve(m, LU.ctypes.data_as(ctypes.c_void_p),
                       piv.ctypes.data_as(ctypes.c_void_p),
                       x.ctypes.data_as(ctypes.c_void_p))
    return x


# ---- hierarchy, plan, V-cycle, Bi-CGSTAB ----------------------------------

def opts(**kw) -> dict:
    o = _Opts()
    lib().orc_opts_default(ctypes.byref(o))
    d = {name: getattr(o, name) for name, _ in _Opts._fields_}
    for key, val in kw.items():
        if key not in d:
            raise KeyError(key)
        d[key] = val
    return d


class Grid:
    """Multigrid hierarchy for one problem (finest n, h, k)."""

    def __init__(self, h, k, **kw):
        self.k = np.ascontiguousarray(k, dtype=np.float64)
        self.n = _n_of(self.k)
        self.h = float(h)
        self.opts = opts(**kw)
        o = _Opts(**self.opts)
        self._ptr = lib().orc_grid_create(
            self.n, self.h, self.k.ctypes.data_as(ctypes.c_void_p), ctypes.byref(o))
        if not self._ptr:
            raise RuntimeError("orc_grid_create failed")

    def close(self):
        if getattr(self, "_ptr", None):
            lib().orc_grid_destroy(self._ptr)
            self._ptr = None

    def __del__(self):
        self.close()

    def plan(self) -> list[dict]:
        p = _Plan()
        lib().orc_grid_plan(self._ptr, ctypes.byref(p))
        names = {SM_GS: "GS", SM_KACZ: "KACZ", SM_LU: "LU"}
        return [dict(n=p.n[l], H=p.H[l], kHmin=p.kHmin[l], kHmax=p.kHmax[l],
                     smoother=names[p.smoother[l]], sigma_relax=p.sigma_relax[l],
                     sigma_resid=p.sigma_resid[l], pre=p.pre[l], post=p.post[l])
                for l in range(p.nlev)]

    def override_level(self, l, smoother, sigma_relax, sigma_resid, pre=1, post=1):
        """Replace the plan of level ``l`` (smoother 'GS', 'KACZ' or 'LU')."""
        code = {"GS": SM_GS, "KACZ": SM_KACZ, "LU": SM_LU}[smoother]
        rc = lib().orc_grid_override_level(self._ptr, l, code, sigma_relax,
                                           sigma_resid, pre, post)
        if rc != 0:
            raise ValueError("invalid override")

    def set_mixed(self, mode=MIX_FUSED, kacz_every=2, block_n=31, round_io=False, fp64_levels=0):
        """Precision form (O11): the V-cycle stores its fields in complex
        float and computes in double.  MIX_FUSED rounds where the fused
        kernels store (the Kaczmarz iterate every ``kacz_every`` sweeps;
        levels with n <= ``block_n`` are one double block); MIX_ONEPASS after
        every elementary step; ``round_io`` also rounds the cycle's input and
        output.  MIX_OFF restores the double V-cycle.  The outer Bi-CGSTAB
        stays double either way.  ``fp64_levels`` (fused mode) keeps the
        finest levels in double; the first float level then takes and
        returns double fields."""
        lib().orc_grid_set_mixed_ex(self._ptr, int(mode), int(kacz_every), int(block_n),
                                    int(bool(round_io)), int(fp64_levels))
        return self

    def set_study(self, fw_transpose=False, coarse_sweeps=0):
        """Readings of Section 5 other than the default, for iteration-count
        studies: ``fw_transpose`` restricts with P^T / 4 (no mirror folding at
        the boundary); ``coarse_sweeps`` > 0 replaces the coarsest dense solve
        by that many Gauss-Seidel sweeps from zero."""
        lib().orc_grid_set_study(self._ptr, int(bool(fw_transpose)), int(coarse_sweeps))
        return self

    def set_ray(self, ray_n):
        """Ray correction (Section 6.1) on a ray grid of ray_n interior nodes
        per side (0: off); the grid's preconditioner then is the V-cycle
        followed by the Galerkin correction over the 8 plane waves times
        bilinear ray functions."""
        if lib().orc_grid_set_ray(self._ptr, int(ray_n)) != 0:
            raise ValueError("singular ray Galerkin matrix")
        return self

    def ray_correct(self, f, u):
        """u + P (P^H L P)^{-1} P^H (f - L u)."""
        f, fp = _c(f, np.complex128)
        u = np.array(u, dtype=np.complex128, order="C", copy=True)
        lib().orc_ray_correct(self._ptr, fp, u.ctypes.data_as(ctypes.c_void_p))
        return u

    def precondition(self, r):
        """The grid's preconditioner: the V-cycle, then the ray correction of
        its residual when one is set."""
        r, rp = _c(r, np.complex128)
        z = self.vcycle(r)
        return self.ray_correct(r, z)

    def cycles(self, f, rtol=1e-7, maxit=200, x0=None):
        """Stationary iteration x <- x + B (f - L x) with the preconditioner as
        the solver; returns (x, cycles, history of relative residuals)."""
        f, fp = _c(f, np.complex128)
        x = np.zeros_like(f) if x0 is None else np.array(x0, np.complex128, order="C")
        hist = np.zeros(maxit + 1, np.float64)
        it = lib().orc_cycles(self._ptr, fp, x.ctypes.data_as(ctypes.c_void_p), rtol, maxit,
                              hist.ctypes.data_as(ctypes.c_void_p))
        return x, it, hist[: it + 1].copy()

    def vcycle(self, f):
        """One V-cycle from zero initial guess: returns B_V f."""
        f, fp = _c(f, np.complex128)
        assert f.shape == self.k.shape
        u = np.empty_like(f)
        lib().orc_vcycle(self._ptr, fp, u.ctypes.data_as(ctypes.c_void_p))
        return u

    def bicgstab(self, b, rtol=1e-6, maxit=500, precond=PREC_VCYCLE, x0=None,
                 history=False, force_breakdown_at=0, true_res_every=0, nan_at=0):
        # force_breakdown_at = K > 0: the breakdown restart (rhat = r) is taken
        # at the start of iteration K + 1 whatever rho is (restart-path tests);
        # true_res_every = K > 0: the residual is recomputed (and the
        # iteration restarted from it) after every K-th full iteration;
        # nan_at = K > 0: the residual norm after iteration K counts as NaN
        # (the not-finite exit, status BREAKDOWN)
        b, bp = _c(b, np.complex128)
        x = np.zeros_like(b) if x0 is None else np.array(x0, np.complex128, order="C")
        info = _Info()
        cap = 4 * maxit + 8
        hist = np.zeros(cap, np.float64)
        lib().orc_bicgstab_ex2(self._ptr, bp, x.ctypes.data_as(ctypes.c_void_p), rtol,
                               maxit, precond, ctypes.byref(info),
                               hist.ctypes.data_as(ctypes.c_void_p), cap, int(force_breakdown_at),
                               int(true_res_every), int(nan_at))
        out = dict(iters=info.halfsteps / 2.0, halfsteps=info.halfsteps,
                   rel_res=info.rel_res, restarts=info.restarts,
                   status=info.status, vcycles=info.vcycles)
        if history:
            out["history"] = hist[: info.halfsteps + 1].copy()
        return x, out
