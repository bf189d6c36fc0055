"""ctypes binding of libhmg (include/hmg.h): argument marshalling only.

Every computation runs in the HIP library; this module raises ``ImportError``
when ``libhmg.so`` has not been built, and never falls back to CPU code.
Host arrays are numpy (``complex128`` fields and ``float64`` wavenumbers of
shape ``(n+2, n+2)``, indexed ``[j, i]``); device arrays for the ``*_dev``
calls are torch tensors (PyTorch provides device memory and streams only).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhmg.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        "libhmg.so is not built (run __graft_entry__.build() or "
        "python -m paper_1312_2880_amd.build)")

_lib = ctypes.CDLL(LIB_PATH)

OK, ERR_INVALID, ERR_NOMEM, ERR_DEVICE, ERR_NOT_CONVERGED = 0, 1, 2, 3, 4
ERR_BREAKDOWN, PENDING, ERR_TOO_LARGE, ERR_UNKNOWN_TICKET, ERR_CANCELLED = 5, 6, 7, 8, 9
SL, HLM, HYB = 0, 1, 2
FP64, MIXED = 0, 1
SM_GS, SM_KACZ, SM_LU = 0, 1, 2
INFO_KH_ABOVE_GUIDE = 1
INFO_BATCHED = 2
ORDER_COLOUR, ORDER_LEX = 0, 1
MAX_LEVELS = 24
STATUS_NAMES = {0: "OK", 1: "INVALID", 2: "NOMEM", 3: "DEVICE", 4: "NOT_CONVERGED",
                5: "BREAKDOWN", 6: "PENDING", 7: "TOO_LARGE", 8: "UNKNOWN_TICKET",
                9: "CANCELLED"}


class HmgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int), ("precision", ctypes.c_int),
                ("beta", ctypes.c_double), ("nu_pre", ctypes.c_int),
                ("nu_post", ctypes.c_int), ("kacz_pre", ctypes.c_int),
                ("kacz_post", ctypes.c_int), ("kacz_band", ctypes.c_int),
                ("coarsest_n", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("one_pass_kernels", ctypes.c_int), ("autotune", ctypes.c_int),
                ("bottom_dense", ctypes.c_int), ("relax_order", ctypes.c_int),
                ("breakdown_at", ctypes.c_int), ("true_res_every", ctypes.c_int),
                ("nan_at", ctypes.c_int), ("fp64_levels", ctypes.c_int),
                ("ray_n", ctypes.c_int), ("hyb_mid", ctypes.c_int)]


class Plan(ctypes.Structure):
    L = MAX_LEVELS
    _fields_ = [("nlev", ctypes.c_int), ("n", ctypes.c_int * L),
                ("H", ctypes.c_double * L), ("kHmin", ctypes.c_double * L),
                ("kHmax", ctypes.c_double * L), ("smoother", ctypes.c_int * L),
                ("sigma_relax", ctypes.c_double * L),
                ("sigma_resid", ctypes.c_double * L),
                ("pre", ctypes.c_int * L), ("post", ctypes.c_int * L)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_double), ("halfsteps", ctypes.c_int),
                ("rel_res_true", ctypes.c_double), ("status", ctypes.c_int),
                ("levels", ctypes.c_int), ("restarts", ctypes.c_int),
                ("seconds", ctypes.c_double), ("flags", ctypes.c_int)]


class Request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("h", ctypes.c_double),
                ("k", ctypes.c_void_p), ("f", ctypes.c_void_p), ("opts", Opts),
                ("rtol", ctypes.c_double), ("maxit", ctypes.c_int)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_double),
                ("rel_res_true", ctypes.c_double), ("t_arrive", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("footprint_bytes", ctypes.c_size_t), ("reused", ctypes.c_int)]


P = ctypes.c_void_p
_i, _d, _sz = ctypes.c_int, ctypes.c_double, ctypes.c_size_t
_SIGS = {
    "hmg_opts_default": (None, [P]),
    "hmg_ctx_create": (_i, [_i, _sz, P]),
    "hmg_ctx_destroy": (None, [P]),
    "hmg_last_error": (ctypes.c_char_p, []),
    "hmg_grid_create": (_i, [P, _i, _d, P, P, _i, P, P]),
    "hmg_grid_destroy": (None, [P]),
    "hmg_grid_plan": (_i, [P, P]),
    "hmg_grid_set_rhs": (_i, [P, _i, P]),
    "hmg_grid_footprint": (_sz, [P]),
    "hmg_vcycle": (_i, [P, P, P]),
    "hmg_vcycle_dev": (_i, [P, P, P, P]),
    "hmg_solve": (_i, [P, P, P, _d, _i, P]),
    "hmg_solve_dev": (_i, [P, _i, P, P, _i, _d, _i, P, P]),
    "hmg_solve_dev_static": (_i, [P, _i, P, P, _i, _d, _i, P, P]),
    "hmg_ray_correct_dev": (_i, [P, P, P, P]),
    "hmg_solve_cycles": (_i, [P, P, P, _d, _i, P]),
    "hmg_solve_batch": (_i, [P, _i, P, P, _d, _i, P]),
    "hmg_submit": (_i, [P, P, P]),
    "hmg_poll": (_i, [P, ctypes.c_uint64, P, P]),
    "hmg_cancel": (_i, [P, ctypes.c_uint64]),
    "hmg_ctx_set_max_active": (_i, [P, _i]),
    "hmg_ctx_clock": (_d, [P]),
    "hmg_op_apply_dev": (_i, [P, _i, _d, P, P, P]),
    "hmg_op_smooth_dev": (_i, [P, _i, _i, _d, _i, _i, P, P, P]),
    "hmg_op_smooth_lex_dev": (_i, [P, _i, _i, _d, _i, _i, P, P, P]),
    "hmg_op_restrict_dev": (_i, [P, _i, _d, P, P, P, P]),
    "hmg_op_prolong_dev": (_i, [P, _i, P, P, P]),
    "hmg_op_coarsest_dev": (_i, [P, P, P, P]),
    "hmg_op_gs_down_dev": (_i, [P, _i, _d, _d, P, P, P, P]),
    "hmg_op_gs_up_dev": (_i, [P, _i, _d, P, P, P, P, P]),
    "hmg_op_kacz_tiled_dev": (_i, [P, _i, _d, _i, P, P, P, P, P]),
    "hmg_op_gs_up_product_dev": (_i, [P, _i, _d, _i, P, P, P, P, P, P, P]),
    "hmg_kacz_tile_config": (_i, [_i, P, P, P]),
    "hmg_kacz_tile_height": (_i, [_i]),
    "hmg_op_kacz_down_dev": (_i, [P, _i, _d, _d, _i, P, P, P, P, P]),
    "hmg_op_kacz_level_dev": (_i, [P, _i, _d, _d, _i, P, P, P, P, P, P]),
    "hmg_solve_history": (_i, [P, _i, P, _i]),
    "hmg_grid_kacz_config": (_i, [P, _i]),
}
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = tuple(_SIGS)


def kacz_tile_configs():
    """[(tile width, sweeps per launch, workgroup size)] of the tiled
    Kaczmarz kernel (kacz_tile_height gives the height)."""
    t, s, w = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    n = _lib.hmg_kacz_tile_config(0, None, None, None)
    out = []
    for c in range(n):
        _lib.hmg_kacz_tile_config(c, ctypes.byref(t), ctypes.byref(s), ctypes.byref(w))
        out.append((t.value, s.value, w.value))
    return out


def kacz_tile_height(config: int) -> int:
    """Tile height of a Kaczmarz tile configuration (its width for square
    tiles)."""
    return _lib.hmg_kacz_tile_height(config)


def _check(status, allow=(OK,)):
    if status not in allow:
        raise HmgError(status, _lib.hmg_last_error().decode())
    return status


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dptr(t):
    """Device pointer of a torch tensor (or an int / None)."""
    if t is None:
        return None
    if isinstance(t, int):
        return ctypes.c_void_p(t)
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def opts(**kw) -> Opts:
    o = Opts()
    _lib.hmg_opts_default(ctypes.byref(o))
    for key, val in kw.items():
        if not hasattr(o, key):
            raise KeyError(key)
        setattr(o, key, val)
    return o


class Context:
    def __init__(self, device: int = 0, budget_bytes: int = 0):
        h = ctypes.c_void_p()
        _check(_lib.hmg_ctx_create(device, budget_bytes, ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        # at interpreter exit the module globals may already be gone; the
        # process end releases the device memory then
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hmg_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def clock(self) -> float:
        return _lib.hmg_ctx_clock(self._h)

    def set_max_active(self, n: int):
        _check(_lib.hmg_ctx_set_max_active(self._h, n))

    # ---- serving ----
    def submit(self, n, h, k, f, rtol=1e-6, maxit=500, **kw) -> int:
        k = np.ascontiguousarray(k, np.float64)
        f = np.ascontiguousarray(f, np.complex128)
        req = Request(n=n, h=h, k=_ptr(k).value, f=_ptr(f).value, opts=opts(**kw),
                      rtol=rtol, maxit=maxit)
        t = ctypes.c_uint64()
        _check(_lib.hmg_submit(self._h, ctypes.byref(req), ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int, n: int | None = None):
        """Returns None while pending, else (x or None, result dict)."""
        res = Result()
        x = None if n is None else np.empty((n + 2, n + 2), np.complex128)
        st = _lib.hmg_poll(self._h, ticket, None if x is None else _ptr(x), ctypes.byref(res))
        if st == PENDING:
            return None
        if st not in (OK, ERR_NOT_CONVERGED, ERR_CANCELLED, ERR_BREAKDOWN):
            _check(st)
        out = {f: getattr(res, f) for f, _ in Result._fields_}
        out["status"] = st
        return (x if st != ERR_CANCELLED else None), out

    def cancel(self, ticket: int):
        _check(_lib.hmg_cancel(self._h, ticket))

    def solve_batch(self, grids, rtol=1e-6, maxit=500):
        count = len(grids)
        handles = (ctypes.c_void_p * count)(*[g._h.value for g in grids])
        xs = [np.zeros((g.nrhs, g.n + 2, g.n + 2), np.complex128) for g in grids]
        infos = [(SolveInfo * g.nrhs)() for g in grids]
        xp = (ctypes.c_void_p * count)(*[_ptr(x).value for x in xs])
        ip = (ctypes.c_void_p * count)(*[ctypes.addressof(i) for i in infos])
        st = _lib.hmg_solve_batch(self._h, count, handles, xp, rtol, maxit, ip)
        _check(st, (OK, ERR_NOT_CONVERGED, ERR_BREAKDOWN))
        return xs, [[_info_dict(i) for i in inf] for inf in infos]


def _info_dict(i: SolveInfo) -> dict:
    return {f: getattr(i, f) for f, _ in SolveInfo._fields_}


class Grid:
    """One problem (n, h, k, f) and its multigrid hierarchy on the device."""

    def __init__(self, ctx: Context, h, k, f=None, nrhs=None, **kw):
        k = np.ascontiguousarray(k, np.float64)
        n = k.shape[0] - 2
        if f is not None:
            f = np.ascontiguousarray(f, np.complex128)
            if f.ndim == 2:
                f = f[None]
            nrhs = f.shape[0] if nrhs is None else nrhs
            assert f.shape == (nrhs, n + 2, n + 2)
        nrhs = 1 if nrhs is None else nrhs
        self.ctx, self.n, self.h, self.nrhs = ctx, n, float(h), nrhs
        self.opts = opts(**kw)
        hdl = ctypes.c_void_p()
        _check(_lib.hmg_grid_create(ctx.handle, n, self.h, _ptr(k),
                                    None if f is None else _ptr(f), nrhs,
                                    ctypes.byref(self.opts), ctypes.byref(hdl)))
        self._h = hdl

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.hmg_grid_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    @property
    def footprint(self) -> int:
        return _lib.hmg_grid_footprint(self._h)

    def plan(self) -> list[dict]:
        p = Plan()
        _check(_lib.hmg_grid_plan(self._h, ctypes.byref(p)))
        names = {SM_GS: "GS", SM_KACZ: "KACZ", SM_LU: "LU"}
        return [dict(n=p.n[l], H=p.H[l], kHmin=p.kHmin[l], kHmax=p.kHmax[l],
                     smoother=names[p.smoother[l]], sigma_relax=p.sigma_relax[l],
                     sigma_resid=p.sigma_resid[l], pre=p.pre[l], post=p.post[l])
                for l in range(p.nlev)]

    def kacz_config(self, level: int) -> int:
        """Index of the tiled-Kaczmarz configuration used on `level` (-1: none)."""
        return _lib.hmg_grid_kacz_config(self._h, level)

    def set_rhs(self, rhs: int, f):
        f = np.ascontiguousarray(f, np.complex128)
        _check(_lib.hmg_grid_set_rhs(self._h, rhs, _ptr(f)))

    def vcycle(self, r):
        r = np.ascontiguousarray(r, np.complex128)
        z = np.empty_like(r)
        _check(_lib.hmg_vcycle(self._h, _ptr(r), _ptr(z)))
        return z

    def vcycle_dev(self, d_r, d_z, stream=None):
        _check(_lib.hmg_vcycle_dev(self._h, _dptr(d_r), _dptr(d_z), _stream(stream)))

    def solve(self, rtol=1e-6, maxit=500, x0=None):
        """Solve every right-hand side; x0: initial guesses (nrhs fields, or
        one field for nrhs = 1), None for zero."""
        x = np.zeros((self.nrhs, self.n + 2, self.n + 2), np.complex128)
        x0p = None
        if x0 is not None:
            x0 = np.ascontiguousarray(np.broadcast_to(x0, x.shape), np.complex128)
            x0p = _ptr(x0)
        infos = (SolveInfo * self.nrhs)()
        st = _lib.hmg_solve(self._h, x0p, _ptr(x), rtol, maxit, infos)
        _check(st, (OK, ERR_NOT_CONVERGED, ERR_BREAKDOWN))
        return x, [_info_dict(i) for i in infos]

    def solve_cycles(self, rtol=1e-7, maxit=200, x0=None):
        """The preconditioner as a stationary solver, x <- x + B (f - L x)
        (Section 6.1); info["iters"] counts cycles."""
        x = np.zeros((self.nrhs, self.n + 2, self.n + 2), np.complex128)
        x0p = None
        if x0 is not None:
            x0 = np.ascontiguousarray(np.broadcast_to(x0, x.shape), np.complex128)
            x0p = _ptr(x0)
        infos = (SolveInfo * self.nrhs)()
        st = _lib.hmg_solve_cycles(self._h, x0p, _ptr(x), rtol, maxit, infos)
        _check(st, (OK, ERR_NOT_CONVERGED))
        return x, [_info_dict(i) for i in infos]

    def history(self, rhs=0):
        """Relative residual per half iteration of the last solve of `rhs`."""
        n = _lib.hmg_solve_history(self._h, rhs, None, 0)
        if n < 0:
            _check(ERR_INVALID)
        out = np.zeros(n, np.float64)
        _lib.hmg_solve_history(self._h, rhs, _ptr(out), n)
        return out

    def solve_dev(self, d_x, d_b=None, rhs=0, x0=False, rtol=1e-6, maxit=500, stream=None):
        info = SolveInfo()
        st = _lib.hmg_solve_dev(self._h, rhs, _dptr(d_b), _dptr(d_x), int(x0), rtol, maxit,
                                ctypes.byref(info), _stream(stream))
        _check(st, (OK, ERR_NOT_CONVERGED, ERR_BREAKDOWN))
        return _info_dict(info)

    def solve_dev_static(self, d_x, d_b=None, rhs=0, x0=False, rtol=1e-6, maxit=500, stream=None):
        """hmg_solve_dev without device allocation (partials and history in
        the library's fixed per-GPU array; no history record afterwards)."""
        info = SolveInfo()
        st = _lib.hmg_solve_dev_static(self._h, rhs, _dptr(d_b), _dptr(d_x), int(x0), rtol, maxit,
                                       ctypes.byref(info), _stream(stream))
        _check(st, (OK, ERR_NOT_CONVERGED, ERR_BREAKDOWN))
        return _info_dict(info)

    def ray_correct_dev(self, d_r, d_z, stream=None):
        """z += P (P^H L P)^{-1} P^H (r - L z) on FP64 finest-level fields
        (Section 6.1 ray correction; the grid needs ray_n > 0)."""
        _check(_lib.hmg_ray_correct_dev(self._h, _dptr(d_r), _dptr(d_z), _stream(stream)))

    # ---- single building blocks on device fields (level precision) ----
    def op_apply(self, level, sigma, d_u, d_out, stream=None):
        _check(_lib.hmg_op_apply_dev(self._h, level, sigma, _dptr(d_u), _dptr(d_out),
                                     _stream(stream)))

    def op_smooth(self, level, smoother, sigma, sweeps, zero_guess, d_f, d_u, stream=None):
        _check(_lib.hmg_op_smooth_dev(self._h, level, smoother, sigma, sweeps, zero_guess,
                                      _dptr(d_f), _dptr(d_u), _stream(stream)))

    def op_smooth_lex(self, level, smoother, sigma, sweeps, zero_guess, d_f, d_u, stream=None):
        _check(_lib.hmg_op_smooth_lex_dev(self._h, level, smoother, sigma, sweeps, zero_guess,
                                          _dptr(d_f), _dptr(d_u), _stream(stream)))

    def op_restrict(self, level, sigma, d_f, d_u, d_fc, stream=None):
        _check(_lib.hmg_op_restrict_dev(self._h, level, sigma, _dptr(d_f), _dptr(d_u),
                                        _dptr(d_fc), _stream(stream)))

    def op_prolong(self, level, d_ec, d_u, stream=None):
        _check(_lib.hmg_op_prolong_dev(self._h, level, _dptr(d_ec), _dptr(d_u),
                                       _stream(stream)))

    def op_gs_down(self, level, sigma_relax, sigma_resid, d_f, d_u, d_fc, stream=None):
        _check(_lib.hmg_op_gs_down_dev(self._h, level, sigma_relax, sigma_resid, _dptr(d_f),
                                       _dptr(d_u), _dptr(d_fc), _stream(stream)))

    def op_gs_up(self, level, sigma_relax, d_f, d_ec, d_uo, stream=None, d_u0=None):
        _check(_lib.hmg_op_gs_up_dev(self._h, level, sigma_relax, _dptr(d_f), _dptr(d_u0),
                                     _dptr(d_ec), _dptr(d_uo), _stream(stream)))

    def op_gs_up_product(self, level, sigma_relax, kind, d_f, d_ec, d_uo, d_mv, d_dot, d_sums, stream=None):
        _check(_lib.hmg_op_gs_up_product_dev(self._h, level, sigma_relax, kind, _dptr(d_f), _dptr(d_ec),
                                             _dptr(d_uo), _dptr(d_mv), _dptr(d_dot), _dptr(d_sums),
                                             _stream(stream)))

    def op_kacz_tiled(self, level, sigma, config, d_f, d_ui, d_ec, d_uo, stream=None):
        _check(_lib.hmg_op_kacz_tiled_dev(self._h, level, sigma, config, _dptr(d_f), _dptr(d_ui),
                                          _dptr(d_ec), _dptr(d_uo), _stream(stream)))

    def op_kacz_down(self, level, sigma_relax, sigma_resid, config, d_f, d_ui, d_uo, d_fc, stream=None):
        _check(_lib.hmg_op_kacz_down_dev(self._h, level, sigma_relax, sigma_resid, config, _dptr(d_f),
                                         _dptr(d_ui), _dptr(d_uo), _dptr(d_fc), _stream(stream)))

    def op_kacz_level(self, level, sigma_relax, sigma_resid, sweeps, d_f, d_ui, d_ec, d_uo, d_fc,
                      stream=None):
        _check(_lib.hmg_op_kacz_level_dev(self._h, level, sigma_relax, sigma_resid, sweeps, _dptr(d_f),
                                          _dptr(d_ui), _dptr(d_ec), _dptr(d_uo), _dptr(d_fc),
                                          _stream(stream)))

    def op_coarsest(self, d_f, d_u, stream=None):
        _check(_lib.hmg_op_coarsest_dev(self._h, _dptr(d_f), _dptr(d_u), _stream(stream)))
