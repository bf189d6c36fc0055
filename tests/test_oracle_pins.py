"""Pins of the FP64 oracle against facts that do not come from the oracle:
closed forms of the paper, numbers it prints, an independent dense-matrix
construction, numpy's direct solver, and brute force on tiny grids.

Each test names the passage of Livshits, arXiv:1312.2880 that fixes it.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import lfa
from tests import dense_ref as D

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
BETA = 0.5


def rng_k(n, seed, lo, hi):
    return np.random.default_rng(seed).uniform(lo, hi, (n + 2, n + 2))


def rng_c(shape, seed):
    g = np.random.default_rng(seed)
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


# ---------------------------------------------------------------------------
# Operator (Section 1 eq:diff / eq:disc, eq:mh; Section 3 symbols)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("sigma", [0.0, BETA])
def test_interior_rows_match_plane_wave_symbol(sigma):
    """Interior rows of L^h and M^h on exp(i(t1 i + t2 j)) give the symbol
    used in eq. symb:helmholtz / symb:shifted:
    (2cos t1 + 2cos t2 - 4 + k^2 h^2 (1 + i sigma)) / h^2."""
    n, h, k0 = 31, 1 / 32, 17.0
    k = np.full((n + 2, n + 2), k0)
    t1, t2 = 0.7, -1.9
    jj, ii = np.meshgrid(np.arange(n + 2), np.arange(n + 2), indexing="ij")
    u = np.exp(1j * (t1 * ii + t2 * jj))
    out = oracle.apply(h, k, sigma, u)
    sym = (2 * math.cos(t1) + 2 * math.cos(t2) - 4 + (k0 * h) ** 2 * (1 + 1j * sigma)) / h ** 2
    inner = (slice(1, -1), slice(1, -1))
    np.testing.assert_allclose(out[inner], sym * u[inner], rtol=1e-12, atol=0)


@pytest.mark.parametrize("n", [1, 3, 7])
@pytest.mark.parametrize("sigma", [0.0, BETA])
def test_operator_equals_ghost_point_construction(n, sigma):
    """Every row, boundary and corner included, equals the plain 5-point
    stencil applied to the grid extended with ghost values from the central
    difference of du/dn - i k u = 0 (Section 1, Sommerfeld condition)."""
    h = 1.0 / (n + 1)
    k = rng_k(n, 10 + n, 2.0, 9.0)
    A_ref = D.assemble_ghost(n, h, k, sigma)
    A = oracle.dense(h, k, sigma)
    np.testing.assert_allclose(A, A_ref, rtol=1e-13, atol=1e-13 * np.abs(A_ref).max())


def test_shift_adds_i_beta_k2_on_every_diagonal():
    """eq:mh: M^h - L^h = i beta k^2 (diagonal, boundary rows included)."""
    n, h = 7, 1 / 8
    k = rng_k(n, 3, 1.0, 12.0)
    diff = oracle.dense(h, k, BETA) - oracle.dense(h, k, 0.0)
    np.testing.assert_allclose(diff, np.diag(1j * BETA * k.reshape(-1) ** 2), atol=1e-12)


# ---------------------------------------------------------------------------
# Manufactured solution: second-order consistency of the discretisation
# ---------------------------------------------------------------------------

def manufactured(n, k0, kfun=None, a=0.3):
    """u* = exp(i k0 (x cos a + y sin a)) (1 + x y^2); f = Lap u* + k^2 u*,
    boundary data g = du*/dn - i k u* folded into the boundary rows
    (u(-1) = u(1) + 2ikh u(0) + 2 h g  =>  row p gets f_p - 2 g_p / h)."""
    h = 1.0 / (n + 1)
    x = np.arange(n + 2) * h
    Y, X = np.meshgrid(x, x, indexing="ij")
    kk = np.full_like(X, k0) if kfun is None else kfun(X, Y)
    E = np.exp(1j * k0 * (X * math.cos(a) + Y * math.sin(a)))
    w = 1 + X * Y ** 2
    u = E * w
    lap = E * (-k0 ** 2 * w + 2j * k0 * (math.cos(a) * Y ** 2 + math.sin(a) * 2 * X * Y) + 2 * X)
    f = lap + kk ** 2 * u
    ux = E * (1j * k0 * math.cos(a) * w + Y ** 2)
    uy = E * (1j * k0 * math.sin(a) * w + 2 * X * Y)
    f = f.astype(np.complex128)
    N = n + 1
    f[:, 0] -= 2 * (-ux[:, 0] - 1j * kk[:, 0] * u[:, 0]) / h
    f[:, N] -= 2 * (ux[:, N] - 1j * kk[:, N] * u[:, N]) / h
    f[0, :] -= 2 * (-uy[0, :] - 1j * kk[0, :] * u[0, :]) / h
    f[N, :] -= 2 * (uy[N, :] - 1j * kk[N, :] * u[N, :]) / h
    return h, kk, f, u


@pytest.mark.parametrize("k0,variable", [(5.0, False), (10.0, False), (8.0, True)])
def test_manufactured_solution_second_order(k0, variable):
    kfun = (lambda X, Y: k0 * (1 + 0.3 * np.sin(2 * X + Y))) if variable else None
    errs = []
    for n in (31, 63, 127, 255):
        h, kk, f, u_exact = manufactured(n, k0, kfun)
        g = oracle.Grid(h, kk, variant=oracle.HYB)
        x, info = g.bicgstab(f, rtol=1e-12, maxit=400)
        assert info["status"] == oracle.OK
        errs.append(np.abs(x - u_exact).max())
    orders = [math.log2(errs[q] / errs[q + 1]) for q in range(len(errs) - 1)]
    assert 1.9 <= orders[-1] <= 2.1, (errs, orders)
    assert all(o > 1.7 for o in orders), (errs, orders)


# ---------------------------------------------------------------------------
# Dense direct solve: the solution is the plain definition x = (L^h)^{-1} f
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,coarsest", [(1, 1), (3, 1), (7, 1), (7, 3)])
@pytest.mark.parametrize("variant", [oracle.SL, oracle.HYB, oracle.HLM])
def test_bicgstab_matches_numpy_dense_solve(n, coarsest, variant):
    h = 1.0 / (n + 1)
    k = rng_k(n, 7 * n + variant, 3.0, 11.0)
    f = rng_c((n + 2, n + 2), 99 + n)
    A_ref = D.assemble_ghost(n, h, k, 0.0)
    x_ref = np.linalg.solve(A_ref, f.reshape(-1)).reshape(f.shape)
    g = oracle.Grid(h, k, variant=variant, coarsest_n=coarsest)
    x, info = g.bicgstab(f, rtol=1e-13, maxit=2000)
    assert info["status"] == oracle.OK
    np.testing.assert_allclose(x, x_ref, rtol=0, atol=1e-10 * np.abs(x_ref).max())


def test_oracle_lu_matches_numpy():
    n, h = 7, 1 / 8
    k = rng_k(n, 5, 4.0, 30.0)
    A = D.assemble_ghost(n, h, k, 0.0)
    b = rng_c(A.shape[0], 6)
    np.testing.assert_allclose(oracle.lu_solve_dense(A, b), np.linalg.solve(A, b),
                               rtol=1e-10, atol=1e-12)


def test_exact_preconditioner_converges_in_half_step():
    """Bi-CGSTAB wiring (Section 6): with B = (L^h)^{-1} the first half step
    s = r - alpha A B r vanishes, so the count is 0.5."""
    n, h = 7, 1 / 8
    k = rng_k(n, 1, 3.0, 9.0)
    f = rng_c((n + 2, n + 2), 2)
    g = oracle.Grid(h, k)
    x, info = g.bicgstab(f, rtol=1e-10, maxit=10, precond=oracle.PREC_EXACT)
    assert info["halfsteps"] == 1 and info["status"] == oracle.OK


def test_point_source_zero_initial_guess():
    """Section 6: x^0 = 0, r^0 = f; f(0.5, 0.5) = 1; the count is reported in
    half iterations (one preconditioner application per half step) and the
    final true residual meets the tolerance.  SL-V with the normal-equation
    band of Section 5."""
    n = 63
    h = 1 / 64
    k = np.full((n + 2, n + 2), 10 * math.pi)
    f = np.zeros((n + 2, n + 2), complex)
    f[32, 32] = 1.0
    g = oracle.Grid(h, k, variant=oracle.SL, kacz_band=1)
    x, info = g.bicgstab(f, rtol=1e-6, maxit=200, history=True)
    assert info["status"] == oracle.OK
    assert info["rel_res"] <= 1e-6
    assert info["history"][0] == pytest.approx(1.0)
    assert info["history"][-1] <= 1e-6
    assert info["vcycles"] == info["halfsteps"]


@pytest.mark.parametrize("K", [2, 5])
def test_forced_breakdown_restart_equals_fresh_solve(K):
    """The breakdown branch (rhat = p = r, rho_old = alpha = omega = 1) is a
    fresh Bi-CGSTAB from the current iterate: forcing it after iteration K
    must give, from half step 2K on, the history of a new solve started at
    x_K (up to the drift between the recursive and the true residual), keep
    the first 2K half steps unchanged, and still converge.  A restart that
    kept the old direction p, or the old omega, fails the comparison."""
    h, k, f = _point63()
    g = oracle.Grid(h, k, variant=oracle.SL)
    _, plain = g.bicgstab(f, rtol=1e-6, maxit=300, history=True)
    _, forced = g.bicgstab(f, rtol=1e-6, maxit=300, history=True, force_breakdown_at=K)
    xK, _ = g.bicgstab(f, rtol=1e-30, maxit=K)
    _, fresh = g.bicgstab(f, rtol=1e-6, maxit=300, x0=xK, history=True)
    hp, hf, hr = plain["history"], forced["history"], fresh["history"]
    assert forced["status"] == oracle.OK and forced["restarts"] == 1 and plain["restarts"] == 0
    np.testing.assert_array_equal(hf[: 2 * K + 1], hp[: 2 * K + 1])
    np.testing.assert_allclose(hf[2 * K: 2 * K + 8], hr[:8], rtol=1e-6)
    assert abs(np.log(hp[2 * K + 4] / hf[2 * K + 4])) > 1e-3   # the branch changes the iteration


@pytest.mark.parametrize("K", [5, 10])
def test_true_residual_every_k_restarts_from_true_residual(K):
    """true_res_every = K: after iteration K the residual is recomputed as
    b - L x and the iteration restarts from it.  The first 2K half steps are
    the plain solve's; the next ones follow a fresh solve started at x_K,
    whose initial residual is the true residual (so the entry at 2K is the
    true, not the recursive, relative residual); every restart is counted."""
    h, k, f = _point63()
    g = oracle.Grid(h, k, variant=oracle.SL)
    _, plain = g.bicgstab(f, rtol=1e-6, maxit=300, history=True)
    _, every = g.bicgstab(f, rtol=1e-6, maxit=300, history=True, true_res_every=K)
    xK, _ = g.bicgstab(f, rtol=1e-30, maxit=K)
    _, fresh = g.bicgstab(f, rtol=1e-6, maxit=300, x0=xK, history=True)
    hp, he, hr = plain["history"], every["history"], fresh["history"]
    assert every["status"] == oracle.OK and every["rel_res"] <= 1e-6
    np.testing.assert_array_equal(he[: 2 * K + 1], hp[: 2 * K + 1])
    # entries 2K+1.. of the periodic solve equal those of the fresh solve
    np.testing.assert_allclose(he[2 * K + 1: 4 * K + 1], hr[1: 2 * K + 1], rtol=1e-9)
    true_rel = np.linalg.norm(f - oracle.apply(h, k, 0.0, xK)) / np.linalg.norm(f)
    assert hr[0] == pytest.approx(true_rel, rel=1e-12)
    assert every["restarts"] == (every["halfsteps"] - 1) // (2 * K)


def test_not_finite_residual_ends_with_breakdown():
    """A residual norm that is not finite ends the solve with status
    BREAKDOWN after that half step, x holding the iterate of that step (the
    test forces the norm after iteration 4 to NaN; x then equals the iterate
    of a solve stopped by maxit after 4 iterations)."""
    h, k, f = _point63()
    g = oracle.Grid(h, k, variant=oracle.SL)
    x, info = g.bicgstab(f, rtol=1e-6, maxit=300, nan_at=4)
    x4, info4 = g.bicgstab(f, rtol=1e-30, maxit=4)
    assert info["status"] == oracle.BREAKDOWN and info["halfsteps"] == 8
    assert info4["status"] == oracle.NOT_CONVERGED
    np.testing.assert_array_equal(x, x4)


def _point63():
    n = 63
    k = np.full((n + 2, n + 2), 10 * math.pi)
    f = np.zeros((n + 2, n + 2), complex)
    f[32, 32] = 1.0
    return 1 / 64, k, f


# ---------------------------------------------------------------------------
# Transfers (Section 5: bilinear interpolation, full weighting)
# ---------------------------------------------------------------------------

def test_restriction_of_constant_is_constant():
    n = 15
    fc = oracle.restrict_fw(np.full((n + 2, n + 2), 3.0 - 2.0j))
    np.testing.assert_allclose(fc, 3.0 - 2.0j, rtol=1e-15)


def test_prolongation_exact_on_bilinear():
    nc = 7
    Xc = np.arange(nc + 2) / (nc + 1)
    Yc, Xc2 = np.meshgrid(Xc, Xc, indexing="ij")
    ec = (1 + 2 * Xc2 - 3 * Yc + 0.5 * Xc2 * Yc) * (1 + 1j)
    n = 2 * nc + 1
    X = np.arange(n + 2) / (n + 1)
    Y, X2 = np.meshgrid(X, X, indexing="ij")
    want = (1 + 2 * X2 - 3 * Y + 0.5 * X2 * Y) * (1 + 1j)
    got = oracle.prolong_add(ec, np.zeros((n + 2, n + 2), complex))
    np.testing.assert_allclose(got, want, rtol=1e-14, atol=1e-14)


def test_transfers_match_matrix_definitions():
    """R (mirrored full weighting) and P (bilinear) as matrices; in the
    interior R = P^T / 4 entrywise."""
    n = 15
    nc = 7
    R = D.restriction_matrix(n)
    P = D.prolongation_matrix(nc)
    r = rng_c((n + 2, n + 2), 4)
    np.testing.assert_allclose(oracle.restrict_fw(r).reshape(-1), R @ r.reshape(-1),
                               rtol=1e-14, atol=1e-14)
    e = rng_c((nc + 2, nc + 2), 5)
    u0 = rng_c((n + 2, n + 2), 6)
    np.testing.assert_allclose(oracle.prolong_add(e, u0).reshape(-1),
                               u0.reshape(-1) + P @ e.reshape(-1), rtol=1e-14, atol=1e-14)
    Mc = nc + 2
    interior = [J * Mc + I for J in range(1, Mc - 1) for I in range(1, Mc - 1)]
    np.testing.assert_allclose(R[interior], P.T[interior] / 4, atol=1e-15)


# ---------------------------------------------------------------------------
# Colourings (red-black, 5-colour)
# ---------------------------------------------------------------------------

def test_five_colouring_brute_force():
    """(i + 2j) mod 5 differs for every pair at Manhattan distance 1 or 2, and
    the 5-point stencils of one colour cover Z^2 exactly once."""
    for di in range(-2, 3):
        for dj in range(-2, 3):
            if 1 <= abs(di) + abs(dj) <= 2:
                assert (di + 2 * dj) % 5 != 0
    L = 40
    for c in range(5):
        cover = np.zeros((L, L), int)
        for j in range(-1, L + 1):
            for i in range(-1, L + 1):
                if (i + 2 * j) % 5 == c:
                    for di, dj in ((0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)):
                        ii, jj = i + di, j + dj
                        if 0 <= ii < L and 0 <= jj < L:
                            cover[jj, ii] += 1
        assert (cover == 1).all()


# ---------------------------------------------------------------------------
# Relaxation (Section 4)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kappa,sigma", [(0.3125, 0.0), (0.625, BETA), (1.25, 0.0),
                                         (1.25, BETA), (2.5, 0.0), (5.0, BETA)])
def test_lex_gs_sweep_matches_conv_formula(kappa, sigma):
    """One oracle lexicographic GS sweep on a plane-wave error: far from the
    sweep start the amplitude ratio is mu(-theta) of eq. conv:helmholtz /
    conv:shifted (the sign of theta is the paper's convention)."""
    n = 255
    H = 1.0 / (n + 1)
    k = np.full((n + 2, n + 2), kappa / H)
    t1, t2 = 2.1, 2.6
    jj, ii = np.meshgrid(np.arange(n + 2), np.arange(n + 2), indexing="ij")
    e0 = np.exp(1j * (t1 * ii + t2 * jj))
    e1 = oracle.gs_lex(H, k, sigma, np.zeros_like(e0), e0)
    ratio = np.abs(e1[120:200, 120:200] / e0[120:200, 120:200])
    mu = lfa.gs_lex_amplification(-t1, -t2, kappa, sigma)
    tol = 1e-3 if kappa == 1.25 else 1e-6
    np.testing.assert_allclose(ratio, mu, rtol=tol)


@pytest.mark.parametrize("kappa,sigma", [(0.98, BETA), (1.963, BETA), (0.5, 0.0), (3.0, 0.0)])
def test_red_black_sweep_plane_wave_factors(kappa, sigma):
    """Red-black order (red = (i+j) even first): red nodes are multiplied by
    -s/d, black nodes by (s/d)^2, exactly, away from the boundary."""
    n = 31
    H = 1.0 / (n + 1)
    k = np.full((n + 2, n + 2), kappa / H)
    t1, t2 = 0.4, 1.3
    jj, ii = np.meshgrid(np.arange(n + 2), np.arange(n + 2), indexing="ij")
    e0 = np.exp(1j * (t1 * ii + t2 * jj))
    e1 = oracle.gs_rb(H, k, sigma, np.zeros_like(e0), e0)
    red_f, black_f = lfa.rb_plane_wave_factors(t1, t2, kappa, sigma)
    sl = (slice(2, -2), slice(2, -2))
    red = ((ii + jj) % 2 == 0)[sl]
    ratio = (e1 / e0)[sl]
    np.testing.assert_allclose(ratio[red], red_f, rtol=1e-11)
    np.testing.assert_allclose(ratio[~red], black_f, rtol=1e-11)


@pytest.mark.parametrize("order", ["lex", "5c"])
@pytest.mark.parametrize("sigma", [0.0, BETA])
def test_kaczmarz_error_is_monotone(order, sigma):
    """Row-action reading of the normal-equation relaxation (Section 4): each
    row update is an orthogonal projection onto {u: a_p u = f_p}, so for a
    consistent system the error 2-norm never grows."""
    n = 15
    H = 1.0 / (n + 1)
    k = np.full((n + 2, n + 2), 1.25 / H)
    u_star = rng_c((n + 2, n + 2), 8)
    f = oracle.apply(H, k, sigma, u_star)
    u = np.zeros_like(f)
    sweep = oracle.kacz_lex if order == "lex" else oracle.kacz_5c
    prev = np.linalg.norm(u - u_star)
    for _ in range(6):
        u = sweep(H, k, sigma, f, u)
        cur = np.linalg.norm(u - u_star)
        assert cur <= prev * (1 + 1e-15)
        prev = cur
    assert prev < np.linalg.norm(u_star)


@pytest.mark.parametrize("sweep,ref", [
    ("gs_lex", "lex"), ("gs_rb", "rb"), ("kacz_lex", "klex"), ("kacz_5c", "k5")])
@pytest.mark.parametrize("sigma", [0.0, BETA])
def test_sweeps_match_matrix_forms(sweep, ref, sigma):
    n = 7
    H = 1 / 8
    k = rng_k(n, 12, 6.0, 12.0)
    f = rng_c((n + 2, n + 2), 13)
    u0 = rng_c((n + 2, n + 2), 14)
    A = D.assemble_ghost(n, H, k, sigma)
    fv, uv = f.reshape(-1), u0.reshape(-1)
    want = {"lex": lambda: D.sweep_gs_lex(A, fv, uv),
            "rb": lambda: D.sweep_gs_colour(A, fv, uv, D.colour_rb(n), 2),
            "klex": lambda: D.sweep_kacz_lex(A, fv, uv),
            "k5": lambda: D.sweep_kacz_colour(A, fv, uv, D.colour_5(n), 5)}[ref]()
    got = getattr(oracle, sweep)(H, k, sigma, f, u0).reshape(-1)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


# ---------------------------------------------------------------------------
# Level plan and V-cycle (Section 5)
# ---------------------------------------------------------------------------

def test_plan_point_source_sl_gs_everywhere():
    """63^2, k = 10 pi, SL with Gauss-Seidel on M on every level (no
    normal-equation band): GS(M) on 63, 31, 15 and LU of M on 7."""
    n = 63
    g = oracle.Grid(1 / 64, np.full((65, 65), 10 * math.pi), variant=oracle.SL, kacz_band=0)
    plan = g.plan()
    assert [p["n"] for p in plan] == [63, 31, 15, 7]
    assert [p["smoother"] for p in plan] == ["GS", "GS", "GS", "LU"]
    assert all(p["sigma_relax"] == BETA and p["sigma_resid"] == BETA for p in plan)
    assert [p["pre"] for p in plan[:3]] == [1, 1, 1]


def test_plan_hybrid_constant_k():
    """HYB-V (Section 5): L for residuals everywhere; M for relaxation near
    kH = 0.625; normal-equation relaxation (4 + 4) near kH = 1.25; L for
    relaxation elsewhere and on the coarsest level."""
    n = 255
    h = 1 / 256
    k = np.full((n + 2, n + 2), 0.3125 / h)     # kH = 0.3125, 0.625, 1.25, 2.5, 5, ...
    plan = oracle.Grid(h, k, variant=oracle.HYB).plan()
    sm = [(p["smoother"], p["sigma_relax"], p["pre"]) for p in plan]
    assert sm[0] == ("GS", 0.0, 1)
    assert sm[1] == ("GS", BETA, 1)
    assert sm[2] == ("KACZ", BETA, 4)
    assert sm[3] == ("GS", 0.0, 1)            # kH = 2.5
    assert sm[-1][0] == "LU" and sm[-1][1] == 0.0
    assert all(p["sigma_resid"] == 0.0 for p in plan)
    sl = oracle.Grid(h, k, variant=oracle.SL).plan()
    assert [p["smoother"] for p in sl[:3]] == ["GS", "GS", "KACZ"]
    assert all(p["sigma_relax"] == BETA and p["sigma_resid"] == BETA for p in sl)
    hlm = oracle.Grid(h, k, variant=oracle.HLM).plan()
    assert hlm[2]["smoother"] == "KACZ" and hlm[2]["sigma_relax"] == 0.0


def test_plan_hybrid_with_intermediate_scales_on_m():
    """hyb_mid (HYB-V): the relaxation operator is M on the levels up to
    kH ~ 2.5 (here kH = 0.625, 1.25 and 2.5), L on the finest (0.3125) and
    on the coarsest scales (5 and beyond); residuals stay on L; SL-V and
    HLM-V ignore the option."""
    n = 255
    h = 1 / 256
    k = np.full((n + 2, n + 2), 0.3125 / h)     # kH = 0.3125, 0.625, 1.25, 2.5, 5, 10
    plan = oracle.Grid(h, k, variant=oracle.HYB, hyb_mid=1).plan()
    assert [(p["smoother"], p["sigma_relax"]) for p in plan] == [
        ("GS", 0.0), ("GS", BETA), ("KACZ", BETA), ("GS", BETA), ("GS", 0.0), ("LU", 0.0)]
    assert all(p["sigma_resid"] == 0.0 for p in plan)
    for variant in (oracle.SL, oracle.HLM):
        assert oracle.Grid(h, k, variant=variant, hyb_mid=1).plan() == oracle.Grid(h, k, variant=variant).plan()


def test_plan_between_the_kaczmarz_band_and_kh_2_5():
    """Section 4: Gauss-Seidel is good only up to kH ~ 0.625 and from ~2.5 on;
    a level between the 1.25 band and 2.5 (here kH = 2.0, where Gauss-Seidel
    on L also loses its pivot) takes the normal-equation relaxation on the
    variant's operator: M for SL-V, L for HYB-V and HLM-V.  Levels at
    kH = 0.3125 * 2^j (the paper's grids) are unaffected (the plan test of
    the constant-k hierarchy above)."""
    n = 127
    h = 1 / 128
    k = np.full((n + 2, n + 2), 0.5 / h)      # kH = 0.5, 1.0, 2.0, 4.0, 8.0
    want = {oracle.SL: [("GS", BETA), ("KACZ", BETA), ("KACZ", BETA), ("GS", BETA), ("LU", BETA)],
            oracle.HYB: [("GS", BETA), ("KACZ", BETA), ("KACZ", 0.0), ("GS", 0.0), ("LU", 0.0)],
            oracle.HLM: [("GS", 0.0), ("KACZ", 0.0), ("KACZ", 0.0), ("GS", 0.0), ("LU", 0.0)]}
    for variant, plan_want in want.items():
        plan = oracle.Grid(h, k, variant=variant).plan()
        assert [(p["smoother"], p["sigma_relax"]) for p in plan] == plan_want, variant
        assert all(p["pre"] == 4 for p in plan if p["smoother"] == "KACZ")
    # kH = 2.5 exactly stays Gauss-Seidel (the constant-k hierarchy of Table 1)
    k = np.full((n + 2, n + 2), 0.625 / h)     # kH = 0.625, 1.25, 2.5, 5, 10
    plan = oracle.Grid(h, k, variant=oracle.SL).plan()
    assert [p["smoother"] for p in plan] == ["GS", "KACZ", "GS", "GS", "LU"]


CASES_P4 = [
    dict(variant=oracle.SL, kacz_band=0, coarsest_n=3, k=(4.0, 6.0)),
    dict(variant=oracle.SL, kacz_band=1, coarsest_n=1, k=(4.0, 6.0)),
    dict(variant=oracle.HYB, kacz_band=1, coarsest_n=1, k=(3.0, 9.0)),
    dict(variant=oracle.HLM, kacz_band=1, coarsest_n=1, k=(6.0, 10.0)),
    dict(variant=oracle.HYB, kacz_band=1, coarsest_n=1, k=(3.0, 9.0),
         gs_order=oracle.ORDER_LEX, kacz_order=oracle.ORDER_LEX),
    # HYB level with Gauss-Seidel on M and residuals on L (kH in [0.45, 0.875])
    dict(variant=oracle.HYB, kacz_band=1, coarsest_n=3, k=(3.6, 7.0)),
    # hyb_mid: Kaczmarz on M at kH in [1.25, 1.75], Gauss-Seidel on M at
    # kH in [2.5, 3.5], residuals on L
    dict(variant=oracle.HYB, kacz_band=1, coarsest_n=1, k=(10.0, 14.0), hyb_mid=1),
]


@pytest.mark.parametrize("case", CASES_P4)
def test_vcycle_equals_dense_matrix_vcycle(case):
    """The V-cycle (zero guess; pre-relax with role (A); residual with role
    (B); full weighting; recursion; bilinear correction; post-relax) equals
    the same composition written with dense matrices."""
    case = dict(case)
    lo, hi = case.pop("k")
    n, h = 7, 1 / 8
    k = rng_k(n, 21, lo, hi)
    g = oracle.Grid(h, k, **case)
    plan = g.plan()
    kinds = {p["smoother"] for p in plan}
    assert "LU" in kinds
    ref = D.DenseVCycle(h, k, plan,
                        gs_order="lex" if case.get("gs_order") == oracle.ORDER_LEX else "rb",
                        kacz_order="lex" if case.get("kacz_order") == oracle.ORDER_LEX else "5c")
    m = (n + 2) ** 2
    for col in range(0, m, 7):
        f = np.zeros(m, complex)
        f[col] = 1.0
        f[(col * 5 + 3) % m] = 0.5j
        want = ref.apply(f)
        got = g.vcycle(f.reshape(n + 2, n + 2)).reshape(-1)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("variant", [oracle.SL, oracle.HYB])
def test_vcycle_on_a_hierarchy_that_is_not_a_power_of_two(variant):
    """h = 1/20 (Table 1's grids halve 80 -> 40 -> 20 -> 10 -> 5): interval
    counts 20 -> 10 -> 5 with the coarsest level at n = 4; the V-cycle equals
    the dense-matrix composition, restriction and prolongation included."""
    n, h = 19, 1 / 20
    k = rng_k(n, 33, 8.0, 14.0)
    g = oracle.Grid(h, k, variant=variant, coarsest_n=4)
    plan = g.plan()
    assert [p["n"] for p in plan] == [19, 9, 4]
    ref = D.DenseVCycle(h, k, plan)
    m = (n + 2) ** 2
    for col in range(0, m, 11):
        f = np.zeros(m, complex)
        f[col] = 1.0
        f[(col * 7 + 5) % m] = -0.25j
        want = ref.apply(f)
        got = g.vcycle(f.reshape(n + 2, n + 2)).reshape(-1)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())


MIXED_MODES = [("fused", 2, 1, False), ("fused", 1, 3, True), ("fused", 4, 0, False),
               ("onepass", 2, 0, True), ("onepass", 2, 0, False)]


@pytest.mark.parametrize("mode", MIXED_MODES, ids=lambda m: f"{m[0]}-e{m[1]}-b{m[2]}-io{int(m[3])}")
@pytest.mark.parametrize("ci", [0, 1, 2, 3, 5])
@pytest.mark.parametrize("n", [7, 15])
def test_mixed_vcycle_equals_dense_mixed_composition(n, ci, mode):
    """Precision form (O11): the V-cycle with its fields stored in complex
    float and its arithmetic in double equals the same composition written
    with dense matrices and explicit float casts at the same stores (k on
    every level, restricted right-hand sides, coarse corrections, Kaczmarz
    iterates every `every` sweeps or every colour pass; the coarsest operator
    from the unrounded k).  The rounding itself is visible: the mixed cycle
    differs from the double one by more than 1e-9 and less than 1e-5
    relative, while the two mixed constructions agree to rounding level."""
    case = dict(CASES_P4[ci])
    lo, hi = case.pop("k")
    h = 1.0 / (n + 1)
    k = rng_k(n, 21, lo, hi) * (1 if n == 7 else 2)
    g = oracle.Grid(h, k, **case)
    plan = g.plan()
    name, every, block_n, round_io = mode
    g.set_mixed(oracle.MIX_FUSED if name == "fused" else oracle.MIX_ONEPASS, every, block_n, round_io)
    ref = D.DenseMixedVCycle(h, k, plan, name, every, block_n, round_io)
    ref64 = D.DenseVCycle(h, k, plan)
    m = (n + 2) ** 2
    effect = 0.0
    for col in range(0, m, 13):
        f = np.zeros(m, complex)
        f[col] = 1.0
        f[(col * 5 + 3) % m] = 0.5j
        want = ref.apply(f)
        got = g.vcycle(f.reshape(n + 2, n + 2)).reshape(-1)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-13 * np.abs(want).max())
        w64 = ref64.apply(f)
        effect = max(effect, np.linalg.norm(want - w64) / np.linalg.norm(w64))
    assert 1e-9 < effect < 1e-5, effect


@pytest.mark.parametrize("t", [1, 2])
@pytest.mark.parametrize("ci", [1, 3, 5])
def test_mixed_vcycle_with_double_fine_levels(ci, t):
    """Precision form with the finest t levels kept in double (their fields
    and k unrounded; level t takes and returns double fields): equals the
    dense construction with the same stores and differs from both the
    all-float and the all-double cycles."""
    n, h = 31, 1 / 32
    case = dict(CASES_P4[ci])
    lo, hi = case.pop("k")
    k = rng_k(n, 21, lo, hi) * 4
    g = oracle.Grid(h, k, **case)
    plan = g.plan()
    ref = D.DenseMixedVCycle(h, k, plan, "fused", 2, 3, False, fp64_levels=t)
    ref32 = D.DenseMixedVCycle(h, k, plan, "fused", 2, 3, False)
    ref64 = D.DenseVCycle(h, k, plan)
    g.set_mixed(oracle.MIX_FUSED, 2, 3, False, fp64_levels=t)
    m = (n + 2) ** 2
    for col in range(0, m, 97):
        f = np.zeros(m, complex)
        f[col] = 1.0
        f[(col * 5 + 3) % m] = 0.5j
        want = ref.apply(f)
        got = g.vcycle(f.reshape(n + 2, n + 2)).reshape(-1)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-13 * np.abs(want).max())
        w64, w32 = ref64.apply(f), ref32.apply(f)
        assert np.linalg.norm(want - w64) > 1e-12 * np.linalg.norm(w64)
        assert np.linalg.norm(want - w32) > 1e-12 * np.linalg.norm(w64)


def test_mixed_onepass_output_is_float():
    """With every store rounded (one-pass schedule, rounded input and
    output) the cycle's result lies on the complex-float grid, and switching
    the precision form off restores the double cycle bit for bit."""
    n, h = 15, 1 / 16
    case = dict(CASES_P4[2])
    lo, hi = case.pop("k")
    k = rng_k(n, 21, lo, hi) * 2
    g = oracle.Grid(h, k, **case)
    f = rng_c((n + 2, n + 2), 5)
    z64 = g.vcycle(f)
    g.set_mixed(oracle.MIX_ONEPASS, 1, 0, True)
    z = g.vcycle(f)
    assert np.array_equal(z, z.astype(np.complex64).astype(np.complex128))
    assert not np.array_equal(z, z64)
    g.set_mixed(oracle.MIX_OFF)
    assert np.array_equal(g.vcycle(f), z64)


def test_vcycle_plans_cover_both_smoothers():
    kinds = set()
    mixed_roles = False
    for case in CASES_P4:
        case = dict(case)
        lo, hi = case.pop("k")
        for p in oracle.Grid(1 / 8, rng_k(7, 21, lo, hi), **case).plan():
            kinds.add(p["smoother"])
            if p["smoother"] == "GS" and p["sigma_relax"] != p["sigma_resid"]:
                mixed_roles = True
    assert kinds == {"GS", "KACZ", "LU"}
    assert mixed_roles


# ---------------------------------------------------------------------------
# Ray correction (Section 6.1): plane waves in the 8 directions j pi / 4
# times smooth (bilinear) ray functions, Galerkin correction
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,ray_n", [(15, 1), (31, 3)])
def test_ray_correction_removes_errors_in_the_ray_space(n, ray_n):
    """An error that is a combination of the 8 plane waves times bilinear ray
    functions is removed exactly by one correction from u = 0: the Galerkin
    projection P (P^H L P)^{-1} P^H L is the identity on the ray space.  P is
    built independently (numpy, from the 1-D hats), so a wrong direction,
    phase sign, hat or a missing conjugate in P^H fails."""
    h = 1.0 / (n + 1)
    k = np.full((n + 2, n + 2), 0.3125 / h)
    P = D.ray_basis(n, h, k, ray_n)
    a = rng_c(P.shape[1], 3)
    e = (P @ a).reshape(n + 2, n + 2)
    f = oracle.apply(h, k, 0.0, e)
    g = oracle.Grid(h, k, variant=oracle.HLM, coarsest_n=1).set_ray(ray_n)
    u = g.ray_correct(f, np.zeros_like(f))
    np.testing.assert_allclose(u, e, rtol=0, atol=1e-10 * np.abs(e).max())


def test_ray_correction_is_galerkin():
    """After a correction the residual is orthogonal to the ray space (P^H
    (f - L u) = 0), so a second correction changes nothing; and the
    corrected preconditioner is B_V + C_R (I - L B_V) with C_R = P (P^H L
    P)^{-1} P^H written with dense matrices."""
    n, ray_n = 31, 3
    h = 1.0 / (n + 1)
    k = rng_k(n, 41, 8.0, 12.0)
    P = D.ray_basis(n, h, k, ray_n)
    g = oracle.Grid(h, k, variant=oracle.HLM, coarsest_n=3).set_ray(ray_n)
    f = rng_c((n + 2, n + 2), 7)
    u = g.ray_correct(f, rng_c((n + 2, n + 2), 8))
    r = (f - oracle.apply(h, k, 0.0, u)).reshape(-1)
    assert np.linalg.norm(P.conj().T @ r) <= 1e-10 * np.linalg.norm(P.conj().T @ f.reshape(-1))
    np.testing.assert_allclose(g.ray_correct(f, u), u, rtol=0, atol=1e-10 * np.abs(u).max())
    # the corrected preconditioner against its dense composition
    A = D.assemble_ghost(n, h, k, 0.0)
    CR = P @ np.linalg.solve(P.conj().T @ A @ P, P.conj().T)
    ref = D.DenseVCycle(h, k, g.plan())
    z_ref = ref.apply(f.reshape(-1))
    z_ref = z_ref + CR @ (f.reshape(-1) - A @ z_ref)
    z = g.precondition(f).reshape(-1)
    np.testing.assert_allclose(z, z_ref, rtol=0, atol=1e-10 * np.abs(z_ref).max())


def test_ray_correction_makes_hlm_v_a_solver():
    """Section 6.1 (trend only): HLM-V as a stationary solver diverges on
    the constant-k point-source problem at kh = 0.3125 (k = 20, h = 1/64,
    coarsest level at kH = 5), and with the ray correction it converges to a
    1e-7 reduction in few cycles (the paper's HLM-V column: 16 at k = 20;
    parity unpinned)."""
    n, h = 63, 1 / 64
    k = np.full((n + 2, n + 2), 20.0)
    f = np.zeros((n + 2, n + 2), complex)
    f[32, 32] = 1.0
    g = oracle.Grid(h, k, variant=oracle.HLM, coarsest_n=3)
    _, it0, hist0 = g.cycles(f, rtol=1e-7, maxit=60)
    assert it0 == 60 and hist0[-1] > 1.0
    g.set_ray(3)
    _, it, hist = g.cycles(f, rtol=1e-7, maxit=60)
    assert it <= 20 and hist[-1] <= 1e-7


# ---------------------------------------------------------------------------
# Fourier analysis vs the numbers printed in Sections 3 and 4
# ---------------------------------------------------------------------------

def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


def test_overall_rate_closed_form_matches_grid_search():
    for kappa in (0.3125, 0.625, 1.25, 5.0):
        for b in (0.0, BETA):
            assert lfa.overall_rate(kappa, b, npts=1601) == pytest.approx(
                lfa.overall_rate_closed(kappa, b), rel=2e-3)


def test_smoothing_numbers_printed_in_section_4():
    """Values printed in the Section 4 list that the formulas reproduce."""
    gold = load_golden("paper_section4_rates.json")
    for item in gold["checks"]:
        kappa, beta = item["kH"], (BETA if item["op"] == "M" else 0.0)
        if item["quantity"] == "mu_hat":
            val = lfa.overall_rate_closed(kappa, beta)
        else:
            val = lfa.smoothing_factor(kappa, beta)
        lo, hi = item["range"]
        assert lo <= val <= hi, (item, val)


def test_symbol_statements_section_3():
    """Section 3 list: at kH = 5, L^H approximates L^h well for |w| <= 0.65k
    (read as |w| H <= pi) along w1 = w2 while M^H has a large negative
    imaginary part; for
    kH <= 0.625 the high-frequency symbol ratios of L^H and M^H agree."""
    kh = 0.3125
    k = 40.0
    h = kh / k
    H = 16 * h          # kH = 5; visible on H: |w| H <= pi, i.e. |w| <= 0.628 k
    w = np.linspace(0.0, np.pi / 5, 200) * k / np.sqrt(2)
    tl = lfa.symbol_ratio(w, w, k, h, H)
    ts = lfa.symbol_ratio(w, w, k, h, H, beta=BETA)
    assert np.abs(tl - 1).max() < 0.2
    assert ts.imag.max() < -0.3
    H = 2 * h           # kH = 0.625
    wm = np.linspace(np.pi / 2, np.pi, 200) / H
    tl = lfa.symbol_ratio(wm, wm, k, h, H)
    ts = lfa.symbol_ratio(wm, wm, k, h, H, beta=BETA)
    assert np.abs(ts.real - tl.real).max() < 0.1
    assert np.abs(ts.imag).max() < 0.15


# ---------------------------------------------------------------------------
# Iteration counts of Tables 1-2: trend only (parity unpinned)
# ---------------------------------------------------------------------------

@pytest.mark.slow
def test_table2_trend_sl_counts_do_not_grow_as_h_shrinks():
    """Table 2 (k = 40, h = 1/64 ... 1/256): SL-V counts are flat or falling as
    h shrinks at fixed k.  Only the trend is checked (parity unpinned)."""
    its = []
    for n in (63, 127, 255):
        h = 1.0 / (n + 1)
        k = np.full((n + 2, n + 2), 40.0)
        f = np.zeros((n + 2, n + 2), complex)
        f[(n + 1) // 2, (n + 1) // 2] = 1
        _, info = oracle.Grid(h, k, variant=oracle.SL).bicgstab(f, rtol=1e-7, maxit=300)
        assert info["status"] == oracle.OK
        its.append(info["iters"])
    assert its[1] <= its[0] + 0.5 and its[2] <= its[1] + 0.5, its


@pytest.mark.slow
@pytest.mark.xfail(strict=False, reason=(
    "Table 1 reports HYB-V below SL-V; under the readings taken here (ghost-point "
    "boundary, mirrored full weighting, rediscretised coarse operators, exact LU of L "
    "on the coarsest level) Gauss-Seidel on L near kH = 2.5 amplifies the (pi, pi) "
    "error component and HYB-V needs more iterations than SL-V (parity unpinned)"))
def test_table1_trend_hybrid_not_worse_than_sl():
    """Table 1, k = 40, h = 1/64 (kh = 0.625): the paper reports HYB-V below
    SL-V (parity unpinned)."""
    n = 63
    h = 1 / 64
    k = np.full((n + 2, n + 2), 40.0)
    f = np.zeros((n + 2, n + 2), complex)
    f[32, 32] = 1
    its = {}
    for v in (oracle.SL, oracle.HYB):
        _, info = oracle.Grid(h, k, variant=v).bicgstab(f, rtol=1e-7, maxit=300)
        assert info["status"] == oracle.OK
        its[v] = info["iters"]
    assert its[oracle.HYB] <= its[oracle.SL] + 1.0, its


@pytest.mark.slow
def test_table1_trend_hybrid_below_sl_with_intermediate_scales_on_m():
    """Under the motivation's reading of the hybrid (hyb_mid: M for
    relaxation on the intermediate scales up to kH ~ 2.5), Table 1's
    ordering holds: HYB-V needs no more iterations than SL-V at k = 40, 80
    and 150 (kh = 0.625, coarsest level at kH = 5), and the gap widens with
    k as in the paper (trend only; parity unpinned)."""
    its = {}
    for n, k0, nc in ((63, 40.0, 7), (127, 80.0, 15), (239, 150.0, 29)):
        h = 1.0 / (n + 1)
        k = np.full((n + 2, n + 2), k0)
        f = np.zeros((n + 2, n + 2), complex)
        f[(n + 1) // 2, (n + 1) // 2] = 1
        row = []
        for v, mid in ((oracle.SL, 0), (oracle.HYB, 1)):
            _, info = oracle.Grid(h, k, variant=v, coarsest_n=nc, hyb_mid=mid).bicgstab(f, rtol=1e-7, maxit=300)
            assert info["status"] == oracle.OK
            row.append(info["iters"])
        its[k0] = row
    assert all(hyb <= sl for sl, hyb in its.values()), its
    gaps = [sl - hyb for sl, hyb in its.values()]
    assert gaps[-1] > gaps[0], its


# ---------------------------------------------------------------------------
# study switches (readings other than the default, for the iteration-count
# study of Section 5's choices): each equals its dense composition
# ---------------------------------------------------------------------------

class _DenseCoarseSweeps(D.DenseVCycle):
    """The dense V-cycle with the coarsest dense solve replaced by `sweeps`
    red-black Gauss-Seidel sweeps from zero on the coarsest operator."""

    def __init__(self, h, k, plan, sweeps):
        super().__init__(h, k, plan)
        self.sweeps = sweeps

    def apply(self, f, l=0):
        lev = self.levels[l]
        if lev["smoother"] == "LU":
            u = np.zeros_like(f)
            for _ in range(self.sweeps):
                u = D.sweep_gs_colour(lev["A_relax"], f, u, D.colour_rb(lev["n"]), 2)
            return u
        return super().apply(f, l)


def _compare_vcycle(g, ref, n):
    m = (n + 2) ** 2
    for col in range(0, m, 11):
        f = np.zeros(m, complex)
        f[col] = 1.0
        f[(col * 7 + 5) % m] = -0.25j
        want = ref.apply(f)
        got = g.vcycle(f.reshape(n + 2, n + 2)).reshape(-1)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("variant", [oracle.SL, oracle.HYB])
def test_study_restriction_is_the_transpose_of_interpolation(variant):
    """fw_transpose: the V-cycle with R = P^T / 4 on every level (the boundary
    weights dropped, not mirrored) equals that dense composition."""
    n, h = 15, 1 / 16
    k = rng_k(n, 61, 4.0, 30.0)
    g = oracle.Grid(h, k, variant=variant).set_study(fw_transpose=True)
    ref = D.DenseVCycle(h, k, g.plan())
    for lev in ref.levels[:-1]:
        lev["R"] = lev["P"].T / 4.0
    _compare_vcycle(g, ref, n)
    # and it differs from full weighting with mirror folding at the boundary
    rng = np.random.default_rng(3)
    f = rng.standard_normal((n + 2, n + 2)) + 1j * rng.standard_normal((n + 2, n + 2))
    base = oracle.Grid(h, k, variant=variant).vcycle(f)
    assert np.linalg.norm(g.vcycle(f) - base) > 1e-6 * np.linalg.norm(base)


@pytest.mark.parametrize("sweeps", [1, 3])
def test_study_coarsest_sweeps_replace_the_dense_solve(sweeps):
    n, h = 15, 1 / 16
    k = rng_k(n, 62, 4.0, 30.0)
    g = oracle.Grid(h, k, variant=oracle.HYB).set_study(coarse_sweeps=sweeps)
    _compare_vcycle(g, _DenseCoarseSweeps(h, k, g.plan(), sweeps), n)


def test_study_boundary_row_scale():
    """Rows with b boundary faces scaled by 2^-b: the operator equals D A with
    A the independent ghost-point matrix, and the scaled operator is complex
    symmetric (the doubled inward weights are halved); the V-cycle with it
    equals the dense composition with D A for relaxation, residuals and the
    coarsest solve."""
    n, h = 7, 1 / 8
    k = rng_k(n, 63, 2.0, 20.0)
    M = n + 2
    jj, ii = np.meshgrid(np.arange(M), np.arange(M), indexing="ij")
    b = ((ii == 0).astype(int) + (ii == n + 1) + (jj == 0) + (jj == n + 1)).reshape(-1)
    Dm = np.diag(2.0 ** (-b))
    try:
        oracle.set_boundary_row_scale(True)
        for sigma in (0.0, 0.5):
            A = oracle.dense(h, k, sigma)
            want = Dm @ D.assemble_ghost(n, h, k, sigma)
            np.testing.assert_allclose(A, want, rtol=0, atol=1e-12 * np.abs(want).max())
            np.testing.assert_allclose(A, A.T, rtol=0, atol=1e-12 * np.abs(A).max())
        g = oracle.Grid(h, k, variant=oracle.HYB)
        ref = D.DenseVCycle(h, k, g.plan())
        for lev in ref.levels:
            nl = lev["n"]
            Ml = nl + 2
            jl, il = np.meshgrid(np.arange(Ml), np.arange(Ml), indexing="ij")
            bl = ((il == 0).astype(int) + (il == nl + 1) + (jl == 0) + (jl == nl + 1)).reshape(-1)
            Dl = np.diag(2.0 ** (-bl))
            lev["A_relax"] = Dl @ lev["A_relax"]
            lev["A_resid"] = Dl @ lev["A_resid"]
        _compare_vcycle(g, ref, n)
    finally:
        oracle.set_boundary_row_scale(False)
    # off again: the default rows
    np.testing.assert_allclose(oracle.dense(h, k, 0.0), D.assemble_ghost(n, h, k, 0.0),
                               rtol=0, atol=1e-12 * np.abs(D.assemble_ghost(n, h, k, 0.0)).max())
