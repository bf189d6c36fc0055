"""Independent dense-matrix constructions used to pin the oracle.

Everything here is written from the definitions in the paper (and the
readings the oracle takes), with numpy matrices instead of the oracle's
loops, so that a slip in the oracle's indexing, signs or ordering shows up as
a mismatch.  Test infrastructure only.
"""
from __future__ import annotations

import numpy as np


def node_index(n):
    M = n + 2
    return lambda i, j: j * M + i


def assemble_ghost(n, h, k, sigma):
    """A_sigma built as (plain 5-point Laplacian on a grid extended by one
    ghost layer) o (ghost extension from the central-difference Sommerfeld
    condition) + k^2 (1 + i sigma).  Ghost rule: du/dn - i k u = 0 with the
    outward normal, e.g. at x = 0: u(-1) = u(1) + 2 i k(0) h u(0)."""
    M = n + 2
    N = n + 1
    m = M * M
    idx = node_index(n)
    # extension operator E: (M+2)^2 extended nodes from m unknowns
    Me = M + 2
    E = np.zeros((Me * Me, m), np.complex128)

    def eidx(i, j):
        return (j + 1) * Me + (i + 1)

    for j in range(M):
        for i in range(M):
            E[eidx(i, j), idx(i, j)] = 1.0
    for t in range(M):
        # x = 0 side: ghost (-1, t)
        E[eidx(-1, t), idx(1, t)] += 1.0
        E[eidx(-1, t), idx(0, t)] += 2j * k[t, 0] * h
        # x = 1 side: ghost (N+1, t)
        E[eidx(N + 1, t), idx(N - 1, t)] += 1.0
        E[eidx(N + 1, t), idx(N, t)] += 2j * k[t, N] * h
        # y = 0 side: ghost (t, -1)
        E[eidx(t, -1), idx(t, 1)] += 1.0
        E[eidx(t, -1), idx(t, 0)] += 2j * k[0, t] * h
        # y = 1 side: ghost (t, N+1)
        E[eidx(t, N + 1), idx(t, N - 1)] += 1.0
        E[eidx(t, N + 1), idx(t, N)] += 2j * k[N, t] * h
    lap = np.zeros((m, Me * Me))
    for j in range(M):
        for i in range(M):
            r = idx(i, j)
            lap[r, eidx(i, j)] = -4.0 / h ** 2
            for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                lap[r, eidx(i + di, j + dj)] = 1.0 / h ** 2
    A = lap @ E
    A += np.diag((k.reshape(-1) ** 2) * (1 + 1j * sigma))
    return A


def restriction_matrix(n):
    """Full weighting (1,2,1)x(1,2,1)/16 with mirrored fine values outside
    the grid, as a dense (Mc^2 x M^2) matrix."""
    M = n + 2
    N = n + 1
    Nc = N // 2
    Mc = Nc + 1
    R = np.zeros((Mc * Mc, M * M))
    for J in range(Mc):
        for I in range(Mc):
            for e in (-1, 0, 1):
                for d in (-1, 0, 1):
                    i, j = 2 * I + d, 2 * J + e
                    i = -i if i < 0 else (2 * N - i if i > N else i)
                    j = -j if j < 0 else (2 * N - j if j > N else j)
                    R[J * Mc + I, j * M + i] += (2 - abs(d)) * (2 - abs(e)) / 16.0
    return R


def prolongation_matrix(nc):
    """Bilinear interpolation, dense (M^2 x Mc^2), built from the tensor
    product of 1-D linear interpolation."""
    Mc = nc + 2
    M = 2 * (nc + 1) + 1
    p1 = np.zeros((M, Mc))
    for I in range(Mc):
        p1[2 * I, I] = 1.0
        if 2 * I + 1 < M:
            p1[2 * I + 1, I] += 0.5
        if 2 * I - 1 >= 0:
            p1[2 * I - 1, I] += 0.5
    return np.kron(p1, p1)   # row index j*M + i, column J*Mc + I


def colour_rb(n):
    M = n + 2
    jj, ii = np.meshgrid(np.arange(M), np.arange(M), indexing="ij")
    return ((ii + jj) % 2).reshape(-1)


def colour_5(n):
    M = n + 2
    jj, ii = np.meshgrid(np.arange(M), np.arange(M), indexing="ij")
    return ((ii + 2 * jj) % 5).reshape(-1)


def sweep_gs_lex(A, f, u):
    D_L = np.tril(A)
    U = A - D_L
    return np.linalg.solve(D_L, f - U @ u)


def sweep_gs_colour(A, f, u, colours, ncol):
    u = u.copy()
    for c in range(ncol):
        S = colours == c
        sub = A[np.ix_(S, S)]
        # rows of one colour are not coupled, so the block is diagonal
        assert np.count_nonzero(sub - np.diag(np.diag(sub))) == 0
        rhs = f[S] - A[S][:, ~S] @ u[~S]
        u[S] = rhs / np.diag(sub)
    return u


def sweep_kacz_lex(A, f, u):
    u = u.copy()
    for p in range(A.shape[0]):
        a = A[p]
        u = u + np.conj(a) * (f[p] - a @ u) / np.vdot(a, a).real
    return u


def sweep_kacz_colour(A, f, u, colours, ncol):
    u = u.copy()
    for c in range(ncol):
        S = colours == c
        Ac = A[S]
        d = np.einsum("ij,ij->i", Ac, np.conj(Ac)).real
        u = u + np.conj(Ac).T @ ((f[S] - Ac @ u) / d)
    return u


class DenseVCycle:
    """The V-cycle written with dense matrices, levels described by the
    oracle's plan (smoother, relaxation / residual shifts, sweep counts)."""

    def __init__(self, h, k, plan, gs_order="rb", kacz_order="5c", inject=None):
        self.levels = []
        kl = k
        H = h
        for l, p in enumerate(plan):
            n = p["n"]
            assert kl.shape == (n + 2, n + 2)
            lev = dict(p, k=kl, H=H,
                       A_relax=assemble_ghost(n, H, kl, p["sigma_relax"]),
                       A_resid=assemble_ghost(n, H, kl, p["sigma_resid"]))
            if l + 1 < len(plan):
                lev["R"] = restriction_matrix(n)
                lev["P"] = prolongation_matrix(plan[l + 1]["n"])
                kl = kl[::2, ::2].copy()
                H = 2 * H
            self.levels.append(lev)
        self.gs_order = gs_order
        self.kacz_order = kacz_order

    def _relax(self, lev, f, u, sweeps):
        A = lev["A_relax"]
        n = lev["n"]
        for _ in range(sweeps):
            if lev["smoother"] == "GS":
                if self.gs_order == "lex":
                    u = sweep_gs_lex(A, f, u)
                else:
                    u = sweep_gs_colour(A, f, u, colour_rb(n), 2)
            else:
                if self.kacz_order == "lex":
                    u = sweep_kacz_lex(A, f, u)
                else:
                    u = sweep_kacz_colour(A, f, u, colour_5(n), 5)
        return u

    def apply(self, f, l=0):
        lev = self.levels[l]
        if lev["smoother"] == "LU":
            return np.linalg.solve(lev["A_relax"], f)
        u = np.zeros_like(f)
        u = self._relax(lev, f, u, lev["pre"])
        r = f - lev["A_resid"] @ u
        e = self.apply(lev["R"] @ r, l + 1)
        u = u + lev["P"] @ e
        return self._relax(lev, f, u, lev["post"])


def round32(a):
    """Round a complex128 array to complex float (RNE per component) and
    widen it back."""
    return np.asarray(a, np.complex128).astype(np.complex64).astype(np.complex128)


class DenseMixedVCycle(DenseVCycle):
    """The precision form of the V-cycle written with dense matrices: fields
    are rounded to complex float where they are stored, arithmetic is double.

    mode "fused":  k on every level; each restricted right-hand side; each
                   coarse correction; on Kaczmarz levels the iterate after
                   every `every` sweeps (the pre-smoothing residual is formed
                   before that leg's last rounding); levels with n <= block_n
                   are evaluated in double as a whole.
    mode "onepass": every colour pass, restriction, prolongation-and-add and
                   coarsest result is rounded.
    round_io rounds the input and the output of the whole cycle.  The
    coarsest operator keeps the unrounded k.  fp64_levels = t ("fused"):
    levels finer than t (clamped to the first double-block or coarsest level)
    keep double fields and k, and level t takes its right-hand side and
    returns its correction unrounded."""

    def __init__(self, h, k, plan, mode, every=2, block_n=31, round_io=False, fp64_levels=0):
        super().__init__(h, k, plan)
        self.mode, self.every, self.block_n, self.round_io = mode, every, block_n, round_io
        t = fp64_levels if mode == "fused" else 0
        for l, p in enumerate(plan[:t]):
            if p["n"] <= block_n or p["smoother"] == "LU":
                t = l
                break
        self.t = t
        for l, lev in enumerate(self.levels):
            lev["level"] = l
            if l < t:
                continue
            k32 = lev["k"].astype(np.float32).astype(np.float64)
            if lev["smoother"] != "LU":
                lev["A_relax"] = assemble_ghost(lev["n"], lev["H"], k32, lev["sigma_relax"])
                lev["A_resid"] = assemble_ghost(lev["n"], lev["H"], k32, lev["sigma_resid"])
            lev["A_relax32"] = assemble_ghost(lev["n"], lev["H"], k32, lev["sigma_relax"])
            lev["A_resid32"] = assemble_ghost(lev["n"], lev["H"], k32, lev["sigma_resid"])

    def _double_block(self, f, l):
        """Levels l.. in double with the rounded k (coarsest: unrounded k)."""
        lev = self.levels[l]
        if lev["smoother"] == "LU":
            return np.linalg.solve(lev["A_relax"], f)
        u = self._relax(lev, f, np.zeros_like(f), lev["pre"])
        r = f - lev["A_resid"] @ u
        u = u + lev["P"] @ self._double_block(lev["R"] @ r, l + 1)
        return self._relax(lev, f, u, lev["post"])

    def _leg(self, lev, f, u, sweeps, last_store):
        A, n = lev["A_relax"], lev["n"]
        kacz = lev["smoother"] == "KACZ"
        if lev["level"] < self.t:
            return self._relax(lev, f, u, sweeps)
        colours, ncol = (colour_5(n), 5) if kacz else (colour_rb(n), 2)
        for it in range(sweeps):
            for c in range(ncol):
                S = colours == c
                if kacz:
                    Ac = A[S]
                    d = np.einsum("ij,ij->i", Ac, np.conj(Ac)).real
                    u = u + np.conj(Ac).T @ ((f[S] - Ac @ u) / d)
                else:
                    sub = np.diag(A[np.ix_(S, S)])
                    u = u.copy()
                    u[S] = (f[S] - A[S][:, ~S] @ u[~S]) / sub
                if self.mode == "onepass":
                    u = round32(u)
            if (self.mode == "fused" and kacz and (it + 1) % self.every == 0
                    and (it + 1 < sweeps or last_store)):
                u = round32(u)
        return u

    def _level(self, f, l):
        lev = self.levels[l]
        if lev["smoother"] == "LU":
            return np.linalg.solve(lev["A_relax"], f)
        if self.mode == "fused" and lev["n"] <= self.block_n:
            return self._double_block(f, l)
        kacz = lev["smoother"] == "KACZ"
        stores, cstores = l >= self.t, l + 1 > self.t
        keep = lambda a: a
        rc = round32 if cstores else keep
        u = self._leg(lev, f, np.zeros_like(f), lev["pre"], False)
        r = f - lev["A_resid"] @ u
        if stores and kacz and self.mode == "fused" and lev["pre"] > 0:
            u = round32(u)
        fc = rc(lev["R"] @ r)
        e = rc(self._level(fc, l + 1))
        u = u + lev["P"] @ e
        if self.mode == "onepass":
            u = round32(u)
        return self._leg(lev, f, u, lev["post"], True)

    def apply(self, f, l=0):
        rio = self.round_io and self.t == 0
        if rio:
            f = round32(f)
        u = self._level(np.asarray(f, np.complex128), 0)
        return round32(u) if rio else u


def ray_basis(n, h, k, ray_n):
    """The ray correction's basis (Section 6.1 ansatz) as a dense matrix,
    columns (d, a) for direction theta = (d + 1) pi / 4 and ray-grid node a:
    exp(i kr (cos theta x + sin theta y)) times the bilinear hat of a, kr the
    mean of k; built from the 1-D hats' tensor product."""
    M = n + 2
    Mr = ray_n + 2
    L = (n + 1) * h
    Hr = L / (ray_n + 1)
    x = np.arange(M) * h
    hat1 = np.maximum(0.0, 1.0 - np.abs(x[:, None] / Hr - np.arange(Mr)[None, :]))   # (M, Mr)
    kr = float(np.mean(k))
    cols = []
    for d in range(8):
        th = (d + 1) * np.pi / 4
        wave = np.exp(1j * kr * (np.cos(th) * x[None, :] + np.sin(th) * x[:, None]))   # [j, i]
        for a in range(Mr * Mr):
            ia, ja = a % Mr, a // Mr
            phi = np.outer(hat1[:, ja], hat1[:, ia])      # [j, i]
            cols.append((wave * phi).reshape(-1))
    return np.stack(cols, axis=1)
