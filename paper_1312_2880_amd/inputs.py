"""Seeded synthetic inputs (wavenumber fields, sources, request streams).

This module holds no arithmetic of the solver itself: it only draws the
problems that the GPU library and the CPU oracle are both run on.  Grids use
the convention of the library: ``n`` interior nodes per side, ``h = 1/(n+1)``,
arrays of shape ``(n+2, n+2)`` indexed ``[j, i]`` with node (i, j) at
(i h, j h) on the unit square.

Workloads (the paper's own media are not available, so these stand in):
  * constant k with a unit point source at the centre (the setting of the
    paper's Tables 1 and 2);
  * a layered medium (the benchmark medium): 8 horizontal layers with seeded
    interfaces and speeds c in [1.5, 4.5], times (1 + 0.05 g / max|g|) for a
    sum g of 64 seeded Gaussian bumps of width 0.05; k = omega / c;
  * a wedge-type medium (Table 3 analogue, own geometry: the paper's picture
    of its medium is missing): three regions of constant k = k_ref,
    1.5 k_ref and 2 k_ref separated by two slanted interfaces that meet
    inside the domain, unit source at the middle of the upper edge;
  * batches of constant-k instances of mixed sizes with several point sources;
  * Poisson request streams of layered-medium solves of mixed sizes.
"""
from __future__ import annotations

import math

import numpy as np

LAYERS = 8
BUMPS = 64
BUMP_WIDTH = 0.05
PERTURB = 0.05
C_RANGE = (1.5, 4.5)
LATTICE_N = 1023          # g is normalised by its max on this fixed lattice


def grid_h(n: int) -> float:
    return 1.0 / (n + 1)


def node_coords(n: int) -> np.ndarray:
    return np.arange(n + 2, dtype=np.float64) / (n + 1)


# ---- constant wavenumber --------------------------------------------------

def constant_k(n: int, k: float) -> np.ndarray:
    return np.full((n + 2, n + 2), float(k), np.float64)


def point_source(n: int, i: int, j: int, value: complex = 1.0) -> np.ndarray:
    f = np.zeros((n + 2, n + 2), np.complex128)
    f[j, i] = value
    return f


def centre_source(n: int) -> np.ndarray:
    c = (n + 1) // 2
    return point_source(n, c, c)


# ---- layered medium -------------------------------------------------------

class LayeredMedium:
    """Continuous speed field c(x, y) on [0,1]^2 drawn from ``seed``; it can
    be sampled on any grid, so one medium serves every resolution."""

    def __init__(self, seed: int):
        rng = np.random.default_rng(seed)
        self.interfaces = np.sort(rng.uniform(0.0, 1.0, LAYERS - 1))
        self.speeds = rng.uniform(C_RANGE[0], C_RANGE[1], LAYERS)
        self.amp = rng.uniform(-1.0, 1.0, BUMPS)
        self.centres = rng.uniform(0.0, 1.0, (BUMPS, 2))
        self.source_xy = rng.uniform(0.05, 0.95, 2)
        xs = node_coords(LATTICE_N)
        self.gmax = float(np.abs(self._bumps(xs)).max())

    def _bumps(self, xs: np.ndarray) -> np.ndarray:
        # separable Gaussians: g[j, i] = sum_m a_m gx_m(x_i) gy_m(y_j).  The
        # same bits on every host and thread count: the exponentials come
        # from the C library one value at a time (vectorised exponentials
        # differ between instruction sets) and the sum over m is accumulated
        # elementwise in a fixed order (a BLAS product rounds differently
        # with the number of threads).
        s2 = 2.0 * BUMP_WIDTH ** 2
        gx = np.array([[math.exp(-(x - c) ** 2 / s2) for x in xs] for c in self.centres[:, 0]])   # (m, nx)
        gy = np.array([[math.exp(-(y - c) ** 2 / s2) for y in xs] for c in self.centres[:, 1]])   # (m, ny)
        g = np.zeros((xs.size, xs.size))
        for m in range(self.amp.size):
            g += np.multiply.outer(self.amp[m] * gy[m], gx[m])
        return g

    def speed(self, n: int) -> np.ndarray:
        xs = node_coords(n)
        layer = np.searchsorted(self.interfaces, xs, side="right")
        cl = self.speeds[layer]                      # depends on y only
        g = self._bumps(xs)
        return cl[:, None] * (1.0 + PERTURB * g / self.gmax)

    def k(self, n: int, omega: float) -> np.ndarray:
        return omega / self.speed(n)

    def source(self, n: int) -> np.ndarray:
        i = int(round(self.source_xy[0] * (n + 1)))
        j = int(round(self.source_xy[1] * (n + 1)))
        i = min(max(i, 1), n)
        j = min(max(j, 1), n)
        return point_source(n, i, j)


def layered_problem(n: int, seed: int, omega: float):
    med = LayeredMedium(seed)
    return grid_h(n), med.k(n, omega), med.source(n)


# ---- wedge-type medium ----------------------------------------------------

WEDGE_UPPER = (0.75, -0.25)   # interface y = a + b x between the upper and the middle region
WEDGE_LOWER = (0.20, 0.35)    # interface between the middle (wedge) and the lower region
WEDGE_K = (1.0, 1.5, 2.0)     # k / k_ref in the upper, middle and lower region


def wedge_k(n: int, k_ref: float) -> np.ndarray:
    """k on the (n+2)^2 nodes: lower region y <= 0.20 + 0.35 x (2 k_ref),
    middle region up to y = 0.75 - 0.25 x (1.5 k_ref; it narrows to nothing
    at x = 11/12), upper region above both (k_ref)."""
    xs = node_coords(n)
    x, y = xs[None, :], xs[:, None]
    lower = y <= WEDGE_LOWER[0] + WEDGE_LOWER[1] * x
    middle = ~lower & (y <= WEDGE_UPPER[0] + WEDGE_UPPER[1] * x)
    k = np.full((n + 2, n + 2), WEDGE_K[0] * k_ref)
    k[middle] = WEDGE_K[1] * k_ref
    k[lower] = WEDGE_K[2] * k_ref
    return k


def wedge_problem(n: int):
    """Table 3 setting: k_ref h = 15/64 (k_ref = 15 on h = 1/64 up to 240 on
    h = 1/1024), unit source at the node nearest (0.5, 1)."""
    k_ref = 15.0 * (n + 1) / 64.0
    return grid_h(n), wedge_k(n, k_ref), point_source(n, (n + 1) // 2, n + 1)


# ---- named workloads ------------------------------------------------------

def workload_const_point(n: int = 63, k: float = 10 * math.pi):
    """Constant k, unit source at the centre node (default: 63^2, k = 10 pi)."""
    return grid_h(n), constant_k(n, k), centre_source(n)


def workload_layered_1023(seed: int = 2):
    """1023^2 layered medium, omega = 2 pi 40."""
    return layered_problem(1023, seed, 2 * math.pi * 40)


def workload_layered_2047(seed: int = 2):
    """The same medium on 2047^2 with omega = 2 pi 80 (same max kh)."""
    return layered_problem(2047, seed, 2 * math.pi * 80)


def batch_instances(seed: int = 4, count: int = 64, nrhs: int = 4,
                    sizes=(127, 255, 511, 1023), kh_range=(0.3, 0.6)):
    """Independent constant-k instances of mixed size, each with ``nrhs``
    point sources at distinct interior nodes."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.choice(sizes))
        kh = float(rng.uniform(*kh_range))
        k = kh * (n + 1)
        flat = rng.choice(n * n, size=nrhs, replace=False)
        rhs = []
        for q in flat:
            j, i = divmod(int(q), n)
            rhs.append(point_source(n, i + 1, j + 1))
        out.append(dict(n=n, h=grid_h(n), kh=kh, k=constant_k(n, k), f=rhs))
    return out


def request_stream(seed: int = 5, rate: float = 20.0, count: int = 300,
                   sizes=(255, 511, 1023, 2047)):
    """Poisson arrivals (exponential gaps, mean 1/rate) of layered-medium
    solves; omega = 2 pi 40 (n+1)/1024 keeps max kh fixed across sizes."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for q in range(count):
        t += float(rng.exponential(1.0 / rate))
        n = int(rng.choice(sizes))
        med_seed = int(rng.integers(0, 2 ** 31 - 1))
        out.append(dict(t_arrive=t, n=n, seed=med_seed,
                        omega=2 * math.pi * 40 * (n + 1) / 1024))
    return out


def random_field(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n + 2, n + 2)) + 1j * rng.standard_normal((n + 2, n + 2))
    return (scale * z).astype(np.complex128)


def random_k(n: int, seed: int, lo: float, hi: float) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, (n + 2, n + 2))
