"""Closed forms of the paper's Fourier analysis (Livshits, arXiv:1312.2880).

TEST INFRASTRUCTURE ONLY (pins for the oracle).

Section 3, eq. symb:helmholtz and symb:shifted: the symbol ratios of the
finest-grid Helmholtz operator to the coarse Helmholtz / shifted operator for
a Fourier component exp(i(w1 x + w2 y)).  Section 4, eq. conv:helmholtz and
conv:shifted: the amplitude change of one lexicographic Gauss-Seidel sweep,
and the smoothing factor (max over the high frequencies) and the overall rate
(max over all frequencies) defined right after them.

All functions take the dimensionless kH (``kappa``) or k, h, H and angles
theta = omega * H.
"""
from __future__ import annotations

import numpy as np

BETA = 0.5


def symbol_ratio(w1, w2, k, h, H, beta=None):
    """tau_H(w1, w2) = L~^h / A~^H, with A = L (beta None or 0) or M.

    Numerator and denominator are the plane-wave symbols of the 5-point
    operators, (2cos(w1 h) + 2cos(w2 h) - 4 + k^2 h^2 (1 + i beta)) / h^2."""
    b = 0.0 if beta is None else beta
    num = (2 * np.cos(w1 * h) + 2 * np.cos(w2 * h) - 4 + (k * h) ** 2) * H ** 2
    den = (2 * np.cos(w1 * H) + 2 * np.cos(w2 * H) - 4
           + (k * H) ** 2 * (1 + 1j * b)) * h ** 2
    return num / den


def gs_lex_amplification(t1, t2, kappa, beta=0.0):
    """mu_H(theta1, theta2) of eq. conv:helmholtz (beta = 0) / conv:shifted."""
    num = np.exp(-1j * t1) + np.exp(-1j * t2)
    den = np.exp(1j * t1) + np.exp(1j * t2) - 4 + kappa ** 2 * (1 + 1j * beta)
    return np.abs(num / den)


def _square(npts):
    t = np.linspace(-np.pi, np.pi, npts)
    return np.meshgrid(t, t, indexing="ij")


def smoothing_factor(kappa, beta=0.0, npts=1201):
    """mu~_H: max of mu over pi/2 <= max(|t1|, |t2|) <= pi."""
    t1, t2 = _square(npts)
    mu = gs_lex_amplification(t1, t2, kappa, beta)
    high = np.maximum(np.abs(t1), np.abs(t2)) >= np.pi / 2
    return float(mu[high].max())


def overall_rate(kappa, beta=0.0, npts=1201):
    """mu^_H: max of mu over the whole square [-pi, pi]^2 (grid search)."""
    t1, t2 = _square(npts)
    return float(gs_lex_amplification(t1, t2, kappa, beta).max())


def overall_rate_closed(kappa, beta=0.0):
    """Exact max over the square of mu.  With z_m = exp(i t_m) on the unit
    circle the numerator is |z1 + z2| = |conj(z1) + conj(z2)| = |s| and the
    denominator is |s - c| with c = 4 - kappa^2 (1 + i beta), s = z1 + z2
    ranging over the disc |s| <= 2.  The ratio |s| / |s - c| is maximal on
    |s| = 2 at s = 2 c / |c|, giving 2 / (|c| - 2) when |c| > 2, else
    unbounded (the denominator vanishes inside the disc)."""
    c = abs(4 - kappa ** 2 * (1 + 1j * beta))
    return 2.0 / (c - 2.0) if c > 2.0 else np.inf


def diagonal_rates(kappa, beta=0.0, npts=4001):
    """mu along w1 = w2 for |w| H <= pi; returns (|w|H / kappa, mu)."""
    t = np.linspace(0, np.pi / np.sqrt(2), npts)
    mu = gs_lex_amplification(t, t, kappa, beta)
    return np.sqrt(2) * t / kappa, mu


def rb_plane_wave_factors(t1, t2, kappa, beta=0.0):
    """One red-black Gauss-Seidel sweep on the constant-coefficient interior
    stencil applied to the error exp(i(t1 i + t2 j)) on both colours.  With
    d = -4 + kappa^2 (1 + i beta) and s = 2 cos t1 + 2 cos t2, the red update
    (neighbours all black, unchanged) multiplies the error by -s/d and the
    black update (neighbours all red, already updated) by (s/d)^2.  Both
    factors are exact at nodes at least two steps from the boundary.  Returns
    (red factor, black factor)."""
    d = -4 + kappa ** 2 * (1 + 1j * beta)
    s = 2 * np.cos(t1) + 2 * np.cos(t2)
    return -s / d, (s / d) ** 2


def rb_spectral_radius(kappa, beta=0.0):
    """max over theta of |s/d|^2, attained at s = +-4: (4 / |d|)^2."""
    d = abs(-4 + kappa ** 2 * (1 + 1j * beta))
    return (4.0 / d) ** 2
