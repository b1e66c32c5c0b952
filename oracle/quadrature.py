"""Quadrature nodes/weights and the rational filter (test infrastructure).

The paper approximates the spectral projector, the contour integral of
(zI - A)^{-1} (Section 2.2, equation eq:integral), by a quadrature with n_e
nodes and weights, Gauss by default with eight nodes per interval, giving the
rational filter r(x) = sum_j w_j / (z_j - x).

Readings (the paper is silent or garbled here):
* the factor 1/(2 pi i) missing from eq:integral is restored;
* the contour is the circle through the slice ends, center c = (lo+hi)/2,
  radius r = (hi-lo)/2; Gauss-Legendre nodes are placed on the upper half only
  and the lower half is its mirror image, because for Hermitian B the
  integrand on the lower half is the conjugate transpose of the upper one.
  With theta = (pi/2)(1 - x) the nodes and weights are
  z_j = c + r e^{i theta_j}, w_j = (omega_j / 4) r e^{i theta_j}, and the filter
  becomes r(x) = sum_j 2 Re[w_j / (z_j - x)].

Filter variants (the other contours and rules Section 2.2 names): an ellipse
through the slice ends, z(t) = c + r (cos t + i rho sin t), and the trapezoid
(midpoint) rule with 2k equispaced angles t_j = pi (j + 1/2) / k on the whole
curve.  In general w_j = (dt_j / (2 pi)) z'(t_j) / i with dt_j the weight of the
rule in the angle, (pi/2) omega_j for Gauss-Legendre and pi / k for the
midpoint rule.

Pinned by: ``numpy.polynomial.legendre.leggauss``, sum(omega) = 2, exactness
on polynomials of degree <= 2k-1, and the closed forms r(c) = 1 and
r(c +- r) = 1/2 (tests); the midpoint rule on the circle by its closed form
r(x) = 1 / (1 + ((x - c)/r)^(2k)); the ellipse by Cauchy's formula (r -> the
indicator of the inside as k grows).
"""
from __future__ import annotations

import numpy as np

from .jacobi import jacobi_eigh


def gauss_legendre(k: int):
    """Nodes x_j (ascending) and weights omega_j on [-1, 1] by Golub-Welsch.

    The symmetric tridiagonal Jacobi matrix of the Legendre recurrence has
    off-diagonals beta_i = i / sqrt(4 i^2 - 1), i = 1..k-1; its eigenvalues are
    the nodes and the weights are 2 * (first eigenvector component)^2."""
    J = np.zeros((k, k))
    for i in range(1, k):
        beta = i / np.sqrt(4.0 * i * i - 1.0)
        J[i, i - 1] = J[i - 1, i] = beta
    x, V = jacobi_eigh(J, tol=1e-17, max_sweeps=60)
    w = 2.0 * V[0, :] ** 2
    return x, w


def contour(lo: float, hi: float, k: int = 8, rule: str = "gauss", ratio: float = 1.0):
    """Nodes z_j and weights w_j on the upper half of the contour through the
    slice ends [lo, hi): the circle (ratio 1) or an ellipse of vertical
    semi-axis ratio * r, with the Gauss-Legendre or the midpoint rule."""
    c = 0.5 * (lo + hi)
    r = 0.5 * (hi - lo)
    rho = ratio if ratio > 0 else 1.0
    if rule == "gauss":
        x, om = gauss_legendre(k)
        theta = 0.5 * np.pi * (1.0 - x)
        dt = 0.5 * np.pi * om
    elif rule == "trapezoid":
        theta = np.pi * (np.arange(k) + 0.5) / k
        dt = np.full(k, np.pi / k)
    else:
        raise ValueError(rule)
    z = c + r * (np.cos(theta) + 1j * rho * np.sin(theta))
    dz_over_i = r * (rho * np.cos(theta) + 1j * np.sin(theta))  # z'(t) / i
    return z, dt / (2.0 * np.pi) * dz_over_i


def filter_value(lam, z, w):
    """r(lambda) = sum_j 2 Re[w_j / (z_j - lambda)]: the scalar the filter
    applies to an eigenvector with eigenvalue lambda."""
    lam = np.asarray(lam, dtype=np.float64)
    return sum(2.0 * np.real(wj / (zj - lam)) for zj, wj in zip(z, w))
