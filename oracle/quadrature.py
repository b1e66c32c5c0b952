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

Zolotarev rule (the third filter Section 2.2 names): the best uniform
rational approximation Z of type (2m-1, 2m) to sign(x) on [-1, -l] U [l, 1],
Z(x) = M x prod_{j<m} (x^2 + c_{2j}) / prod_{j<=m} (x^2 + c_{2j-1}) with
c_j = l^2 sn^2(j K'/(2m); k') / cn^2(j K'/(2m); k'), k' = sqrt(1 - l^2),
K' = K(k') (Zolotarev's classical solution), composed with the Moebius map
x = sqrt(l) (1 + t) / (1 - t) of the scaled slice variable t = (lambda - c)/r,
which sends (-1, 1) to x > 0, the rest of the real line to x < 0 and the
poles x = +-i sqrt(c_{2j-1}) onto the unit circle.  f(t) = (1 + Z(x(t))) / 2
is then 1 within delta on |t| <= b and 0 within delta on |t| >= 1/b, with
b the inner fraction (``ratio``) and l = ((1 - b)/(1 + b))^2.  M makes the
error equioscillate: the extrema on [l, 1] sit at x = l / dn(j K'/(2m); k'),
minima at even j, maxima at odd j.  Readings: m = the number of nodes in the
upper half; the constant f(infinity), at most delta/2 in size, is dropped
so that the filter keeps the FEAST form sum_j 2 Re[w_j / (z_j - lambda)].

Pinned by: ``numpy.polynomial.legendre.leggauss``, sum(omega) = 2, exactness
on polynomials of degree <= 2k-1, and the closed forms r(c) = 1 and
r(c +- r) = 1/2 (tests); the midpoint rule on the circle by its closed form
r(x) = 1 / (1 + ((x - c)/r)^(2k)); the ellipse by Cauchy's formula (r -> the
indicator of the inside as k grows); the Zolotarev rule by equioscillation of
Z - 1 at 2m + 1 points of [l, 1] with the error bound holding on a dense grid
(the Chebyshev alternation property that makes Z the best approximation),
and the node-weight sum against (1 + Z(x(t))) / 2 - f(infinity).
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


def elliptic_k(k: float, kc: float | None = None) -> float:
    """Complete elliptic integral of the first kind K(k) (modulus k) by the
    arithmetic-geometric mean: K = pi / (2 AGM(1, k_c)), k_c = sqrt(1 - k^2)
    (pass k_c when it is known exactly: 1 - k^2 cancels for k near 1)."""
    a, b = 1.0, np.sqrt(1.0 - k * k) if kc is None else kc
    for _ in range(64):                # converges quadratically; rounding can
        if abs(a - b) <= 4e-16 * a:     # leave a and b an ulp apart for good
            break
        a, b = 0.5 * (a + b), np.sqrt(a * b)
    return np.pi / (2.0 * a)


def jacobi_sn_cn_dn(u: float, k: float, kc: float | None = None):
    """Jacobi elliptic functions sn, cn, dn of argument u and modulus k by the
    descending Landen (AGM) scheme: a_0 = 1, b_0 = sqrt(1 - k^2), c_0 = k;
    a_{i+1} = (a_i + b_i)/2, b_{i+1} = sqrt(a_i b_i), c_{i+1} = (a_i - b_i)/2;
    phi_N = 2^N a_N u, phi_{i-1} = (phi_i + asin(c_i sin(phi_i) / a_i)) / 2;
    sn = sin phi_0, cn = cos phi_0, dn = cos phi_0 / cos(phi_1 - phi_0)."""
    a, b, c = [1.0], [np.sqrt(1.0 - k * k) if kc is None else kc], [k]
    while abs(c[-1]) > 4e-16 * a[-1] and len(a) < 64:
        a.append(0.5 * (a[-1] + b[-1]))
        b.append(np.sqrt(a[-2] * b[-1]))
        c.append(0.5 * (a[-2] - b[-2]))
    N = len(a) - 1
    phi = [0.0] * (N + 1)
    phi[N] = 2.0 ** N * a[N] * u
    for i in range(N, 0, -1):
        phi[i - 1] = 0.5 * (phi[i] + np.arcsin(c[i] * np.sin(phi[i]) / a[i]))
    sn, cn = np.sin(phi[0]), np.cos(phi[0])
    dn = cn / np.cos(phi[1] - phi[0]) if N > 0 else 1.0
    return sn, cn, dn


def zolotarev_sign(m: int, ell: float):
    """Zolotarev's best approximation of type (2m-1, 2m) to sign(x) on
    [-1, -ell] U [ell, 1]: returns (c_1..c_{2m-1}, M, delta, K') with
    Z(x) = M x prod_{j<m}(x^2 + c_{2j}) / prod_{j<=m}(x^2 + c_{2j-1}) and
    max |Z - 1| on [ell, 1] = delta."""
    kp = np.sqrt(1.0 - ell * ell)
    Kp = elliptic_k(kp, ell)
    cj = np.zeros(2 * m)                      # cj[j] = c_j, j = 1..2m-1
    for j in range(1, 2 * m):
        sn, cn, _ = jacobi_sn_cn_dn(j * Kp / (2 * m), kp, ell)
        cj[j] = ell * ell * sn * sn / (cn * cn)
    def zt(x):
        num, den = x, 1.0
        for j in range(1, m):
            num = num * (x * x + cj[2 * j])
        for j in range(1, m + 1):
            den = den * (x * x + cj[2 * j - 1])
        return num / den
    _, _, dn1 = jacobi_sn_cn_dn(Kp / (2 * m), kp, ell)
    lo_v, hi_v = zt(ell), zt(ell / dn1)        # a minimum and a maximum
    M = 2.0 / (lo_v + hi_v)
    return cj[1:], M, (hi_v - lo_v) / (hi_v + lo_v), Kp


def zolotarev_filter(m: int, b: float):
    """The Zolotarev filter on the scaled slice (-1, 1) with inner fraction
    b: upper-half poles t_k, weights w_k (f = f_inf + sum_k 2 Re[w_k/(t_k - t)])
    and the dropped constant f_inf, together with (ell, M, c)."""
    ell = ((1.0 - b) / (1.0 + b)) ** 2
    s = np.sqrt(ell)
    c, M, delta, _ = zolotarev_sign(m, ell)
    cc = np.concatenate([[0.0], c])            # cc[j] = c_j
    t = np.zeros(m, complex)
    w = np.zeros(m, complex)
    for q in range(1, m + 1):
        a2 = cc[2 * q - 1]
        # Z = sum_q rho_q [1/(x - i a) + 1/(x + i a)], rho_q = residue at x = i a
        # (= the residue at -i a: Z is odd and real)
        num = M
        for j in range(1, m):
            num *= cc[2 * j] - a2
        den = 2.0
        for j in range(1, m + 1):
            if j != q:
                den *= cc[2 * j - 1] - a2
        rho = num / den
        p = 1j * np.sqrt(a2)
        tp = (p - s) / (p + s)                 # pole on the unit circle, Im > 0
        # 1/(x - p) = -1/(s + p) + (1 - tp) / ((s + p)(t - tp)); f = (1 + Z)/2
        t[q - 1] = tp
        w[q - 1] = -0.5 * rho * (1.0 - tp) / (s + p)
    zinf = M * (-s)
    for j in range(1, m):
        zinf *= s * s + cc[2 * j]
    for j in range(1, m + 1):
        zinf /= s * s + cc[2 * j - 1]
    return t, w, 0.5 * (1.0 + zinf), (ell, M, c, delta)


def contour(lo: float, hi: float, k: int = 8, rule: str = "gauss", ratio: float = 1.0):
    """Nodes z_j and weights w_j on the upper half of the contour through the
    slice ends [lo, hi): the circle (ratio 1) or an ellipse of vertical
    semi-axis ratio * r, with the Gauss-Legendre or the midpoint rule; or the
    Zolotarev rule with inner fraction ratio (0 < ratio < 1)."""
    c = 0.5 * (lo + hi)
    r = 0.5 * (hi - lo)
    if rule == "zolotarev":
        if not 0.0 < ratio < 1.0:
            raise ValueError("the Zolotarev rule needs 0 < ratio < 1")
        t, w, _, _ = zolotarev_filter(k, ratio)
        return c + r * t, r * w
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
