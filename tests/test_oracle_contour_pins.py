"""Pins of the oracle's contour variants (Section 2.2: the contour and the
quadrature rule of the projector's integral are choices): the midpoint rule
on the circle has the closed form r(x) = 1 / (1 + t^(2k)), t = (x - c)/r; on
an ellipse both rules converge to Cauchy's value, the indicator of the
inside; ratio 1 is the circle."""
import numpy as np
import pytest

from oracle import quadrature as q


@pytest.mark.parametrize("k", [4, 8, 16])
def test_midpoint_rule_on_circle_closed_form(k):
    c, r = 0.3, 2.0
    z, w = q.contour(c - r, c + r, k, "trapezoid")
    t = np.array([0.0, 0.25, 0.5, 0.9, 0.99, 1.01, 1.5, 2.0, -0.7, -3.0])
    f = q.filter_value(c + t * r, z, w)
    np.testing.assert_allclose(f, 1.0 / (1.0 + t ** (2 * k)), rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("rule,k,tol", [("trapezoid", 64, 1e-12), ("gauss", 64, 1e-9)])
@pytest.mark.parametrize("rho", [0.5, 2.0])
def test_ellipse_converges_to_indicator(rule, k, tol, rho):
    c, r = -1.0, 3.0
    z, w = q.contour(c - r, c + r, k, rule, rho)
    assert np.all(z.imag > 0)
    inside = c + r * np.array([0.0, 0.4, -0.5])
    outside = c + r * np.array([1.8, -2.5, 4.0])
    assert np.abs(q.filter_value(inside, z, w) - 1.0).max() <= tol
    assert np.abs(q.filter_value(outside, z, w)).max() <= tol


@pytest.mark.parametrize("rule", ["gauss", "trapezoid"])
def test_ratio_one_is_circle_and_symmetric(rule):
    z1, w1 = q.contour(-2.0, 5.0, 8, rule, 1.0)
    z0, w0 = q.contour(-2.0, 5.0, 8, rule, 0.0)
    assert np.array_equal(z1, z0) and np.array_equal(w1, w0)
    if rule == "gauss":
        zc, wc = q.contour(-2.0, 5.0, 8)
        assert np.array_equal(z1, zc) and np.array_equal(w1, wc)
    # the filter of an ellipse is even about the centre
    z, w = q.contour(-2.0, 5.0, 8, rule, 0.4)
    t = np.array([0.3, 1.7, 3.2, 6.0])
    np.testing.assert_allclose(q.filter_value(1.5 + t, z, w), q.filter_value(1.5 - t, z, w),
                               rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("nodes,rule,ratio,m0f", [(16, "gauss", 1.0, 1.5), (8, "gauss", 1.0, 3.0),
                                                  (12, "trapezoid", 0.3, 1.5),
                                                  (8, "zolotarev", 0.9, 1.5)])
def test_sharp_filters_converge(nodes, rule, ratio, m0f):
    """Filters that damp many directions of the block below 1e-7 (16 nodes,
    m0 = 3m, a flat ellipse): FEAST reaches 1e-10 (the rank decision of the
    orthonormalisation is taken on the well-scaled second pass; truncating in
    the first pass held these cases near 1e-8)."""
    import math
    import synth
    from oracle import band as oband
    from oracle import feast as ofeast
    n = 300
    ab = synth.band_matrix(n, 6, 12, True, -8, 8)
    lam = np.linalg.eigvalsh(oband.dense_from_band(ab))
    lo, hi = -1.3, 2.1
    m = int(((lam >= lo) & (lam < hi)).sum())
    Y = synth.rhs_block(n, max(math.ceil(m0f * m), m + 10), 13, True)
    r = ofeast.feast_slice(ab, lo, hi, Y, n_nodes=nodes, rule=rule, ratio=ratio, max_iter=8)
    assert r.info == 0 and len(r.lam) == m and r.iters <= 4
    assert np.abs(r.lam - lam[(lam >= lo) & (lam < hi)]).max() <= 1e-12 * oband.norm1(ab)


@pytest.mark.parametrize("k", [0.3, 0.9, 0.99999])
def test_elliptic_functions_against_library(k):
    from scipy.special import ellipj, ellipk
    assert abs(q.elliptic_k(k) - ellipk(k * k)) <= 1e-14 * ellipk(k * k)
    for u in (0.05, 0.6, 1.4, 0.99 * ellipk(k * k)):
        sn, cn, dn = q.jacobi_sn_cn_dn(u, k)
        ref = ellipj(u, k * k)[:3]
        # near k = 1 and u = K the small cn is conditioned like eps K / cn
        np.testing.assert_allclose([sn, cn, dn], ref, rtol=1e-11, atol=1e-14)


@pytest.mark.parametrize("m,ell", [(1, 0.3), (3, 0.05), (6, 1e-2), (8, 1e-3), (16, 1e-3)])
def test_zolotarev_equioscillates(m, ell):
    """Z - 1 reaches +-delta with alternating signs at the 2m + 1 points
    x_j = ell / dn(j K'/(2m); k') of [ell, 1] and stays within delta between
    them: the alternation property of the best approximation."""
    c, M, delta, Kp = q.zolotarev_sign(m, ell)
    kp = np.sqrt(1 - ell * ell)

    def Z(x):
        num, den = M * x, 1.0
        for j in range(1, m):
            num = num * (x * x + c[2 * j - 1])
        for j in range(1, m + 1):
            den = den * (x * x + c[2 * j - 2])
        return num / den
    # dn(K'; k') = ell gives x = 1 at j = 2m (cos phi_0 / cos(phi_1 - phi_0) is 0/0 there)
    xs = np.array([ell / q.jacobi_sn_cn_dn(j * Kp / (2 * m), kp, ell)[2]
                   for j in range(2 * m)] + [1.0])
    assert abs(xs[0] - ell) < 1e-15 and np.all(np.diff(xs) > 0)
    e = Z(xs) - 1.0
    np.testing.assert_allclose(np.abs(e), delta, rtol=1e-9, atol=1e-12)
    assert np.all(np.sign(e[:-1]) == -np.sign(e[1:]))
    grid = np.geomspace(ell, 1.0, 200001)
    # allowance: rounding of Z near 1 (a product of 4m - 1 factors) and of its coefficients
    assert np.abs(Z(grid) - 1.0).max() <= delta * (1 + 1e-9) + 1e-12
    assert 0 < delta < 1


@pytest.mark.parametrize("m,b", [(4, 0.9), (8, 0.95), (6, 0.8)])
def test_zolotarev_filter_shape(m, b):
    """The FEAST form of the Zolotarev filter: poles on the circle through
    the slice ends, the node sum plus the dropped constant equal to
    (1 + Z(x(t))) / 2, within delta of 1 on |t| <= b and of 0 on |t| >= 1/b."""
    lo, hi = -1.0, 3.0
    cc, rr = 1.0, 2.0
    z, w = q.contour(lo, hi, m, "zolotarev", b)
    t, wt, finf, (ell, M, c, delta) = q.zolotarev_filter(m, b)
    assert np.all(z.imag > 0) and np.abs(np.abs(z - cc) - rr).max() < 1e-14
    tt = np.linspace(-4, 4, 4001)
    tt = tt[np.abs(np.abs(tt) - 1) > 1e-6]
    f = q.filter_value(cc + rr * tt, z, w)
    s = np.sqrt(ell)
    x = s * (1 + tt) / (1 - tt)
    num, den = M * x, 1.0
    for j in range(1, m):
        num = num * (x * x + c[2 * j - 1])
    for j in range(1, m + 1):
        den = den * (x * x + c[2 * j - 2])
    np.testing.assert_allclose(f + finf, 0.5 * (1 + num / den), rtol=0, atol=1e-13)
    assert np.abs(f[np.abs(tt) <= b] - 1).max() <= delta * (1 + 1e-9)
    assert np.abs(f[np.abs(tt) >= 1 / b]).max() <= delta * (1 + 1e-9)
    assert abs(finf) <= 0.5 * delta * (1 + 1e-9)
    with pytest.raises(ValueError):
        q.contour(lo, hi, m, "zolotarev", 1.0)
