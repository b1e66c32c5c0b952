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
                                                  (12, "trapezoid", 0.3, 1.5)])
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
