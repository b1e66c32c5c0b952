"""Pins of the planner's density-of-states features (oracle/chebyshev.py)
against definitions outside the oracle: hand-computed Jackson factors, the
Jackson kernel's construction as an autocorrelation, numerical quadrature of
the damped Chebyshev density, spectra whose moments are known in closed
form, and the band statistics recomputed from the dense matrix."""
from __future__ import annotations

import math

import numpy as np
import pytest
import scipy.integrate
import scipy.stats

import synth
from oracle import band as oband
from oracle import chebyshev as och


def test_jackson_hand_values():
    # N = K + 1 moments, a = pi / (N + 1):
    # g_k = [(N - k + 1) cos(a k) + sin(a k) cot(a)] / (N + 1)
    # K = 2 (a = pi/4): 1, (3 cos a + cos a) / 4 = cos(pi/4), (0 + 1) / 4
    assert np.allclose(och.jackson(2), [1.0, math.sqrt(0.5), 0.25], rtol=0, atol=1e-15)
    # K = 3 (a = pi/5): g_1 = cos(pi/5); g_2 = 1/sqrt(5); g_3 = (5 - sqrt(5))/20
    ref = [1.0, math.cos(math.pi / 5), 1.0 / math.sqrt(5.0), (5.0 - math.sqrt(5.0)) / 20.0]
    assert np.allclose(och.jackson(3), ref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("K", [1, 2, 3, 7, 16, 40])
def test_jackson_is_sine_autocorrelation(K):
    # Jackson's kernel is |sum_nu a_nu e^{i nu x}|^2 normalised, with
    # a_nu = sin(pi (nu + 1) / (N + 1)), nu = 0..N-1: its Chebyshev
    # coefficients are the normalised autocorrelation of a
    N = K + 1
    a = np.sin(np.pi * (np.arange(N) + 1) / (N + 1))
    ac = np.array([np.dot(a[: N - k], a[k:]) for k in range(N)]) / np.dot(a, a)
    assert np.abs(och.jackson(K) - ac).max() < 1e-14
    # g_1 = cos(pi / (N + 1)) (the kernel's variance)
    assert abs(och.jackson(K)[1] - math.cos(math.pi / (N + 1))) < 1e-14


def _damped_density(mbar, x):
    K = len(mbar) - 1
    g = och.jackson(K)
    s = g[0] * mbar[0] + 2.0 * sum(g[k] * mbar[k] * math.cos(k * math.acos(x))
                                   for k in range(1, K + 1))
    return s  # the weight 1 / (pi sqrt(1 - x^2)) is left to the quadrature


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_kpm_cdf_against_quadrature(seed):
    # the CDF of the damped expansion rho(x) = [g_0 mu_0 + 2 sum g_k mu_k
    # T_k(x)] / (pi sqrt(1 - x^2)), integrated in x from -1 by adaptive
    # quadrature with the algebraic end-point weight (1 + x)^-1/2 (the
    # factor (1 - x)^-1/2 is smooth on [-1, t] for t < 1)
    rng = np.random.default_rng(seed)
    K = 16
    mbar = np.r_[1.0, rng.uniform(-0.5, 0.5, K) / (1 + np.arange(K))]
    for t in (-0.95, -0.4, 0.0, 0.3, 0.77, 0.99):
        val, _ = scipy.integrate.quad(lambda x: _damped_density(mbar, x) / math.sqrt(1.0 - x),
                                      -1.0, t, weight="alg", wvar=(-0.5, 0.0), epsabs=1e-13,
                                      epsrel=1e-13, limit=200)
        ref = val / math.pi
        got = och.kpm_cdf(mbar, np.array([t]))[0]
        assert abs(got - ref) < 1e-11, (t, got, ref)


def test_kpm_cdf_exact_on_chebyshev_node_spectrum():
    # eigenvalues at the Chebyshev nodes cos(pi (i + 1/2) / n): every moment
    # with 0 < k < 2n vanishes, so the damped expansion is the arcsine law
    # 1 - arccos(t)/pi, which the empirical CDF approaches within 1/n
    n = 4000
    d = np.cos(np.pi * (np.arange(n) + 0.5) / n)
    mu = np.array([np.mean(np.cos(k * np.arccos(d))) for k in range(17)])
    assert np.abs(mu[1:]).max() < 1e-12 and abs(mu[0] - 1.0) < 1e-15
    t = np.linspace(-0.99, 0.99, 25)
    got = och.kpm_cdf(mu, t)
    assert np.abs(got - (1.0 - np.arccos(t) / np.pi)).max() < 1e-12
    emp = np.array([(d < s).mean() for s in t])
    assert np.abs(got - emp).max() <= 1.0 / n + 1e-12


def test_kpm_cdf_converges_to_exact_cdf():
    # a diagonal B: the Rademacher estimate is exact per probe; with many
    # moments the damped CDF approaches the exact eigenvalue CDF (Jackson
    # broadening ~ pi / K in the angle) at points away from the eigenvalues
    n = 3000
    rng = np.random.default_rng(3)
    d = np.sort(np.r_[rng.uniform(-6, -1, n // 2), rng.normal(3, 0.7, n - n // 2)])
    ab = np.zeros((1, n))
    ab[0] = d
    K = 400
    mu = och.cheb_moments(ab, K=K, P=2, seed=1)
    assert np.allclose(mu[0], mu[1], atol=1e-13)   # every probe exact
    c, h = och.scaling(ab)
    t = np.array([-5.0, -3.0, -1.5, 0.5, 2.0, 3.0, 4.0, 5.5])
    got = och.kpm_cdf(mu[0], (t - c) / h)
    exact = np.array([(d < s).mean() for s in t])
    assert np.abs(got - exact).max() < 0.01
    # with 16 moments the same estimate is coarse but still ordered
    mu16 = och.cheb_moments(ab, K=16, P=1, seed=1)[0]
    g16 = och.kpm_cdf(mu16, (t - c) / h)
    assert np.all(np.diff(g16) > 0)


@pytest.mark.parametrize("cplx,seed", [(False, 5), (True, 6)])
def test_band_statistics_against_dense(cplx, seed):
    n, b = 700, 9
    ab = synth.band_matrix(n, b, seed, cplx, -20, 20)
    A = oband.dense_from_band(ab)
    f = och.planner_features(ab, seed=0)
    st = f[66:80]
    nrm = np.linalg.norm(A, 1)
    d = np.real(np.diag(A))
    radii = np.sum(np.abs(A), axis=1) - np.abs(np.diag(A))
    glo, ghi = np.min(d - radii), np.max(d + radii)
    fro2 = np.linalg.norm(A, "fro") ** 2
    ref = [math.log2(n) / 16.0, b / 128.0, 1.0 if cplx else 0.0,
           d.mean() / nrm, d.std() / nrm, d.min() / nrm, d.max() / nrm,
           scipy.stats.skew(d), scipy.stats.kurtosis(d, fisher=True) / 10.0,
           (fro2 - np.sum(d * d)) / n / nrm ** 2, math.log10(nrm), (ghi - glo) / nrm,
           fro2 / n / nrm ** 2, (d.max() - d.min()) / (ghi - glo)]
    assert np.allclose(st, ref, rtol=1e-12, atol=1e-14), np.abs(st - np.array(ref))
    # the two leading features: Gershgorin bounds over ||B||_1, from the rows
    assert np.allclose(f[:2], [glo / nrm, ghi / nrm], rtol=1e-13, atol=0)
    # the mean moments: averages over the 20 probes of the dense recurrence
    P = och.rademacher(n, 20, 0)
    c, h = 0.5 * (glo + ghi), 1.01 * 0.5 * (ghi - glo)
    Ah = (A - c * np.eye(n)) / h
    T0, T1 = P.astype(complex), Ah @ P
    mus = [np.real(np.sum(P * T1, axis=0)) / n]
    for _ in range(2, 17):
        T0, T1 = T1, 2 * Ah @ T1 - T0
        mus.append(np.real(np.sum(P * T1, axis=0)) / n)
    mus = np.array(mus)
    assert np.allclose(f[2:18], mus.mean(axis=1), atol=1e-12)
    assert np.allclose(f[18:34], mus.std(axis=1), atol=1e-12)
