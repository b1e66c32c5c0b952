"""Pins of the oracle's slice placement from previous eigenvalues (Section
3.1, Algorithm alg:kmeans; Section 3.2, Algorithm alg:lower_upper): worked
cluster examples, equal spacing fixed points, the paper's step parameters
(alpha = 1e-3, m1 = 6) on diagonal matrices whose inertia is a plain count,
and exact slice counts against dense eigenvalues."""
import numpy as np
import pytest

import synth
from oracle import band as oband
from oracle import planner as opl


def _diag(a):
    return np.asarray(a, dtype=np.float64).reshape(1, -1)


def test_kmeans_separates_worked_clusters():
    # 25 points in clusters of 3, 10, 5, 7: the initial groups (7, 6, 6, 6)
    # move in one sweep to the clusters (worked by hand)
    d = np.concatenate([0.0 + 1e-3 * np.arange(3), 10 + 1e-3 * np.arange(10),
                        20 + 1e-3 * np.arange(5), 30 + 1e-3 * np.arange(7)])
    s, v, c = opl.kmeans_1d(d, 4)
    assert c == [3, 10, 5, 7]
    assert s == [0, 3, 13, 18, 25]
    np.testing.assert_array_equal(v, [(0.002 + 10) / 2, (10.009 + 20) / 2, (20.004 + 30) / 2])


@pytest.mark.parametrize("n,K", [(24, 4), (25, 4), (7, 7), (100, 9)])
def test_kmeans_equal_spacing_is_a_fixed_point(n, K):
    d = np.arange(n, dtype=np.float64)
    s, v, c = opl.kmeans_1d(d, K)
    q, r = divmod(n, K)
    assert c == [q + 1 if i < r else q for i in range(K)]
    np.testing.assert_array_equal(v, [s[j] - 0.5 for j in range(1, K)])


def test_kmeans_degenerate_inputs():
    s, v, c = opl.kmeans_1d(np.zeros(10), 3)  # one cluster: groups merge
    assert c == [10] and v == []
    d = np.array([0.0, 1.0, 5.0])
    s, v, c = opl.kmeans_1d(d, 8)  # more groups than points
    assert c == [1, 1, 1]
    np.testing.assert_array_equal(v, [0.5, 3.0])


def test_kmeans_invariants_random():
    rng = np.random.default_rng(5)
    for _ in range(50):
        n = int(rng.integers(1, 300))
        K = int(rng.integers(1, 20))
        d = np.sort(rng.standard_normal(n) * rng.uniform(0.1, 10))
        s, v, c = opl.kmeans_1d(d, K)
        assert s[0] == 0 and s[-1] == n and all(b > a for a, b in zip(s, s[1:]))
        assert sum(c) == n and len(c) <= K and len(v) == len(c) - 1
        for j, x in enumerate(v, start=1):
            assert d[s[j] - 1] <= x <= d[s[j]]


def test_upper_bound_steps_paper_parameters():
    a = np.arange(10.0)
    ab = _diag(a)
    # d_nev = 1, delta = 1: step max(1e-3, 6) = 6, b = 7 and n_-(7) = 7 >= 5
    assert opl.upper_bound_search(ab, a - 3.0, 5) == 7.0
    # d_nev = -16: b = -10, -4, 2 (two eigenvalues below), 8 (eight)
    log = []
    assert opl.upper_bound_search(ab, a - 20.0, 5, log=log) == 8.0
    assert log == [-10.0, -4.0, 2.0, 8.0]
    # alpha term: d_nev = 1000.009, gaps 1e-3: step max(1e-3 d_nev, 6e-3)
    d = 1000.0 + 1e-3 * np.arange(10)
    assert opl.upper_bound_search(_diag(d), d, 10) == d[9] + 1e-3 * d[9]


def test_lower_bound_steps_paper_parameters():
    a = np.arange(10.0)
    ab = _diag(a)
    # d_1 = 20, d_2 - d_1 = 1: step 6, b = 14, 8, 2, -4 (nothing below)
    log = []
    assert opl.lower_bound_search(ab, a + 20.0, log=log) == -4.0
    assert log == [14.0, 8.0, 2.0, -4.0]


@pytest.mark.parametrize("cplx", [False, True])
def test_plan_prev_exact_counts_against_dense(cplx):
    n, b, nev, K = 240, 5, 90, 6
    ab = synth.band_matrix(n, b, 11, cplx, -10, 10)
    E = synth.hermitian_perturbation(n, b, 12, cplx)
    prev = np.linalg.eigvalsh(oband.dense_from_band(ab + 1e-2 * E))
    lam = np.linalg.eigvalsh(oband.dense_from_band(ab))
    bounds, counts, Kp, nshift = opl.plan_prev(ab, prev, nev, K)
    assert Kp == len(counts) <= K and nshift > 0
    assert bounds[0] < lam[0]
    assert np.sum(lam < bounds[-1]) >= nev
    for i in range(Kp):
        assert counts[i] == np.sum((lam >= bounds[i]) & (lam < bounds[i + 1]))
    assert counts.sum() == np.sum(lam < bounds[-1])
