"""Pins of the planner part of the oracle: probe generator, BF16 rounding,
Chebyshev moments, features and the network's backward pass and optimiser."""
import os

import numpy as np
import pytest

import synth
from oracle import band as oband
from oracle import chebyshev as och
from oracle import jacobi
from oracle import mlp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_sequence():
    want = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    g = 0x9E3779B97F4A7C15
    ctr = np.array([(j * g) % 2**64 for j in range(len(want))], dtype=np.uint64)
    assert [int(v) for v in och.splitmix64(ctr)] == want


def test_rademacher_probes_are_pm1_and_seeded():
    V = och.rademacher(1000, 4, seed=3)
    assert set(np.unique(V)) == {-1.0, 1.0}
    assert abs(V.mean()) < 0.1
    assert np.array_equal(V, och.rademacher(1000, 4, seed=3))
    assert not np.array_equal(V, och.rademacher(1000, 4, seed=4))


def test_bf16_rounding_against_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(1000) * 10.0 ** rng.uniform(-20, 20, 1000),
                        [1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, np.pi, 0.0, -0.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).double().numpy()
    assert np.array_equal(mlp.bf16(x), ref)
    assert mlp.bf16(np.array([1 + 2 ** -8]))[0] == 1.0             # tie to even
    assert mlp.bf16(np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6  # tie to even


def test_cheb_moments_diagonal_exact():
    d = np.linspace(-7, 3, 300)
    ab = np.zeros((3, 300))
    ab[0] = d
    mu = och.cheb_moments(ab, K=16, P=5, seed=1)
    c, h = och.scaling(ab)
    th = np.arccos((d - c) / h)
    exact = np.array([np.mean(np.cos(k * th)) for k in range(17)])
    assert np.allclose(mu, exact[None, :], atol=1e-13)


@pytest.mark.parametrize("cplx", [False, True])
def test_cheb_recurrence_against_dense(cplx):
    n = 120
    ab = synth.band_matrix(n, 5, 8, cplx, -6, 6)
    mu = och.cheb_moments(ab, K=12, P=3, seed=2)
    lam, V = jacobi.jacobi_eigh(oband.dense_from_band(ab))
    c, h = och.scaling(ab)
    lh = (lam - c) / h
    P = och.rademacher(n, 3, 2)
    W = V.conj().T @ P
    for k in range(13):
        ref = np.real(np.sum(np.abs(W) ** 2 * np.cos(k * np.arccos(lh))[:, None], axis=0)) / n
        assert np.allclose(mu[:, k], ref, atol=1e-12)
    assert np.allclose(mu[:, 0], 1.0) and np.all(np.abs(mu) <= 1.0 + 1e-12)


def test_kpm_cdf_ends_and_jackson():
    g = och.jackson(16)
    assert abs(g[0] - 1.0) < 1e-15 and np.all(np.diff(g) < 0)
    mbar = np.r_[1.0, np.zeros(16)]
    assert abs(och.kpm_cdf(mbar, np.array([-1.0]))[0]) < 1e-15
    assert abs(och.kpm_cdf(mbar, np.array([1.0]))[0] - 1.0) < 1e-15
    # semicircle-free flat density: CDF = (pi - theta)/pi
    t = np.linspace(-0.9, 0.9, 7)
    assert np.allclose(och.kpm_cdf(mbar, t), (np.pi - np.arccos(t)) / np.pi)


def test_features_shape_and_values():
    ab = synth.band_matrix(512, 16, 4, True, -20, 20)
    f = och.planner_features(ab, seed=0)
    assert f.shape == (80,) and np.all(np.isfinite(f))
    lo, hi = oband.gershgorin(ab)
    nrm = oband.norm1(ab)
    assert f[0] == lo / nrm and f[1] == hi / nrm
    cdf = f[34:66]
    assert np.all(cdf > -0.05) and np.all(cdf < 1.05)
    ev = np.linalg.eigvalsh(oband.dense_from_band(ab))
    t = lo + (np.arange(32) + 0.5) * (hi - lo) / 32
    true = np.array([(ev < s).mean() for s in t])
    assert np.abs(cdf - true).max() < 0.1   # a 16-moment estimate of the distribution


def test_mlp_backward_finite_differences():
    rng = np.random.default_rng(1)
    p = mlp.init_params(3)
    X = rng.standard_normal((7, 80))
    T = rng.uniform(0, 1, (7, 64))
    _, g = mlp.backward(p, X, T, rounding=False)
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        flat = p[k].ravel()
        for idx in rng.choice(flat.size, 4, replace=False):
            old = flat[idx]
            h = 1e-6 * max(1.0, abs(old))
            flat[idx] = old + h
            lp = mlp.loss(p, X, T, rounding=False)
            flat[idx] = old - h
            lm = mlp.loss(p, X, T, rounding=False)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[k].ravel()[idx]
            assert abs(fd - an) <= 1e-6 * max(1e-3, abs(an)), (k, idx, fd, an)


def test_adam_first_step_closed_form():
    p = {"w": np.array([1.0, -2.0, 0.5])}
    g = {"w": np.array([0.3, -1e-3, 4.0])}
    st = {}
    mlp.adam_step(p, g, st, t=1, lr=1e-2)
    assert np.allclose(p["w"], [1.0 - 1e-2, -2.0 + 1e-2, 0.5 - 1e-2], atol=1e-7)
