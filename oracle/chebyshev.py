"""Stochastic Chebyshev moments and the slice-planner features (test
infrastructure).

The paper names density-of-states estimation from matrix-vector products as
the alternative to inertia for a first partition of the spectrum (Section
3.1, "Spectrum Partition").  The planner's features are built from such an
estimate: Chebyshev moments of the spectrum of B scaled into [-1, 1],

    mu_k = v^T T_k(Bh) v / n,   Bh = (B - c I) / h,

with c, h from the Gershgorin interval widened by 1 %, averaged over
Rademacher probes v (+-1 entries).  The probes come from a counter-based
generator so that any implementation can reproduce them: entry i of probe p
is 1 - 2 * (SplitMix64(seed * 2^40 + p * 2^32 + i) & 1), SplitMix64 being
the published mixing function of Steele, Lea and Flood (2014) as given by
Vigna (state increment 0x9e3779b97f4a7c15, multipliers 0xbf58476d1ce4e5b9
and 0x94d049bb133111eb, shifts 30, 27, 31).

Pinned by: for diagonal B every probe gives the exact value
(1/n) sum_i T_k(d_i) (v_i^2 = 1); mu_0 = 1 and |mu_k| <= 1; the recurrence
against v^T V T_k(Lambda) V^H v from a dense eigendecomposition; the
published SplitMix64 output sequence for seed 0 (tests).
"""
from __future__ import annotations

import math

import numpy as np

from .band import band_matmul, gershgorin, norm1

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output for the 64-bit counters x (wrapping arithmetic)."""
    z = np.asarray(x, dtype=np.uint64) + np.uint64(0x9E3779B97F4A7C15)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def rademacher(n: int, P: int, seed: int) -> np.ndarray:
    """(n, P) matrix of +-1 probe entries."""
    i = np.arange(n, dtype=np.uint64)
    out = np.empty((n, P))
    for p in range(P):
        ctr = np.uint64(seed) * np.uint64(1 << 40) + np.uint64(p) * np.uint64(1 << 32) + i
        bit = (splitmix64(ctr) & np.uint64(1)).astype(np.float64)
        out[:, p] = 1.0 - 2.0 * bit
    return out


def scaling(ab: np.ndarray):
    """(c, h): Bh = (B - c I) / h maps the Gershgorin interval, widened by
    1 %, onto [-1, 1]."""
    lo, hi = gershgorin(ab)
    return 0.5 * (lo + hi), 1.01 * 0.5 * (hi - lo)


def cheb_moments(ab: np.ndarray, K: int = 16, P: int = 20, seed: int = 0) -> np.ndarray:
    """(P, K+1) array: mu[p, k] = v_p^T T_k(Bh) v_p / n (three-term recurrence
    T_{k+1}(x) = 2 x T_k(x) - T_{k-1}(x))."""
    n = ab.shape[1]
    c, h = scaling(ab)
    V = rademacher(n, P, seed)
    mu = np.zeros((P, K + 1))

    def apply(X):
        return (band_matmul(ab, X) - c * X) / h

    t0 = V.astype(np.complex128)
    mu[:, 0] = np.real(np.sum(V * t0, axis=0)) / n
    if K >= 1:
        t1 = apply(t0)
        mu[:, 1] = np.real(np.sum(V * t1, axis=0)) / n
        for k in range(2, K + 1):
            t2 = 2.0 * apply(t1) - t0
            mu[:, k] = np.real(np.sum(V * t2, axis=0)) / n
            t0, t1 = t1, t2
    return mu


def jackson(K: int) -> np.ndarray:
    """Jackson damping factors g_0..g_K for K+1 moments."""
    N = K + 1
    k = np.arange(K + 1)
    a = np.pi / (N + 1)
    return ((N - k + 1) * np.cos(a * k) + np.sin(a * k) / np.tan(a)) / (N + 1)


def kpm_cdf(mbar: np.ndarray, that: np.ndarray) -> np.ndarray:
    """Fraction of the spectrum below the scaled points that (in (-1, 1)) from
    the damped Chebyshev expansion of the density: with t = cos(theta),
    CDF = [g_0 mu_0 (pi - theta) - 2 sum_k g_k mu_k sin(k theta) / k] / pi."""
    K = len(mbar) - 1
    g = jackson(K)
    th = np.arccos(np.clip(that, -1.0, 1.0))
    val = g[0] * mbar[0] * (np.pi - th)
    for k in range(1, K + 1):
        val = val - 2.0 * g[k] * mbar[k] * np.sin(k * th) / k
    return val / np.pi


N_FEATURES = 80
N_OUTPUTS = 64


def planner_features(ab: np.ndarray, seed: int = 0, K: int = 16, P: int = 20) -> np.ndarray:
    """The 80 planner features of B:
    [g_lo/||B||_1, g_hi/||B||_1] + mean over probes of mu_1..mu_16 +
    their standard deviations + the damped Chebyshev CDF at 32 evenly spaced
    points of the Gershgorin interval + 14 scalars (log2 n / 16, b / 128,
    complex flag, diagonal mean, std, min, max over ||B||_1, diagonal skew
    and excess kurtosis / 10, off-diagonal energy per row over ||B||_1^2,
    log10 ||B||_1, Gershgorin width over ||B||_1, ||B||_F^2 / n / ||B||_1^2,
    diagonal range over Gershgorin width)."""
    n = ab.shape[1]
    b = ab.shape[0] - 1
    lo, hi = gershgorin(ab)
    nrm = norm1(ab)
    c, h = scaling(ab)
    mu = cheb_moments(ab, K, P, seed)
    mbar = mu.mean(axis=0)
    f = [lo / nrm, hi / nrm]
    f += list(mbar[1:])
    f += list(mu[:, 1:].std(axis=0))
    t = lo + (np.arange(32) + 0.5) * (hi - lo) / 32
    f += list(kpm_cdf(mbar, (t - c) / h))
    d = ab[0].real.astype(np.float64)
    dm = d.mean()
    ds = d.std()
    skew = np.mean((d - dm) ** 3) / ds ** 3 if ds > 0 else 0.0
    kurt = np.mean((d - dm) ** 4) / ds ** 4 - 3.0 if ds > 0 else 0.0
    off = 2.0 * sum(np.sum(np.abs(ab[k, : n - k]) ** 2) for k in range(1, b + 1))
    fro2 = np.sum(d * d) + off
    f += [math.log2(n) / 16.0, b / 128.0, 1.0 if np.iscomplexobj(ab) else 0.0,
          dm / nrm, ds / nrm, d.min() / nrm, d.max() / nrm, skew, kurt / 10.0,
          off / n / nrm ** 2, math.log10(nrm), (hi - lo) / nrm, fro2 / n / nrm ** 2,
          (d.max() - d.min()) / (hi - lo)]
    return np.array(f)


def planner_shifts(ab: np.ndarray) -> np.ndarray:
    """The 64 label shifts s_k = g_lo + (k + 1/2)(g_hi - g_lo)/64."""
    lo, hi = gershgorin(ab)
    return lo + (np.arange(N_OUTPUTS) + 0.5) * (hi - lo) / N_OUTPUTS
