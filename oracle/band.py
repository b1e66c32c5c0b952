"""Band-matrix helpers (test infrastructure, see the package docstring).

Storage: ``ab`` of shape (b+1, n), ``ab[d, j] = B[j+d, j]`` (lower band of a
Hermitian or real symmetric matrix, the compact LAPACK form the paper keeps on
every process, Section 3 "Proposed algorithm").
"""
from __future__ import annotations

import numpy as np


def bandwidth(ab: np.ndarray) -> int:
    return ab.shape[0] - 1


def dense_from_band(ab: np.ndarray) -> np.ndarray:
    """Expand the lower band into the full Hermitian matrix B.

    Pinned by: Hermitian symmetry and the band product (tests)."""
    b = bandwidth(ab)
    n = ab.shape[1]
    B = np.zeros((n, n), dtype=np.result_type(ab.dtype, np.float64))
    for d in range(b + 1):
        idx = np.arange(n - d)
        B[idx + d, idx] = ab[d, : n - d]
        if d > 0:
            B[idx, idx + d] = np.conj(ab[d, : n - d])
    # the diagonal of a Hermitian matrix is real
    B[np.arange(n), np.arange(n)] = ab[0].real
    return B


def band_matmul(ab: np.ndarray, X: np.ndarray) -> np.ndarray:
    """B @ X using only the stored diagonals (no dense expansion).

    (B X)[i] = sum_d B[i, i-d] X[i-d] + sum_{d>0} B[i, i+d] X[i+d] with
    B[i+d, i] = ab[d, i] and B[i, i+d] = conj(ab[d, i]).
    Pinned by: dense product of ``dense_from_band`` (tests)."""
    b = bandwidth(ab)
    n = ab.shape[1]
    X = np.asarray(X)
    vec = X.ndim == 1
    if vec:
        X = X[:, None]
    Y = np.zeros((n, X.shape[1]), dtype=np.result_type(ab.dtype, X.dtype, np.float64))
    Y += ab[0].real[:, None] * X
    for d in range(1, b + 1):
        sub = ab[d, : n - d][:, None]
        Y[d:] += sub * X[: n - d]               # B[i, i-d] for i >= d
        Y[: n - d] += np.conj(sub) * X[d:]      # B[i, i+d]
    return Y[:, 0] if vec else Y


def norm1(ab: np.ndarray) -> float:
    """||B||_1 = max column sum of |B_ij| over the full matrix.

    Pinned by: ``numpy.linalg.norm(dense, 1)`` (tests)."""
    b = bandwidth(ab)
    n = ab.shape[1]
    s = np.abs(ab[0].real).astype(np.float64)
    for d in range(1, b + 1):
        a = np.abs(ab[d, : n - d])
        s[: n - d] += a      # column j holds B[j+d, j]
        s[d:] += a           # column j+d holds B[j, j+d]
    return float(s.max())


def gershgorin(ab: np.ndarray) -> tuple[float, float]:
    """Gershgorin interval [min(a_ii - R_i), max(a_ii + R_i)], R_i = sum_{j!=i} |B_ij|.

    Pinned by: containment of the dense spectrum (tests)."""
    b = bandwidth(ab)
    n = ab.shape[1]
    r = np.zeros(n)
    for d in range(1, b + 1):
        a = np.abs(ab[d, : n - d])
        r[d:] += a
        r[: n - d] += a
    dg = ab[0].real
    return float((dg - r).min()), float((dg + r).max())
