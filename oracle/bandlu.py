"""Band LU with partial pivoting of the shifted systems (test infrastructure).

Computing the filtered block Q amounts to n_e independent shifted systems
(z_j I - A) Q^(j) = X with many right-hand sides, one factorisation per
integration node (Section 2.2, equation eq:feast_L2).  The oracle factors
A = zI - B (lower and upper bandwidth b) by Gaussian elimination with partial
pivoting (row interchanges), which widens U to bandwidth 2b, and solves with
A (N) and with A^H (H); for Hermitian B, (conj(z) I - B)^{-1} = (zI - B)^{-H},
so one factorisation serves the node and its mirror image.

Elimination step j: the pivot is the row p in [j, j+b] of largest |a_pj|^2
(lowest row on ties), rows j and p are exchanged, the multipliers
l = A[j+1:j+b+1, j] / A[j, j] are stored, and the window
A[j+1:j+b+1, j+1:j+2b+1] receives the rank-one update -l A[j, j+1:j+2b+1].
The factorisation is A = P_0 L_0 P_1 L_1 ... P_{n-1} L_{n-1} U.

Storage of the working matrix: row i keeps columns i-b .. i+2b at positions
0..3b (``R[i, c - i + b] = A[i, c]``); at step j every entry that can be
nonzero in rows j..j+b, columns j..j+2b lies inside these windows.

Pinned by: dense ``numpy.linalg.solve`` and ``scipy.linalg.solve_banded``,
the backward error of the computed solution, and diagonal B where
x = y / (z - d) (tests).  Parity with the GPU path is on solutions, which are
unique, not on factors or pivots.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class BandLU:
    n: int
    b: int
    z: complex
    ipiv: np.ndarray    # (n,) row exchanged with row j at step j
    lower: np.ndarray   # (n, b): lower[j, i-1] = multiplier of row j+i at step j
    upper: np.ndarray   # (n, 2b+1): upper[j, k] = U[j, j+k]
    singular: bool


def shifted_band_lu(ab: np.ndarray, z: complex) -> BandLU:
    """Factor A = z I - B (B given by its lower band ``ab``)."""
    b = ab.shape[0] - 1
    n = ab.shape[1]
    R = np.zeros((n, 3 * b + 1), dtype=np.complex128)
    for d in range(1, b + 1):
        R[d:, b - d] = -ab[d, : n - d]                 # A[j+d, j] = -B[j+d, j]
        R[: n - d, b + d] = -np.conj(ab[d, : n - d])   # A[j, j+d] = -conj(B[j+d, j])
    R[:, b] = z - ab[0].real
    ipiv = np.zeros(n, dtype=np.int64)
    lower = np.zeros((n, b), dtype=np.complex128)
    upper = np.zeros((n, 2 * b + 1), dtype=np.complex128)
    singular = False
    for j in range(n):
        last = min(j + b, n - 1)
        rows = np.arange(j, last + 1)
        colj = R[rows, j - rows + b]
        p = j + int(np.argmax(colj.real ** 2 + colj.imag ** 2))
        ipiv[j] = p
        cols = np.arange(j, min(j + 2 * b, n - 1) + 1)
        if p != j:
            rj = R[j, cols - j + b].copy()
            R[j, cols - j + b] = R[p, cols - p + b]
            R[p, cols - p + b] = rj
        upper[j, : len(cols)] = R[j, cols - j + b]
        piv = R[j, b]
        if piv == 0:
            singular = True
            continue
        if last > j:
            below = rows[1:]
            l = R[below, j - below + b] / piv
            lower[j, : len(below)] = l
            c1 = cols[1:]
            if len(c1):
                R[below[:, None], c1[None, :] - below[:, None] + b] -= np.outer(l, upper[j, 1 : len(cols)])
            R[below, j - below + b] = 0.0
    return BandLU(n, b, complex(z), ipiv, lower, upper, singular)


def lu_solve(F: BandLU, Y: np.ndarray) -> np.ndarray:
    """X = A^{-1} Y: forward sweep with the row exchanges and multipliers,
    then back substitution with U (bandwidth 2b)."""
    n, b = F.n, F.b
    X = np.array(Y, dtype=np.complex128, copy=True)
    vec = X.ndim == 1
    if vec:
        X = X[:, None]
    for j in range(n):
        p = F.ipiv[j]
        if p != j:
            X[[j, p]] = X[[p, j]]
        k = min(b, n - 1 - j)
        if k:
            X[j + 1 : j + 1 + k] -= np.outer(F.lower[j, :k], X[j])
    for j in range(n - 1, -1, -1):
        k = min(2 * b, n - 1 - j)
        s = X[j] - F.upper[j, 1 : k + 1] @ X[j + 1 : j + 1 + k] if k else X[j]
        X[j] = s / F.upper[j, 0]
    return X[:, 0] if vec else X


def lu_solve_h(F: BandLU, Y: np.ndarray) -> np.ndarray:
    """X = A^{-H} Y: forward substitution with U^H, then the multipliers and
    row exchanges applied in reverse order as A^{-H} = P_0 L_0^{-H} ... U^{-H}."""
    n, b = F.n, F.b
    X = np.array(Y, dtype=np.complex128, copy=True)
    vec = X.ndim == 1
    if vec:
        X = X[:, None]
    for j in range(n):
        k = min(2 * b, j)
        if k:
            c = np.arange(j - k, j)
            coef = np.conj(F.upper[c, j - c])          # conj(U[c, j])
            X[j] = X[j] - coef @ X[j - k : j]
        X[j] = X[j] / np.conj(F.upper[j, 0])
    for j in range(n - 1, -1, -1):
        k = min(b, n - 1 - j)
        if k:
            X[j] = X[j] - np.conj(F.lower[j, :k]) @ X[j + 1 : j + 1 + k]
        p = F.ipiv[j]
        if p != j:
            X[[j, p]] = X[[p, j]]
    return X[:, 0] if vec else X


def shifted_residual(ab: np.ndarray, z: complex, X: np.ndarray, Y: np.ndarray,
                     herm: bool = False) -> np.ndarray:
    """Per-column ||y - A x||_2 / ||y||_2 for A = zI - B (herm: A^H = conj(z) I - B)."""
    from .band import band_matmul
    zz = np.conj(z) if herm else z
    R = Y - (zz * X - band_matmul(ab, X))
    return np.linalg.norm(R, axis=0) / np.linalg.norm(Y, axis=0)
