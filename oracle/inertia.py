"""Sylvester inertia of B - sigma I (test infrastructure).

The paper places and validates slices with Sylvester's law of inertia: an
LDL^H factorisation of (D - s I) gives the number of eigenvalues below s
(Section 3.1 "Spectrum Partition", and Section 3.2 "Validation and Other
Details", where m_i = n_-(b_i) - n_-(b_{i-1}) checks every slice).  The paper
computes only the inertia, with a simplified retraction algorithm; the
reading taken here is a band LDL^H without pivoting in FP64, which yields the
same counts whenever sigma is not within rounding distance of an eigenvalue
(slice boundaries are certified to stay away from eigenvalues).

A pivot with |d_k| < pivmin = eps^2 * ||B||_1 is counted as zero (n_0) and
replaced by -pivmin so that the elimination can continue.

Pinned by: dense eigenvalue counts, diagonal B (n_- = #{a_ii < sigma}), the
closed-form spectrum of a tridiagonal Toeplitz matrix, n_- + n_0 + n_+ = n,
monotonicity in sigma, n_-(g_lo) = 0 and n_-(g_hi) = n at the Gershgorin
bounds (tests).
"""
from __future__ import annotations

import numpy as np

from .band import norm1

_EPS = np.finfo(np.float64).eps


def inertia(ab: np.ndarray, sigma: float) -> tuple[int, int, int]:
    """(n_-, n_0, n_+) of B - sigma I by band LDL^H without pivoting."""
    b = ab.shape[0] - 1
    n = ab.shape[1]
    pivmin = _EPS * _EPS * norm1(ab)
    W = np.array(ab, dtype=np.result_type(ab.dtype, np.float64), copy=True)
    W[0] = ab[0].real - sigma
    neg = zero = 0
    tri = {}
    for k in range(n):
        dk = float(np.real(W[0, k]))
        if abs(dk) < pivmin:
            zero += 1
            dk = -pivmin
        elif dk < 0.0:
            neg += 1
        m = min(b, n - 1 - k)
        if m == 0:
            continue
        if m not in tri:
            tri[m] = np.tril_indices(m)
        I, J = tri[m]
        a = W[1 : m + 1, k]
        # A[k+1+i, k+1+j] -= A[k+1+i, k] conj(A[k+1+j, k]) / d_k for j <= i,
        # stored at W[i - j, k + 1 + j]
        W[I - J, k + 1 + J] -= a[I] * np.conj(a[J]) / dk
    return neg, zero, n - neg - zero


def count_in(ab: np.ndarray, lo: float, hi: float) -> int:
    """Eigenvalues of B in [lo, hi): n_-(hi) - n_-(lo)."""
    return inertia(ab, hi)[0] - inertia(ab, lo)[0]
