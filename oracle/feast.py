"""The FEAST iteration on a band Hermitian matrix (test infrastructure).

Follows the FEAST algorithm as the paper states it (Section 2.2, Algorithm
alg:FEAST): while the eigen-residual is above the tolerance, apply the
rational filter Q = r(A) X by the shifted solves, project with Rayleigh-Ritz
A_q = Q^H A Q, solve A_q W = W Lambda, and set X = Q W.  The slice count m is
known exactly from two inertias and every slice is checked against it
(Section 3.2 "Validation and Other Details").

Readings of points the paper leaves open:
* stop test: the number of Ritz pairs with eigenvalue in [lo, hi) and
  residual ||B x - lambda x||_2 / ||B||_1 <= tol (||x||_2 = 1) equals the
  inertia count m; at most ``max_iter`` iterations.  Ritz pairs inside the
  slice whose residual stays large are spurious (mixtures of eigenvectors
  outside the slice that the unconverged edge of the search subspace
  produces) and are not reported; the exact count is what tells them apart;
* orthonormalisation (the mass matrix of the standard problem is I): two
  passes over the eigen-decomposition Q^H Q = V s V^H.  The first forms Q V
  over every eigenvector and keeps the columns whose norm, measured on the
  product, exceeds 1e-12 times the largest, each scaled to unit norm; the
  second replaces that block by Q' V' s'^{-1/2}, dropping directions with
  s'_k <= 1e-14 max(s') (if any are dropped, the next start block keeps the
  trailing columns of the previous one);
* for complex Hermitian B the filter is
  Q = sum_j [w_j (z_j I - B)^{-1} Y + conj(w_j) (z_j I - B)^{-H} Y];
  for real symmetric B with real Y it is Q = sum_j 2 Re[w_j (z_j I - B)^{-1} Y].

The small dense Hermitian eigenproblems use ``numpy.linalg.eigh`` as a
library step.

Pinned by: for diagonal B, Q = diag(r(d_i)) Y exactly; for small B,
Q = V r(Lambda) V^H Y from the oracle's own dense Jacobi; the converged
eigenvalues against dense eigenvalues of B; counts against inertia; the
invariants of a full-spectrum run (sum lambda = tr B,
sum lambda^2 = ||B||_F^2); orthonormality (tests).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .band import band_matmul, norm1
from .bandlu import lu_solve, lu_solve_h, shifted_band_lu
from .inertia import count_in
from .quadrature import contour


def factor_nodes(ab: np.ndarray, z) -> list:
    """One band LU per integration node (equation eq:feast_L2)."""
    return [shifted_band_lu(ab, zj) for zj in z]


def filter_apply(ab: np.ndarray, factors, w, Y: np.ndarray) -> np.ndarray:
    """Q = r(B) Y by the shifted solves, summed over the nodes in order."""
    if np.iscomplexobj(ab):
        Q = np.zeros(Y.shape, dtype=np.complex128)
        for F, wj in zip(factors, w):
            Q += wj * lu_solve(F, Y)
            Q += np.conj(wj) * lu_solve_h(F, Y)
        return Q
    Q = np.zeros(Y.shape, dtype=np.float64)
    for F, wj in zip(factors, w):
        Q += 2.0 * np.real(wj * lu_solve(F, Y))
    return Q


def _orthonormalise_once(Q: np.ndarray, drop: float):
    G = Q.conj().T @ Q
    G = 0.5 * (G + G.conj().T)
    s, V = np.linalg.eigh(G)
    keep = s > drop * s.max() if s.max() > 0 else np.zeros(len(s), bool)
    return (Q @ V[:, keep]) / np.sqrt(s[keep])


def orthonormalise(Q: np.ndarray, drop: float = 1e-14, floor: float = 1e-12):
    """Two passes.  The filtered block is ill-conditioned by design: its
    Gram matrix Q^H Q spans more orders of magnitude than FP64 resolves, so
    its smallest eigenvalues s_k are rounding noise (often negative) while
    the directions Q v_k themselves, formed from Q, are still accurate to
    about eps ||Q|| / ||Q v_k||.  Those directions carry the last digits of
    the wanted eigenvectors: dropping the ones whose computed s_k is at or
    below eps max(s) makes the residuals stall (near 1e-10 with 16 nodes
    from an almost converged block, near 1e-8 when directions below 1e-7 are
    dropped).  So the first pass takes Q V over every eigenvector, measures
    each column's norm on the product, keeps the columns above floor times
    the largest and scales them to unit norm; the second pass
    orthonormalises that well-scaled block as Q' V' s'^{-1/2} and takes the
    rank decision, s' > drop max(s'), bringing Q''^H Q'' - I to rounding
    level."""
    G = Q.conj().T @ Q
    G = 0.5 * (G + G.conj().T)
    _, V = np.linalg.eigh(G)
    Q1 = Q @ V
    c = np.linalg.norm(Q1, axis=0)
    keep = c > floor * c.max() if c.max() > 0 else np.zeros(len(c), bool)
    Q2 = _orthonormalise_once(Q1[:, keep] / c[keep], drop)
    return Q2, Q2.shape[1]


def _cholesky_upper(G: np.ndarray, piv_min: float):
    """Upper R with G = R^H R by the column-oriented Cholesky recurrence
    (r_jj = sqrt(g_jj - sum_i<j |r_ij|^2), r_jk = (g_jk - sum_i<j conj(r_ij)
    r_ik) / r_jj); None when a pivot r_jj^2 is not above piv_min (or NaN)."""
    m = G.shape[0]
    R = np.zeros_like(G)
    for j in range(m):
        d = np.real(G[j, j]) - np.real(np.vdot(R[:j, j], R[:j, j]))
        if not d > piv_min:
            return None
        R[j, j] = np.sqrt(d)
        R[j, j + 1:] = (G[j, j + 1:] - R[:j, j].conj() @ R[:j, j + 1:]) / R[j, j]
    return R


def orthonormalise_cholqr(Q: np.ndarray, piv_min: float = 1e-12):
    """Cholesky QR applied twice to the column-equilibrated block, or None
    when it does not apply.  D scales every column of Q to unit norm (the
    filtered block's columns differ in norm by the filter's range, which the
    scaling takes out of the Gram matrix); G = (QD)^H (QD) = R^H R and
    Q1 = Q D R^{-1}; then Q1^H Q1 = R2^H R2 and Q2 = Q1 R2^{-1}.  The first
    pass applies while every pivot r_jj^2 of G (a unit-diagonal matrix:
    r_jj is the sine of the angle between column j and the span of the
    columns before it) is above piv_min, i.e. the equilibrated Gram matrix
    has no eigenvalue near 1e-12; the second pass must factor too.  A zero
    column also rules it out."""
    c = np.linalg.norm(Q, axis=0)
    if not (c.size and np.all(c > 0) and np.all(np.isfinite(c))):
        return None
    Qd = Q / c
    G = Qd.conj().T @ Qd
    G = 0.5 * (G + G.conj().T)
    R = _cholesky_upper(G, piv_min)
    if R is None:
        return None
    Q1 = Qd @ np.linalg.inv(R)
    G2 = Q1.conj().T @ Q1
    G2 = 0.5 * (G2 + G2.conj().T)
    R2 = _cholesky_upper(G2, piv_min)
    if R2 is None:
        return None
    return Q1 @ np.linalg.inv(R2)


def rayleigh_ritz(ab: np.ndarray, Q: np.ndarray, stats: dict | None = None):
    """Ritz values (ascending) and vectors of B on span(Q).  The basis is
    orthonormalised by Cholesky QR twice when it applies, else by the two
    eigen-decomposition passes (rank decision included)."""
    Qc = orthonormalise_cholqr(Q)
    if Qc is not None:
        Qo, k = Qc, Qc.shape[1]
    else:
        Qo, k = orthonormalise(Q)
    if stats is not None:
        stats["cholqr" if Qc is not None else "eig"] = stats.get(
            "cholqr" if Qc is not None else "eig", 0) + 1
    Aq = Qo.conj().T @ band_matmul(ab, Qo)
    Aq = 0.5 * (Aq + Aq.conj().T)
    lam, W = np.linalg.eigh(Aq)
    X = Qo @ W
    return lam, X, k


def eig_residuals(ab: np.ndarray, X: np.ndarray, lam: np.ndarray, nrm: float) -> np.ndarray:
    """||B x_k - lambda_k x_k||_2 / (||B||_1 ||x_k||_2) per pair."""
    R = band_matmul(ab, X) - X * lam[None, :]
    return np.linalg.norm(R, axis=0) / (nrm * np.linalg.norm(X, axis=0))


def orthogonality(X: np.ndarray) -> float:
    """Orth = ||X^H X - I||_max / n (Section 4, the metric used for Table
    tab:orthogonality)."""
    G = X.conj().T @ X
    return float(np.abs(G - np.eye(G.shape[0])).max() / X.shape[0])


@dataclass
class SliceResult:
    lo: float
    hi: float
    m: int                      # exact count from inertia
    lam: np.ndarray             # in-slice Ritz values, ascending
    X: np.ndarray               # in-slice Ritz vectors
    res: np.ndarray             # their residuals
    iters: int
    info: int                   # 0 ok, 1 not converged, 2 count mismatch
    history: list = field(default_factory=list)
    Y_next: np.ndarray | None = None   # all Ritz vectors (warm start)


def feast_slice(ab: np.ndarray, lo: float, hi: float, Y: np.ndarray,
                n_nodes: int = 8, tol: float = 1e-10, max_iter: int = 20,
                m_expected: int | None = None, rule: str = "gauss",
                ratio: float = 1.0) -> SliceResult:
    """Eigenpairs of B in [lo, hi) by FEAST from the start block Y (n x m0)."""
    nrm = norm1(ab)
    m = count_in(ab, lo, hi) if m_expected is None else m_expected
    z, w = contour(lo, hi, n_nodes, rule, ratio)
    factors = factor_nodes(ab, z)
    Y = np.array(Y, dtype=np.complex128 if np.iscomplexobj(ab) else np.float64, copy=True)
    m0 = Y.shape[1]
    hist = []
    info = 1
    it = 0
    for it in range(1, max_iter + 1):
        Q = filter_apply(ab, factors, w, Y)
        lam, X, k = rayleigh_ritz(ab, Q)
        res = eig_residuals(ab, X, lam, nrm)
        inside = (lam >= lo) & (lam < hi)
        good = inside & (res <= tol)
        hist.append((int(inside.sum()), int(good.sum())))
        if k < m0:
            X = np.concatenate([X, Y[:, k:m0]], axis=1)
        Y = X
        if good.sum() == m:
            info = 0
            break
    else:
        info = 2 if good.sum() > m or inside.sum() < m else 1
    return SliceResult(lo, hi, m, lam[good], X[:, : len(lam)][:, good], res[good],
                       it, info, hist, Y)
