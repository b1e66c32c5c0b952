"""Cyclic Jacobi eigensolver for dense Hermitian matrices (test infrastructure).

Used by the oracle for the reduced problems of the Rayleigh-Ritz step
(Section 2.2, "The FEAST Algorithm": A_q W_q = W_q Lambda_q) and for the
Golub-Welsch quadrature nodes.  Textbook two-sided Jacobi (Golub & Van Loan,
symmetric Schur decomposition of 2x2 blocks), with the disjoint pairs of a
round-robin ordering applied together per round.

Pinned by: ``numpy.linalg.eigh`` eigenvalues, V^H V = I and A V = V diag(w)
(tests).
"""
from __future__ import annotations

import numpy as np


def _round_robin(m: int):
    """Rounds of disjoint pairs covering every pair (p, q) once (circle method)."""
    players = list(range(m)) + ([-1] if m % 2 else [])
    k = len(players)
    rounds = []
    for _ in range(k - 1):
        pairs = [(players[i], players[k - 1 - i]) for i in range(k // 2)]
        pairs = [(min(p, q), max(p, q)) for p, q in pairs if p >= 0 and q >= 0]
        rounds.append((np.array([p for p, _ in pairs], dtype=np.int64),
                       np.array([q for _, q in pairs], dtype=np.int64)))
        players = [players[0]] + [players[-1]] + players[1:-1]
    return rounds


def jacobi_eigh(A: np.ndarray, tol: float = 1e-15, max_sweeps: int = 40):
    """Eigen-decomposition A = V diag(w) V^H of a Hermitian matrix, w ascending.

    Each 2x2 block [[a, c], [conj(c), d]] is first made real by the phase
    e^{-i arg c} on index q, then rotated by the symmetric Schur rotation
    t = sign(tau)/(|tau| + sqrt(1+tau^2)), tau = (d-a)/(2|c|).
    Sweeps stop when ||offdiag(A)||_F <= tol * ||A||_F.
    """
    A = np.array(A, dtype=np.result_type(A.dtype, np.float64), copy=True)
    m = A.shape[0]
    cplx = np.iscomplexobj(A)
    V = np.eye(m, dtype=A.dtype)
    if m == 1:
        return A.real.diagonal().copy(), V
    rounds = _round_robin(m)
    fro = np.linalg.norm(A)
    for _ in range(max_sweeps):
        off = np.linalg.norm(A - np.diag(np.diag(A)))
        if off <= tol * fro or off == 0.0:
            break
        for P, Q in rounds:
            a = A[P, P].real
            d = A[Q, Q].real
            c = A[P, Q]
            ac = np.abs(c)
            act = ac > 1e-300
            safe = np.where(act, ac, 1.0)
            tau = (d - a) / (2.0 * safe)
            t = np.where(tau >= 0, 1.0, -1.0) / (np.abs(tau) + np.hypot(1.0, tau))
            cs = 1.0 / np.sqrt(1.0 + t * t)
            sn = t * cs
            cs = np.where(act, cs, 1.0)
            sn = np.where(act, sn, 0.0)
            ph = c / safe if cplx else np.sign(c) + (c == 0)
            ph = np.where(act, ph, 1.0)
            eph = np.conj(ph)          # e^{-i phi}
            # columns: [A_p, A_q] <- [A_p, A_q] [[cs, sn], [-sn e, cs e]]
            Ap = A[:, P].copy()
            Aq = A[:, Q].copy()
            A[:, P] = cs * Ap - sn * eph * Aq
            A[:, Q] = sn * Ap + cs * eph * Aq
            Vp = V[:, P].copy()
            Vq = V[:, Q].copy()
            V[:, P] = cs * Vp - sn * eph * Vq
            V[:, Q] = sn * Vp + cs * eph * Vq
            # rows: [A_p; A_q] <- [[cs, -sn conj(e)], [sn, cs conj(e)]] [A_p; A_q]
            Rp = A[P, :].copy()
            Rq = A[Q, :].copy()
            A[P, :] = cs[:, None] * Rp - (sn * np.conj(eph))[:, None] * Rq
            A[Q, :] = sn[:, None] * Rp + (cs * np.conj(eph))[:, None] * Rq
    w = A.real.diagonal().copy()
    order = np.argsort(w, kind="stable")
    return w[order], V[:, order]
