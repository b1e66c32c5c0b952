"""Slice placement by exact inertia (test infrastructure).

The paper partitions the spectrum by Sylvester inertia (Section 3.1) and
names two simple schemes beside its k-means: equal eigenvalue counts per
slice (Approach-1) and equal-width slices (Approach-2); every slice count is
exact from two inertias (Section 3.2).

Readings:
* a boundary sigma is certified when n_-(sigma - delta) = n_-(sigma + delta)
  with delta = cert_delta * ||B||_1, so that no eigenvalue lies within delta
  of it and any two correct inertia codes agree on every count; an
  uncertified boundary is moved to the first certified point of
  sigma + 2 delta s, s = 1, -1, 2, -2, ... (at most 64 tries);
* equal count: the target cumulative counts are
  t_i = n_lo + round(i (n_hi - n_lo) / K); each interior boundary is bisected
  inside the tightest bracket known so far until |n_-(sigma) - t_i| <= tol_i,
  tol_i = floor(count_tol * (n_hi - n_lo) / K), one shift per open boundary
  per round, at most ``max_rounds`` rounds;
* with no interval given the whole spectrum is partitioned: the Gershgorin
  interval widened by 4 delta + 1e-12 ||B||_1 on each side, since a
  Gershgorin bound can itself be an eigenvalue (diagonal B) and [lo, hi)
  must hold every eigenvalue.

Pinned by: exact counts against dense eigenvalues, and the invariants
(boundaries increasing, counts sum to n_-(hi) - n_-(lo), every boundary
certified) (tests).
"""
from __future__ import annotations

import math

import numpy as np

from .band import gershgorin, norm1
from .inertia import inertia


def _neg(ab, s, log):
    v = inertia(ab, s)[0]
    log.append(s)
    return v


def certify(ab, sigma: float, delta: float, log: list):
    """Move sigma off any eigenvalue closer than delta (see the module readings)."""
    cands = [sigma] + [sigma + 2.0 * delta * s for k in range(1, 33) for s in (k, -k)]
    for c in cands:
        a = _neg(ab, c - delta, log)
        b = _neg(ab, c + delta, log)
        if a == b:
            return c, a
    raise RuntimeError("boundary could not be certified")


def plan_equal_width(ab, K: int, lo: float, hi: float, cert_delta: float = 1e-8):
    log: list = []
    delta = cert_delta * norm1(ab)
    edges = [lo + (hi - lo) * i / K for i in range(K + 1)]
    edges[-1] = hi
    out, cnt = [], []
    for e in edges:
        c, v = certify(ab, e, delta, log)
        out.append(c)
        cnt.append(v)
    counts = [cnt[i + 1] - cnt[i] for i in range(K)]
    return np.array(out), np.array(counts), len(log)


def plan_equal_count(ab, K: int, lo: float | None = None, hi: float | None = None,
                     count_tol: float = 0.05, cert_delta: float = 1e-8,
                     max_rounds: int = 60):
    """Equal-count slices of [lo, hi) by batched bisection on inertia."""
    log: list = []
    g_lo, g_hi = gershgorin(ab)
    nrm = norm1(ab)
    delta = cert_delta * nrm
    pad = 4.0 * delta + 1e-12 * nrm
    lo = g_lo - pad if lo is None or math.isnan(lo) else lo
    hi = g_hi + pad if hi is None or math.isnan(hi) else hi
    lo, n_lo = certify(ab, lo, delta, log)
    hi, n_hi = certify(ab, hi, delta, log)
    total = n_hi - n_lo
    targets = [n_lo + int(round(i * total / K)) for i in range(1, K)]
    tol = int(math.floor(count_tol * total / K))
    known = {lo: n_lo, hi: n_hi}
    found = [None] * (K - 1)
    for _ in range(max_rounds):
        xs = sorted(known)
        shifts = []
        for i, t in enumerate(targets):
            if found[i] is not None:
                continue
            # tightest bracket: a = largest known point with n_-(a) <= t, b = next point
            ia = max(j for j, x in enumerate(xs) if known[x] <= t)
            a, b = xs[ia], xs[min(ia + 1, len(xs) - 1)]
            if abs(known[a] - t) <= tol:
                found[i] = a
            elif abs(known[b] - t) <= tol:
                found[i] = b
            else:
                shifts.append(0.5 * (a + b))
        if not shifts:
            break
        for s in shifts:
            if s not in known:
                known[s] = _neg(ab, s, log)
    xs = sorted(known)
    for i, t in enumerate(targets):
        if found[i] is None:   # closest known point after the round cap
            found[i] = min(xs, key=lambda x: (abs(known[x] - t), x))
    inner = []
    for s in found:
        c, _ = certify(ab, s, delta, log)
        inner.append(c)
    edges = [lo] + inner + [hi]
    negs = [inertia(ab, e)[0] for e in edges]
    counts = np.diff(negs)
    return np.array(edges), counts, len(log)
