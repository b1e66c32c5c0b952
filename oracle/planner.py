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
certified) (tests).  The placement from previous eigenvalues (end of this
module) is pinned by hand-worked clusterings, equal-spacing fixed points,
the paper's bound-search parameters on diagonal matrices (whose inertia is a
plain count) and exact counts against dense eigenvalues.
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


# ---------------------------------------------------------------------------
# Slices from the previous eigenvalues of a sequence (Section 3.1, "K-means
# Clustering", Algorithm alg:kmeans; bounds of Section 3.2, "Validation and
# Other Details", Algorithm alg:lower_upper).  Readings:
# * k-means: the groups are runs of consecutive sorted points, held as split
#   indices; the first (n mod K) groups start with floor(n/K) + 1 points; a
#   sweep visits the K-1 boundaries in order and each update sees the groups
#   as already updated in that sweep (Gauss-Seidel); a group's centroid is
#   the midpoint of its extreme points; the boundary between G_j and G_{j+1}
#   moves to the first point greater than the midpoint of the two centroids;
#   a group left empty is dropped (K decreases); sweeps stop when no split
#   moves, at most max_sweeps (100); the boundary value is the midpoint of
#   the last point of G_j and the first of G_{j+1};
# * bounds for the lowest nev eigenvalues: the upper step is
#   s = max(alpha |d_nev|, m1 (d_nev - d_{nev-1}), 4 delta + 1e-12 ||B||_1)
#   (the last term only keeps the step positive when the first two vanish);
#   b_K = d_nev + s, advanced by s until n_-(b_K) >= nev (the stopping test
#   the text describes: at least nev eigenvalues below b_K); the lower bound
#   mirrors it with s0 = max(alpha |d_1|, m1 (d_2 - d_1), ...), b_0 = d_1 - s0,
#   moved down by s0 until n_-(b_0) = 0; alpha = 1e-3, m1 = 6;
# * every boundary is certified as above and the counts come from inertia.


def kmeans_1d(d, K: int, max_sweeps: int = 100):
    """Simplified 1-D k-means of ascending points d into at most K groups.

    Returns (splits, values, counts): splits[0] = 0 < splits[1] < ... <
    splits[K'] = len(d) delimit the groups, values[j] (j = 1..K'-1) is the
    boundary between groups j and j+1, counts the group sizes."""
    d = np.asarray(d, dtype=np.float64)
    n = d.size
    if n == 0 or K < 1:
        raise ValueError("empty data or K < 1")
    q, r = divmod(n, K)
    s = [0]
    for i in range(K):
        s.append(s[-1] + (q + 1 if i < r else q))
    s = sorted(set(s))  # groups with no point are dropped at once

    def centroid(a, b):  # points d[a:b], b > a
        return (d[a] + d[b - 1]) / 2

    for _ in range(max_sweeps):
        old = list(s)
        for j in range(1, len(s) - 1):
            if s[j] <= s[j - 1] or s[j + 1] <= s[j]:
                continue  # an empty neighbour (removed below)
            c = (centroid(s[j - 1], s[j]) + centroid(s[j], s[j + 1])) / 2
            s[j] = int(np.searchsorted(d, c, side="right"))
        s = sorted(set(s))
        if s == old:
            break
    values = [(d[s[j] - 1] + d[s[j]]) / 2 for j in range(1, len(s) - 1)]
    counts = [s[j + 1] - s[j] for j in range(len(s) - 1)]
    return s, values, counts


def _step(a: float, gap: float, alpha: float, m1: int, floor_: float) -> float:
    return max(alpha * abs(a), m1 * gap, floor_)


def upper_bound_search(ab, d, nev: int, alpha: float = 1e-3, m1: int = 6,
                       cert_delta: float = 1e-8, max_steps: int = 1000, log=None):
    """b_K above the nev lowest eigenvalues (see the readings above)."""
    log = [] if log is None else log
    nrm = norm1(ab)
    d = np.asarray(d, dtype=np.float64)
    gap = d[nev - 1] - d[nev - 2] if nev >= 2 else 0.0
    s = _step(d[nev - 1], gap, alpha, m1, 4.0 * cert_delta * nrm + 1e-12 * nrm)
    b = d[nev - 1] + s
    for _ in range(max_steps):
        if _neg(ab, b, log) >= nev:
            return b
        b = b + s
    raise RuntimeError("upper bound search did not end")


def lower_bound_search(ab, d, alpha: float = 1e-3, m1: int = 6, cert_delta: float = 1e-8,
                       max_steps: int = 1000, log=None):
    """b_0 below every eigenvalue (see the readings above)."""
    log = [] if log is None else log
    nrm = norm1(ab)
    d = np.asarray(d, dtype=np.float64)
    gap = d[1] - d[0] if d.size >= 2 else 0.0
    s = _step(d[0], gap, alpha, m1, 4.0 * cert_delta * nrm + 1e-12 * nrm)
    b = d[0] - s
    for _ in range(max_steps):
        if _neg(ab, b, log) == 0:
            return b
        b = b - s
    raise RuntimeError("lower bound search did not end")


def plan_prev(ab, prev, nev: int, K: int, alpha: float = 1e-3, m1: int = 6,
              cert_delta: float = 1e-8, max_sweeps: int = 100, max_steps: int = 1000):
    """Slices for the lowest nev eigenvalues of B from the previous eigenvalues
    (ascending): k-means boundaries between b_0 and b_K, all certified.
    Returns (bounds, counts, K', number of shifts factorised)."""
    prev = np.asarray(prev, dtype=np.float64)
    if nev < 1 or nev > prev.size or np.any(np.diff(prev) < 0):
        raise ValueError("need 1 <= nev <= len(prev) ascending previous eigenvalues")
    d = prev[:nev]
    log: list = []
    delta = cert_delta * norm1(ab)
    b0 = lower_bound_search(ab, prev, alpha, m1, cert_delta, max_steps, log)
    bK = upper_bound_search(ab, prev, nev, alpha, m1, cert_delta, max_steps, log)
    _, inner, _ = kmeans_1d(d, K, max_sweeps)
    edges, negs = [], []
    for e in [b0] + list(inner) + [bK]:
        c, v = certify(ab, e, delta, log)
        edges.append(c)
        negs.append(v)
    edges = np.array(edges)
    if np.any(np.diff(edges) <= 0):
        raise RuntimeError("certified boundaries out of order")
    return edges, np.diff(negs), len(edges) - 1, len(log)
