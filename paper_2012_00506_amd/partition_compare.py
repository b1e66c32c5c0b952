"""Spectrum partitions compared on one step of a sequence (Section 3.1: the
k-means partition of Algorithm alg:kmeans against Approach-1, equal counts
with boundaries at midpoints between the previous eigenvalues, and
Approach-2, equal widths between the same outer bounds).

The previous matrix B0 has a clustered spectrum; its lowest ``nev``
eigenvalues come from FEAST on B0 itself.  The next matrix is
B1 = B0 + 1e-3 E.  Each partition of the lowest nev eigenvalues of B1 is
certified by exact inertia and solved by FEAST from random start blocks;
the report gives, per partition, the slice counts, the iterations, the time,
the smallest distance from an inner boundary to an eigenvalue (in units of
the mean spacing) and the orthogonality of the computed eigenvectors, split
into max |X_i^H X_i - I| within slices and max |X_i^H X_j| across them.

    python -m paper_2012_00506_amd.partition_compare [--n N] [--nev NEV] [--K K]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np
import torch

from . import api


def clustered_matrix(n: int, b: int, seed: int, clusters: int) -> np.ndarray:
    """Complex Hermitian band: diagonal a Gaussian mixture of ``clusters``
    narrow clusters, off-diagonals complex N(0, 1/b) scaled by 1/4."""
    rng = np.random.default_rng(seed)
    centers = np.sort(rng.uniform(-40.0, 40.0, clusters))
    widths = rng.uniform(0.02, 0.2, clusters)
    which = rng.integers(0, clusters, n)
    diag = np.sort(centers[which] + widths[which] * rng.standard_normal(n))
    ab = np.zeros((b + 1, n), np.complex128)
    ab[0] = diag
    s = 0.25 * np.sqrt(1.0 / (2 * b))
    for k in range(1, b + 1):
        ab[k, : n - k] = (rng.standard_normal(n - k) + 1j * rng.standard_normal(n - k)) * s
    return ab


def perturbation(n: int, b: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    ab = np.zeros((b + 1, n), np.complex128)
    ab[0] = rng.standard_normal(n)
    s = np.sqrt(1.0 / (2 * b))
    for k in range(1, b + 1):
        ab[k, : n - k] = (rng.standard_normal(n - k) + 1j * rng.standard_normal(n - k)) * s
    return ab


def _random_block(n, m, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    return torch.randn((m, n), generator=g, device="cuda", dtype=torch.complex128).t()


def solve_partition(B, bounds, counts, seed, precision, tol, reps=2):
    """FEAST on the partition from seeded random start blocks; the time is
    that of the last of ``reps`` identical runs (the first pays one-off
    set-up)."""
    m0 = [api.m0_rule(int(c)) for c in counts]
    for _ in range(reps):
        Y = [_random_block(B.n, m, seed + i) for i, m in enumerate(m0)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = api.feast_band_slice(B, bounds[:-1], bounds[1:], Y, m_expected=counts, tol=tol,
                                   precision=precision, ir_tol=1e-10 if precision else 1e-12)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    Xs = [r.Y[:, : r.m_found] for r in res if r.m_found]
    X = torch.cat(Xs, dim=1)
    G = X.conj().t() @ X
    G -= torch.eye(G.shape[0], dtype=G.dtype, device=G.device)
    # within-slice blocks of the Gram matrix, then everything else
    within = 0.0
    c0 = 0
    for x in Xs:
        m = x.shape[1]
        within = max(within, float(G[c0:c0 + m, c0:c0 + m].abs().max()))
        G[c0:c0 + m, c0:c0 + m] = 0
        c0 += m
    lam = np.concatenate([r.lam for r in res])
    return {
        "counts": [int(c) for c in counts],
        "balance_max_over_mean": float(np.max(counts) / np.mean(counts)),
        "iters": [r.iters for r in res],
        "info": [r.info for r in res],
        "seconds": dt,
        "orthogonality_within": within,
        "orthogonality_across": float(G.abs().max()),
        "max_resid": float(max(r.resid[: r.m_found].max() for r in res if r.m_found)),
        "lam": lam,
    }


def boundary_gap(bounds, lam):
    """Smallest distance from an inner boundary to an eigenvalue, in units of
    the mean spacing of lam."""
    lam = np.sort(lam)
    spacing = (lam[-1] - lam[0]) / max(len(lam) - 1, 1)
    d = [np.abs(lam - s).min() for s in bounds[1:-1]]
    return float(min(d) / spacing) if d else float("inf")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=6000)
    ap.add_argument("--b", type=int, default=16)
    ap.add_argument("--nev", type=int, default=1500)
    ap.add_argument("--K", type=int, default=8)
    ap.add_argument("--clusters", type=int, default=60)
    ap.add_argument("--precision", type=int, default=1)
    ap.add_argument("--seed", type=int, default=11)
    ap.add_argument("--tol", type=float, default=1e-10)
    a = ap.parse_args(argv)
    ab0 = clustered_matrix(a.n, a.b, a.seed, a.clusters)
    ab1 = ab0 + 1e-3 * perturbation(a.n, a.b, a.seed + 1)
    B0 = api.DeviceBand.from_band(ab0)
    B1 = api.DeviceBand.from_band(ab1)
    # the previous step: the lowest nev eigenvalues of B0 by FEAST on equal-count slices
    b0, c0, _ = api.slice_plan(B0, a.K, mode="equal_count", nev=a.nev)
    r0 = solve_partition(B0, b0, c0, 1000, a.precision, a.tol, reps=1)
    prev = np.sort(r0["lam"])
    # k-means (Algorithm alg:kmeans) with the searched outer bounds
    bk, ck, _ = api.slice_plan_prev(B1, prev, a.nev, a.K)
    lo, hi = bk[0], bk[-1]
    # Approach-1: groups of nev / K previous eigenvalues, midpoints between groups
    idx = [round(i * a.nev / a.K) for i in range(1, a.K)]
    b1 = np.array([lo] + [0.5 * (prev[j - 1] + prev[j]) for j in idx] + [hi])
    b1, _, c1, _, _ = api.slice_certify(B1, b1)
    # Approach-2: equal widths between the same outer bounds
    b2, _, c2, _, _ = api.slice_certify(B1, np.linspace(lo, hi, a.K + 1))
    out = {"n": a.n, "b": a.b, "nev": a.nev, "K": a.K, "clusters": a.clusters,
           "precision": a.precision, "tol": a.tol}
    for name, bb, cc in (("kmeans", bk, ck), ("approach1", b1, c1), ("approach2", b2, c2)):
        r = solve_partition(B1, bb, cc, 2000, a.precision, a.tol)
        r["inner_boundary_gap_over_mean_spacing"] = boundary_gap(bb, r.pop("lam"))
        r["bounds"] = [float(v) for v in bb]
        out[name] = r
    print(json.dumps(out), flush=True)
    return out


if __name__ == "__main__":
    main()
