"""Seeded synthetic inputs for the banded FEAST path.

This module holds only input generation: random band matrices, start blocks and
their recipes.  It computes nothing the method computes (no shifts, factors,
filters, projections or counts), so the CPU oracle and the GPU path may both
draw their inputs from it without sharing any of the method's arithmetic.

Band storage convention used throughout (the LAPACK "lower" band form):
``ab`` has shape (b+1, n) and ``ab[d, j] = B[j+d, j]`` for 0 <= d <= b,
entries with j+d >= n are zero.  The diagonal ``ab[0]`` is real.  B is real
symmetric (float64) or complex Hermitian (complex128).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "band_matrix",
    "hermitian_perturbation",
    "rhs_block",
    "rhs_columns",
    "planner_matrix",
    "scf_matrix",
    "scf_targets",
    "Config",
    "CONFIGS",
]


def band_matrix(n: int, b: int, seed: int, complex_: bool,
                lo: float, hi: float) -> np.ndarray:
    """Diagonal = linspace(lo, hi, n) + N(0,1); sub-diagonal k = N(0, 1/b).

    Draw order from ``numpy.random.default_rng(seed)`` (PCG64):
    the n diagonal noise values, then for k = 1..b the n-k values of
    sub-diagonal k (complex: the real array, then the imaginary array, each
    scaled by sqrt(1/(2b)) so that E|x|^2 = 1/b; real: scaled by sqrt(1/b)).
    """
    if not (0 <= b < n):
        raise ValueError("need 0 <= b < n")
    rng = np.random.default_rng(seed)
    dt = np.complex128 if complex_ else np.float64
    ab = np.zeros((b + 1, n), dtype=dt)
    ab[0] = np.linspace(lo, hi, n) + rng.standard_normal(n)
    for k in range(1, b + 1):
        if complex_:
            s = math.sqrt(1.0 / (2 * b))
            re = rng.standard_normal(n - k)
            im = rng.standard_normal(n - k)
            ab[k, : n - k] = (re + 1j * im) * s
        else:
            ab[k, : n - k] = rng.standard_normal(n - k) * math.sqrt(1.0 / b)
    return ab


def hermitian_perturbation(n: int, b: int, seed: int, complex_: bool) -> np.ndarray:
    """A band perturbation E of the same band: diag N(0,1), off-diagonals N(0,1/b)."""
    return band_matrix(n, b, seed, complex_, 0.0, 0.0)


_RHS_CHUNK = 64


def rhs_columns(n: int, cols, seed: int, complex_: bool) -> np.ndarray:
    """Columns ``cols`` of the seeded start block Y (shape (n, len(cols)), F-order).

    Columns are drawn in chunks of 64: chunk c comes from
    ``default_rng([seed + 100, c])`` as a (64, n) array of N(0,1) values
    (complex: real array then imaginary array, divided by sqrt(2)), and
    column j is row j % 64 of chunk j // 64.  Any subset of columns can
    therefore be regenerated without drawing the whole block.
    """
    cols = np.asarray(cols, dtype=np.int64)
    dt = np.complex128 if complex_ else np.float64
    out = np.empty((n, len(cols)), dtype=dt, order="F")
    cache: dict[int, np.ndarray] = {}
    for i, j in enumerate(cols):
        c = int(j) // _RHS_CHUNK
        if c not in cache:
            rng = np.random.default_rng([seed + 100, c])
            re = rng.standard_normal((_RHS_CHUNK, n))
            if complex_:
                im = rng.standard_normal((_RHS_CHUNK, n))
                cache[c] = (re + 1j * im) / math.sqrt(2.0)
            else:
                cache[c] = re
        out[:, i] = cache[c][int(j) % _RHS_CHUNK]
    return out


def rhs_block(n: int, m: int, seed: int, complex_: bool, col0: int = 0) -> np.ndarray:
    """Columns col0 .. col0+m-1 of the seeded start block (see ``rhs_columns``)."""
    return rhs_columns(n, np.arange(col0, col0 + m), seed, complex_)


def planner_matrix(i: int, scale: int = 1):
    """Training/validation matrix i of the planner set (seed 4000 + i).

    n = 256 * U{16..128} // scale (scale > 1 gives the same family at a
    fraction of the size, for quick tests), b = U{16..128} (clipped below n),
    real or complex
    with probability 1/2, diagonal drawn from one of three families:
    uniform U(-50, 50); a Gaussian mixture of 2..8 clusters; uniform with two
    gaps.  Off-diagonals N(0, 1/b) as in ``band_matrix``.
    Returns (ab, meta dict).
    """
    rng = np.random.default_rng(4000 + i)
    n = 256 * int(rng.integers(16, 129)) // scale
    b = int(rng.integers(16, 129))
    b = min(b, n - 1)
    complex_ = bool(rng.integers(0, 2))
    family = int(rng.integers(0, 3))
    if family == 0:
        diag = rng.uniform(-50.0, 50.0, n)
    elif family == 1:
        k = int(rng.integers(2, 9))
        centers = rng.uniform(-45.0, 45.0, k)
        widths = rng.uniform(0.5, 6.0, k)
        which = rng.integers(0, k, n)
        diag = centers[which] + widths[which] * rng.standard_normal(n)
    else:
        g = np.sort(rng.uniform(-40.0, 40.0, 2))
        gw = rng.uniform(2.0, 10.0, 2)
        diag = rng.uniform(-50.0, 50.0, n)
        for c, w in zip(g, gw):
            inside = np.abs(diag - c) < w / 2
            diag[inside] = np.where(diag[inside] < c, c - w / 2, c + w / 2)
    diag = np.sort(diag)
    seed2 = int(rng.integers(0, 2**31 - 1))
    ab = band_matrix(n, b, seed2, complex_, 0.0, 0.0)
    # keep the N(0,1/b) off-diagonals, replace the diagonal by the family draw
    ab[0] = diag
    meta = {"n": n, "b": b, "complex": complex_, "family": family}
    return ab, meta


@dataclass(frozen=True)
class Config:
    """A named synthetic workload (band matrix recipe plus slicing)."""
    name: str
    n: int
    b: int
    complex_: bool
    seed: int
    lo: float
    hi: float
    slices: tuple            # tuple of (lo, hi) slice bounds, or () if planned
    description: str

    def matrix(self) -> np.ndarray:
        return band_matrix(self.n, self.b, self.seed, self.complex_, self.lo, self.hi)


def _equal_width(lo, hi, k):
    edges = np.linspace(lo, hi, k + 1)
    return tuple((float(edges[i]), float(edges[i + 1])) for i in range(k))


CONFIGS = {
    "real-n2048-b32": Config(
        "real-n2048-b32", 2048, 32, False, 1, -10.0, 10.0, ((-1.0, 1.0),),
        "real symmetric band n=2048 b=32, one slice [-1,1], 8-node half contour"),
    "cplx-n16384-b64": Config(
        "cplx-n16384-b64", 16384, 64, True, 2, -50.0, 50.0, _equal_width(-50.0, 50.0, 16),
        "complex Hermitian band n=16384 b=64, 16 equal-width slices on [-50,50] x 8 nodes"),
    "cplx-n32768-b64-seq": Config(
        "cplx-n32768-b64-seq", 32768, 64, True, 3, -50.0, 50.0, (),
        "SCF-like sequence B_k = B_0 + 1e-3 E_k, n=32768 b=64, uneven slices"),
    "cplx-n65536-b128": Config(
        "cplx-n65536-b128", 65536, 128, True, 5, -50.0, 50.0, (),
        "complex Hermitian band n=65536 b=128, lowest 25600 eigenvalues in 64 slices"),
}


def scf_matrix(cfg: "Config", k: int) -> np.ndarray:
    """Matrix k of the SCF-like sequence: B_0 = cfg.matrix(), and for k >= 1
    B_k = B_0 + 1e-3 E_k with E_k a band perturbation of the same band
    (seed 3000 + k, diagonal N(0,1), off-diagonals N(0, 1/b))."""
    ab = cfg.matrix()
    if k > 0:
        ab = ab + 1e-3 * hermitian_perturbation(cfg.n, cfg.b, 3000 + k, cfg.complex_)
    return ab


def scf_targets(K: int = 32, seed: int = 303) -> np.ndarray:
    """Uneven slice counts of the sequence workload: U{43..341} (seed 303)."""
    return np.random.default_rng(seed).integers(43, 342, K)


def rhs_block_device(n: int, m: int, seed: int, complex_: bool, device="cuda"):
    """A seeded N(0,1) start block generated on the device with torch's
    Philox generator (real, or (N + iN)/sqrt(2) complex), column-major (n, m).
    Used where the block is too large to draw on the host; values differ from
    ``rhs_block`` for the same seed."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed + 100)
    if complex_:
        re = torch.randn((m, n), generator=g, device=device, dtype=torch.float64)
        im = torch.randn((m, n), generator=g, device=device, dtype=torch.float64)
        out = torch.complex(re, im) / math.sqrt(2.0)
        del re, im
    else:
        out = torch.randn((m, n), generator=g, device=device, dtype=torch.float64)
    return out.t()
