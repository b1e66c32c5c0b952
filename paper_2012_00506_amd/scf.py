"""A sequence of related band matrices solved slice by slice, each FEAST run
started from the previous matrix's Ritz vectors (the warm start of the
self-consistent-field use in Section 3, Algorithm alg:PDESHEP, where the
eigenvectors of the previous SCF step seed the next one).

The slice boundaries are placed once (on the first matrix) and re-certified
on every later matrix by exact inertia: a boundary that comes within
cert_delta ||B||_1 of an eigenvalue of the new matrix is moved to the first
certified point of s + 2 delta k, k = 1, -1, 2, -2, ...  The counts of every
matrix are exact (two inertias per slice), and the search-space size of a
slice follows them (m0 = max(ceil(1.5 m), m + 10)); a warm start block is cut
or filled with fresh random columns to that size.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import api


def m0_rule(m: int) -> int:
    return max(math.ceil(1.5 * m), m + 10)


def certify(B, bounds, cert_delta=1e-8, max_tries=64):
    """Certified copies of the boundaries on B and n_-(s) at each (one batched
    inertia launch per try round)."""
    B = api._as_band(B)
    _, g = api.cheb_moments(B, K=0, P=1)
    delta = cert_delta * g[2]
    base = np.asarray(bounds, np.float64)
    out = base.copy()
    neg = np.zeros(len(base), np.int64)
    open_ = np.ones(len(base), bool)
    tries = np.zeros(len(base), np.int64)
    for _ in range(max_tries + 1):
        idx = np.nonzero(open_)[0]
        if len(idx) == 0:
            return out, neg
        k = np.where(tries[idx] == 0, 0.0,
                     np.where(tries[idx] % 2 == 1, (tries[idx] + 1) // 2, -(tries[idx] // 2)))
        c = base[idx] + 2.0 * delta * k
        sh = np.empty(2 * len(idx))
        sh[0::2] = c - delta
        sh[1::2] = c + delta
        n_, _, _ = api.band_inertia(B, sh)
        ok = n_[0::2] == n_[1::2]
        out[idx[ok]] = c[ok]
        neg[idx[ok]] = n_[0::2][ok]
        open_[idx[ok]] = False
        tries[idx[~ok]] += 1
    raise RuntimeError("a boundary could not be certified")


@dataclass
class StepResult:
    step: int
    seconds: float
    iters: list
    info: list
    counts: list
    m0: list
    max_resid: float
    results: list = field(repr=False, default_factory=list)


class SliceSequence:
    """FEAST on fixed slices of a sequence of matrices with warm starts."""

    def __init__(self, bounds, precision=1, warm=True, seed=0, **feast_kw):
        self.bounds = np.asarray(bounds, np.float64)
        self.precision = precision
        self.warm = warm
        self.feast_kw = feast_kw
        self.prev = None
        self.gen = torch.Generator(device="cuda")
        self.gen.manual_seed(seed)
        self.step_no = 0

    def _random(self, n, m, complex_):
        if complex_:
            re = torch.randn((m, n), generator=self.gen, device="cuda", dtype=torch.float64)
            im = torch.randn((m, n), generator=self.gen, device="cuda", dtype=torch.float64)
            return (torch.complex(re, im) / math.sqrt(2.0)).t()
        return torch.randn((m, n), generator=self.gen, device="cuda", dtype=torch.float64).t()

    def _start(self, i, n, m0, complex_):
        if not self.warm or self.prev is None:
            return self._random(n, m0, complex_)
        y = self.prev[i]
        if y.shape[1] >= m0:
            return y[:, :m0]
        extra = self._random(n, m0 - y.shape[1], complex_)
        return torch.cat([y, extra], dim=1)

    def step(self, B) -> StepResult:
        B = api._as_band(B)
        t0 = time.perf_counter()
        bounds, neg = certify(B, self.bounds)
        self.bounds = bounds
        counts = np.diff(neg)
        m0 = [m0_rule(int(c)) for c in counts]
        Y = []
        for i, m in enumerate(m0):
            y = self._start(i, B.n, m, B.complex_)
            Y.append(y.contiguous().t().contiguous().t())  # column-major copy
        res = api.feast_band_slice(B, bounds[:-1], bounds[1:], Y, m_expected=counts,
                                   precision=self.precision, **self.feast_kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        self.prev = [r.Y for r in res]
        self.step_no += 1
        mr = max((float(r.resid[:r.m_found].max()) for r in res if r.m_found), default=0.0)
        return StepResult(self.step_no, dt, [r.iters for r in res], [r.info for r in res],
                          [int(c) for c in counts], m0, mr, res)
