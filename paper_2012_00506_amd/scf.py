"""A sequence of related band matrices solved slice by slice, each FEAST run
started from the previous matrix's Ritz vectors (the warm start of the
self-consistent-field use in Section 3, Algorithm alg:PDESHEP, where the
eigenvectors of the previous SCF step seed the next one).

Fixed slices: the boundaries are placed once (on the first matrix) and
re-certified on every later matrix by exact inertia: a boundary that comes
within cert_delta ||B||_1 of an eigenvalue of the new matrix is moved to the
first certified point of s + 2 delta k, k = 1, -1, 2, -2, ...

Re-partitioned slices (``replan_nev`` > 0): from the second matrix on, the
slices for the lowest nev eigenvalues are placed from the previous matrix's
converged eigenvalues (slice_plan_prev: the k-means of Section 3.1 and the
bound searches of Section 3.2), and each new slice starts from the previous
Ritz vectors whose eigenvalues fall inside it, filled with fresh random
columns when the slice needs more start vectors and cut when it needs fewer
(the interlace and trim of Section 3.1).

The counts of every matrix are exact (two inertias per slice), and the
search-space size of a slice follows them (m0 = max(ceil(1.5 m), m + 10)).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import api


def m0_rule(m: int) -> int:
    """Subspace size of a slice of m eigenvalues (fb_m0_rule in the library)."""
    return api.m0_rule(m)


def certify(B, bounds, cert_delta=1e-8):
    """Certified copies of the boundaries on B and n_-(s) at each
    (slice_certify in the library)."""
    b, neg, _, _, _ = api.slice_certify(B, bounds, cert_delta)
    return b, neg.astype(np.int64)


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

    def __init__(self, bounds, precision=1, warm=True, seed=0, replan_nev=0, **feast_kw):
        self.bounds = np.asarray(bounds, np.float64)
        self.K = len(self.bounds) - 1
        self.precision = precision
        self.warm = warm
        self.replan_nev = int(replan_nev)
        self.feast_kw = feast_kw
        self.prev = None
        self.prev_pairs = None  # (ascending eigenvalues, their vectors) of the last step
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

    def _pairs(self, res):
        """Converged in-slice pairs of a step, ascending."""
        lam = np.concatenate([r.lam for r in res]) if res else np.zeros(0)
        if lam.size == 0:
            return lam, None
        X = torch.cat([r.Y[:, : r.m_found] for r in res if r.m_found], dim=1)
        order = np.argsort(lam, kind="stable")
        idx = torch.as_tensor(order, device=X.device)
        return lam[order], X.index_select(1, idx)

    def _start_from_pairs(self, lo, hi, m0, n, complex_):
        lam, X = self.prev_pairs
        sel = np.nonzero((lam >= lo) & (lam < hi))[0]
        if sel.size >= m0:
            sel = sel[:m0]
        y = X.index_select(1, torch.as_tensor(sel, device=X.device)) if sel.size else None
        if y is not None and y.shape[1] >= m0:
            return y
        extra = self._random(n, m0 - (0 if y is None else y.shape[1]), complex_)
        return extra if y is None else torch.cat([y, extra], dim=1)

    def step(self, B) -> StepResult:
        B = api._as_band(B)
        t0 = time.perf_counter()
        replanned = False
        if (self.replan_nev > 0 and self.prev_pairs is not None
                and self.prev_pairs[0].size >= self.replan_nev):
            bounds, counts, _ = api.slice_plan_prev(B, self.prev_pairs[0], self.replan_nev,
                                                    self.K)
            replanned = True
            m0 = [m0_rule(int(c)) for c in counts]
        else:
            bounds, _, counts, m0, _ = api.slice_certify(B, self.bounds)
            m0 = [int(v) for v in m0]
        self.bounds = np.asarray(bounds, np.float64)
        Y = []
        for i, m in enumerate(m0):
            if replanned and self.warm:
                y = self._start_from_pairs(self.bounds[i], self.bounds[i + 1], m, B.n, B.complex_)
            else:
                y = self._start(i, B.n, m, B.complex_)
            Y.append(y.contiguous().t().contiguous().t())  # column-major copy
        res = api.feast_band_slice(B, self.bounds[:-1], self.bounds[1:], Y, m_expected=counts,
                                   precision=self.precision, **self.feast_kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        self.prev = [r.Y for r in res]
        if self.replan_nev > 0:
            self.prev_pairs = self._pairs(res)
        self.step_no += 1
        mr = max((float(r.resid[:r.m_found].max()) for r in res if r.m_found), default=0.0)
        return StepResult(self.step_no, dt, [r.iters for r in res], [r.info for r in res],
                          [int(c) for c in counts], m0, mr, res)
