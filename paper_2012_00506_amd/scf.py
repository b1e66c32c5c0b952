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

import json
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

    def __init__(self, bounds, precision=1, warm=True, seed=0, replan_nev=0, log_path=None,
                 **feast_kw):
        self.bounds = np.asarray(bounds, np.float64)
        self.K = len(self.bounds) - 1
        self.precision = precision
        self.warm = warm
        self.replan_nev = int(replan_nev)
        self.feast_kw = feast_kw
        self.log_path = log_path  # one JSON line per step when set
        self.prev = None
        self.prev_pairs = None  # (ascending eigenvalues, their vectors) of the last step
        self.gen = torch.Generator(device="cuda")
        self.gen.manual_seed(seed)
        self.step_no = 0

    # ------------------------------------------------------------ checkpoint
    def save(self, path):
        """Write the sequence state (boundaries, step number, the last step's
        start blocks, and with re-partitioning its eigenpairs, the random
        generator) to an .npz file that ``load`` reads back."""
        arrays = {"bounds": self.bounds, "step_no": np.int64(self.step_no),
                  "precision": np.int64(self.precision), "warm": np.int64(self.warm),
                  "replan_nev": np.int64(self.replan_nev),
                  "gen_state": self.gen.get_state().numpy()}
        if self.prev is not None:
            arrays["n_prev"] = np.int64(len(self.prev))
            for i, y in enumerate(self.prev):
                arrays[f"prev_{i}"] = y.cpu().numpy()
        if self.prev_pairs is not None and self.prev_pairs[1] is not None:
            arrays["pairs_lam"] = self.prev_pairs[0]
            arrays["pairs_X"] = self.prev_pairs[1].cpu().numpy()
        np.savez(path, **arrays)

    @classmethod
    def load(cls, path, **feast_kw):
        """A sequence resumed from ``save``: the next ``step`` continues
        exactly as the saved sequence would have."""
        z = np.load(path, allow_pickle=False)
        seq = cls(z["bounds"], precision=int(z["precision"]), warm=bool(z["warm"]),
                  replan_nev=int(z["replan_nev"]), **feast_kw)
        seq.step_no = int(z["step_no"])
        seq.gen.set_state(torch.from_numpy(z["gen_state"].copy()))
        if "n_prev" in z.files:
            seq.prev = [torch.from_numpy(z[f"prev_{i}"]).cuda() for i in range(int(z["n_prev"]))]
        if "pairs_lam" in z.files:
            seq.prev_pairs = (z["pairs_lam"], torch.from_numpy(z["pairs_X"]).cuda())
        return seq

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

    def _log(self, dt, counts, m0, res):
        """Append one JSON line: counts, sizes, iterations, info codes, the
        largest eigen-residual, the orthogonality max |X^H X - I| per slice,
        and per kernel class its launches, time and achieved FLOP/s."""
        prof = api.profile_read()
        api.profile_enable(False)
        orth = []
        for r in res:
            X = r.Y[:, : r.m_found]
            if r.m_found == 0:
                orth.append(0.0)
                continue
            G = X.conj().t() @ X
            G -= torch.eye(r.m_found, dtype=G.dtype, device=G.device)
            orth.append(float(G.abs().max()))
        rec = {"step": self.step_no + 1, "seconds": dt,
               "bounds": [float(v) for v in self.bounds],
               "counts": [int(c) for c in counts], "m0": [int(v) for v in m0],
               "iters": [r.iters for r in res], "info": [r.info for r in res],
               "max_resid": max((float(r.resid[:r.m_found].max()) for r in res if r.m_found),
                                default=0.0),
               "orthogonality": orth,
               "kernels": {k: {"launches": v[0], "ms": v[1],
                               "tflops": (v[2] / v[1] / 1e9) if v[1] > 0 else 0.0}
                           for k, v in prof.items() if v[0]}}
        with open(self.log_path, "a") as f:
            f.write(json.dumps(rec) + "\n")

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
        if self.log_path:
            api.profile_enable(True)
        res = api.feast_band_slice(B, self.bounds[:-1], self.bounds[1:], Y, m_expected=counts,
                                   precision=self.precision, **self.feast_kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if self.log_path:
            self._log(dt, counts, m0, res)
        self.prev = [r.Y for r in res]
        if self.replan_nev > 0:
            self.prev_pairs = self._pairs(res)
        self.step_no += 1
        mr = max((float(r.resid[:r.m_found].max()) for r in res if r.m_found), default=0.0)
        return StepResult(self.step_no, dt, [r.iters for r in res], [r.info for r in res],
                          [int(c) for c in counts], m0, mr, res)
