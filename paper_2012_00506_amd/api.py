"""Python binding of the banded FEAST library.

Argument marshalling only: every step runs in the HIP kernels behind the C
ABI of include/feastband.h.  PyTorch supplies device memory and streams.

Conventions: a band matrix is given as its compact lower band ``ab`` of
shape (b+1, n) with ``ab[d, j] = B[j+d, j]`` (numpy or torch); it is moved to
the device in the LAPACK column-major layout the ABI takes.  Blocks of
vectors are (n, m) tensors in column-major storage (``colmajor``).
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass

import numpy as np
import torch

from . import _native as N


def _stream_handle(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def colmajor(n: int, m: int, dtype=torch.complex128, device="cuda") -> torch.Tensor:
    """Uninitialised (n, m) tensor stored column by column (leading dim n)."""
    return torch.empty((m, n), dtype=dtype, device=device).t()


def to_colmajor(a, device="cuda", dtype=None) -> torch.Tensor:
    t = torch.as_tensor(np.asarray(a)) if not isinstance(a, torch.Tensor) else a
    if dtype is not None:
        t = t.to(dtype)
    out = colmajor(t.shape[0], t.shape[1], t.dtype, device)
    out.copy_(t)
    return out


@dataclass
class DeviceBand:
    """A band Hermitian matrix resident on the device (LAPACK lower layout)."""
    n: int
    b: int
    complex_: bool
    data: torch.Tensor   # (n, b+1), row j = column j of the LAPACK array

    @classmethod
    def from_band(cls, ab, device="cuda") -> "DeviceBand":
        ab = np.asarray(ab)
        b1, n = ab.shape
        cplx = np.iscomplexobj(ab)
        host = np.ascontiguousarray(ab.T.astype(np.complex128 if cplx else np.float64))
        data = torch.from_numpy(host).to(device)
        return cls(n, b1 - 1, cplx, data)

    def struct(self) -> N.fb_band:
        return N.fb_band(self.n, self.b, N.FB_COMPLEX128 if self.complex_ else N.FB_REAL64,
                         self.b + 1, C.c_void_p(self.data.data_ptr()))


def _as_band(B) -> DeviceBand:
    return B if isinstance(B, DeviceBand) else DeviceBand.from_band(B)


def _workspace(call, lw: C.c_size_t, device) -> torch.Tensor:
    return torch.empty(max(int(lw.value), 256), dtype=torch.uint8, device=device)


def band_inertia(B, shifts, stream=None):
    """(n_neg, n_zero, n_pos) of B - s I for each shift (numpy int32 arrays)."""
    B = _as_band(B)
    sh = np.ascontiguousarray(np.asarray(shifts, dtype=np.float64).ravel())
    k = len(sh)
    neg = np.zeros(k, np.int32)
    zero = np.zeros(k, np.int32)
    pos = np.zeros(k, np.int32)
    bs = B.struct()
    lw = C.c_size_t(0)
    L = N.lib()
    pd = sh.ctypes.data_as(N.PD)
    pn, pz, pp = (a.ctypes.data_as(N.PI32) for a in (neg, zero, pos))
    N.check("band_inertia", L.band_inertia(C.byref(bs), k, pd, pn, pz, pp, None, C.byref(lw),
                                           C.c_void_p(_stream_handle(stream))))
    ws = _workspace(None, lw, B.data.device)
    lw2 = C.c_size_t(ws.numel())
    N.check("band_inertia", L.band_inertia(C.byref(bs), k, pd, pn, pz, pp,
                                           C.c_void_p(ws.data_ptr()), C.byref(lw2),
                                           C.c_void_p(_stream_handle(stream))))
    return neg, zero, pos


@dataclass
class SolveResult:
    X: list
    XH: list
    resid: np.ndarray
    passes: np.ndarray
    status: int


def band_shifted_solve(B, z, Y, want_h=True, precision=0, ir_tol=1e-10, ir_max=4,
                       resid=True, X=None, XH=None, stream=None) -> SolveResult:
    """Solve (z_s I - B) X_s = Y_s (and the conjugate-transposed systems).

    ``z``: sequence of complex shifts; ``Y``: one (n, m_s) complex128
    column-major device tensor per shift (the same tensor may be shared).
    """
    B = _as_band(B)
    z = np.asarray(z, dtype=np.complex128).ravel()
    ns = len(z)
    if len(Y) != ns:
        raise ValueError("one right-hand-side block per shift")
    zz = np.ascontiguousarray(np.stack([z.real, z.imag], axis=1).ravel())
    m = np.array([y.shape[1] for y in Y], np.int32)
    for y in Y:
        if y.dtype != torch.complex128 or y.stride(0) != 1:
            raise ValueError("Y blocks must be complex128 column-major")
    if X is None:
        X = [colmajor(B.n, int(mm), device=B.data.device) for mm in m]
    if want_h and XH is None:
        XH = [colmajor(B.n, int(mm), device=B.data.device) for mm in m]
    ldy = np.array([y.stride(1) if y.shape[1] > 1 else B.n for y in Y], np.int64)
    ldx = np.array([x.stride(1) if x.shape[1] > 1 else B.n for x in X], np.int64)
    Yp = (C.c_void_p * ns)(*[y.data_ptr() for y in Y])
    Xp = (C.c_void_p * ns)(*[x.data_ptr() for x in X])
    XHp = (C.c_void_p * ns)(*[x.data_ptr() for x in XH]) if want_h else None
    res = np.zeros(ns, np.float64)
    passes = np.zeros(ns, np.int32)
    o = N.fb_solve_opts(precision, ir_tol, ir_max, 0)
    bs = B.struct()
    L = N.lib()
    sh = C.c_void_p(_stream_handle(stream))
    args = (C.byref(bs), ns, zz.ctypes.data_as(N.PD), m.ctypes.data_as(N.PI32), Yp,
            ldy.ctypes.data_as(N.PI64), Xp, XHp, ldx.ctypes.data_as(N.PI64),
            res.ctypes.data_as(N.PD) if resid else None, passes.ctypes.data_as(N.PI32),
            C.byref(o))
    lw = C.c_size_t(0)
    N.check("band_shifted_solve", L.band_shifted_solve(*args, None, C.byref(lw), sh))
    ws = _workspace(None, lw, B.data.device)
    lw2 = C.c_size_t(ws.numel())
    rc = L.band_shifted_solve(*args, C.c_void_p(ws.data_ptr()), C.byref(lw2), sh)
    N.check("band_shifted_solve", rc, allow_positive=True)
    return SolveResult(X, XH if want_h else None, res, passes, rc)


def device_info():
    cus = C.c_int32(0)
    name = C.create_string_buffer(64)
    N.check("fb_device_info", N.lib().fb_device_info(C.byref(cus), name, 64))
    return int(cus.value), name.value.decode()


@dataclass
class SliceResult:
    lo: float
    hi: float
    m_found: int
    iters: int
    info: int
    evals: np.ndarray      # all m0 Ritz values, converged in-slice pairs first
    resid: np.ndarray      # their eigen-residuals ||Bx - lx|| / ||B||_1
    Y: torch.Tensor        # (n, m0) Ritz vectors in the same order (in/out block)

    @property
    def lam(self) -> np.ndarray:
        return self.evals[: self.m_found]

    @property
    def X(self) -> torch.Tensor:
        return self.Y[:, : self.m_found]


# quadrature rules of the contour integral (fb_feast_opts.rule)
_RULES = {"gauss": 0, "trapezoid": 1, "zolotarev": 2}


def contour_nodes(lo, hi, k=8, rule="gauss", ratio=1.0):
    """Upper-half nodes z and weights w (complex arrays of length k) of the
    filter r(x) = sum_j 2 Re[w_j / (z_j - x)] on [lo, hi); host only."""
    z = np.zeros(2 * k)
    w = np.zeros(2 * k)
    N.check("fb_contour", N.lib().fb_contour(float(lo), float(hi), int(k), _RULES[rule],
                                              float(ratio), z.ctypes.data_as(N.PD),
                                              w.ctypes.data_as(N.PD)))
    return z[0::2] + 1j * z[1::2], w[0::2] + 1j * w[1::2]


def feast_band_slice(B, lo, hi, Y, m_expected=None, n_nodes=8, tol=1e-10, max_iter=20,
                     precision=0, ir_tol=1e-12, ir_max=8, batched=True, hbm_budget=0.0,
                     pairs=0, rule="gauss", ratio=1.0, tune_cache=None, rerun=True,
                     ir_from=1e-4, stream=None):
    """FEAST on the slices [lo_i, hi_i) of B from the start blocks Y[i]
    ((n, m0_i) column-major device tensors in the dtype of B; overwritten with
    the Ritz vectors).  Returns one SliceResult per slice.

    rerun: a slice that ends with info 2 (count mismatch) or 5 (m0 < m) is
    run once more (the rerun with more start vectors of Section 3.2) from a
    new block of m0' = ceil(1.5 max(m, m_found)) + 10 columns: its Ritz
    vectors first, then seeded random columns.  That slice's SliceResult
    then refers to the new block, not to Y[i].

    ir_from (precision 1): a slice's complex64 solves skip refinement and the
    FP64 residuals while its eigen-residuals are above ir_from (at most 3
    iterations); 0 refines from the first iteration."""
    B = _as_band(B)
    lo = np.ascontiguousarray(np.asarray(lo, dtype=np.float64).ravel())
    hi = np.ascontiguousarray(np.asarray(hi, dtype=np.float64).ravel())
    ns = len(lo)
    if len(hi) != ns or len(Y) != ns:
        raise ValueError("lo, hi and Y must have one entry per slice")
    want = torch.complex128 if B.complex_ else torch.float64
    for y in Y:
        if y.dtype != want or y.stride(0) != 1:
            raise ValueError(f"start blocks must be column-major {want}")
    m0 = np.array([y.shape[1] for y in Y], np.int32)
    ldy = np.array([y.stride(1) if y.shape[1] > 1 else B.n for y in Y], np.int64)
    dev = B.data.device
    ev = [torch.empty(int(m), dtype=torch.float64, device=dev) for m in m0]
    rs = [torch.empty(int(m), dtype=torch.float64, device=dev) for m in m0]
    Yp = (C.c_void_p * ns)(*[y.data_ptr() for y in Y])
    Ep = (C.c_void_p * ns)(*[e.data_ptr() for e in ev])
    Rp = (C.c_void_p * ns)(*[r.data_ptr() for r in rs])
    mexp = None if m_expected is None else np.ascontiguousarray(np.asarray(m_expected, np.int32))
    mf = np.zeros(ns, np.int32)
    its = np.zeros(ns, np.int32)
    inf = np.zeros(ns, np.int32)
    o = N.fb_feast_opts(n_nodes, tol, max_iter, precision, ir_tol, ir_max, 1 if batched else 0,
                        float(hbm_budget), int(pairs), _RULES[rule], float(ratio),
                        None if tune_cache is None else str(tune_cache).encode(), 0,
                        float(ir_from))
    bs = B.struct()
    L = N.lib()
    sh = C.c_void_p(_stream_handle(stream))
    args = (C.byref(bs), ns, lo.ctypes.data_as(N.PD), hi.ctypes.data_as(N.PD),
            m0.ctypes.data_as(N.PI32), None if mexp is None else mexp.ctypes.data_as(N.PI32),
            Yp, ldy.ctypes.data_as(N.PI64), Ep, Rp, mf.ctypes.data_as(N.PI32),
            its.ctypes.data_as(N.PI32), inf.ctypes.data_as(N.PI32), C.byref(o))
    lw = C.c_size_t(0)
    N.check("feast_band_slice", L.feast_band_slice(*args, None, C.byref(lw), sh))
    ws = _workspace(None, lw, dev)
    lw2 = C.c_size_t(ws.numel())
    rc = L.feast_band_slice(*args, C.c_void_p(ws.data_ptr()), C.byref(lw2), sh)
    N.check("feast_band_slice", rc, allow_positive=True)
    out = []
    for i in range(ns):
        out.append(SliceResult(float(lo[i]), float(hi[i]), int(mf[i]), int(its[i]), int(inf[i]),
                               ev[i].cpu().numpy(), rs[i].cpu().numpy(), Y[i]))
    redo = [i for i in range(ns) if out[i].info in (2, 5)]
    if rerun and redo:
        if mexp is None:
            edges = np.concatenate([lo[redo], hi[redo]])
            neg, _, _ = band_inertia(B, edges, stream=stream)
            m_exact = neg[len(redo):] - neg[:len(redo)]
        else:
            m_exact = mexp[redo]
        Y2 = []
        for a, i in enumerate(redo):
            m_new = math.ceil(1.5 * max(int(m_exact[a]), out[i].m_found)) + 10
            m_new = min(m_new, B.n)
            keep = min(int(m0[i]), m_new)
            y = torch.empty((m_new, B.n), dtype=want, device=dev).t()  # column-major
            y[:, :keep] = Y[i][:, :keep]
            if m_new > keep:
                g = torch.Generator(device=dev)
                g.manual_seed(7919 * (i + 1) + m_new)
                fill = torch.randn((m_new - keep, B.n), generator=g, device=dev,
                                   dtype=torch.float64 if not B.complex_ else torch.complex128)
                y[:, keep:] = fill.t()
            Y2.append(y)
        res2 = feast_band_slice(B, lo[redo], hi[redo], Y2, m_expected=np.asarray(m_exact),
                                n_nodes=n_nodes, tol=tol, max_iter=max_iter,
                                precision=precision, ir_tol=ir_tol, ir_max=ir_max,
                                batched=batched, hbm_budget=hbm_budget, pairs=pairs, rule=rule,
                                ratio=ratio, tune_cache=tune_cache, rerun=False, ir_from=ir_from,
                                stream=stream)
        for a, i in enumerate(redo):
            out[i] = res2[a]
    return out


@dataclass
class RitzResult:
    lam: np.ndarray      # Ritz values, ascending (rank of them)
    resid: np.ndarray    # ||B x - lam x||_2 / ||B||_1
    X: torch.Tensor      # (n, m) column-major; the first rank columns are the Ritz vectors
    rank: int
    path: int            # 0 Cholesky QR twice, 1 eigen-decomposition passes


def rayleigh_ritz(B, Q, stream=None) -> list:
    """Orthonormalisation and Rayleigh-Ritz of the blocks Q[i] ((n, m_i)
    column-major device tensors in the dtype of B; not modified)."""
    B = _as_band(B)
    want = torch.complex128 if B.complex_ else torch.float64
    for q in Q:
        if q.dtype != want or q.stride(0) != 1:
            raise ValueError(f"blocks must be column-major {want}")
    ns = len(Q)
    m = np.array([q.shape[1] for q in Q], np.int32)
    ldq = np.array([q.stride(1) if q.shape[1] > 1 else B.n for q in Q], np.int64)
    dev = B.data.device
    X = [colmajor(B.n, int(mm), want, device=dev) for mm in m]
    ldx = np.array([B.n] * ns, np.int64)
    ev = [torch.empty(max(int(mm), 1), dtype=torch.float64, device=dev) for mm in m]
    rs = [torch.empty(max(int(mm), 1), dtype=torch.float64, device=dev) for mm in m]
    rank = np.zeros(ns, np.int32)
    path = np.zeros(ns, np.int32)
    Qp = (C.c_void_p * ns)(*[q.data_ptr() for q in Q])
    Xp = (C.c_void_p * ns)(*[x.data_ptr() for x in X])
    Ep = (C.c_void_p * ns)(*[e.data_ptr() for e in ev])
    Rp = (C.c_void_p * ns)(*[r.data_ptr() for r in rs])
    bs = B.struct()
    L = N.lib()
    sh = C.c_void_p(_stream_handle(stream))
    args = (C.byref(bs), ns, m.ctypes.data_as(N.PI32), Qp, ldq.ctypes.data_as(N.PI64), Xp,
            ldx.ctypes.data_as(N.PI64), Ep, Rp, rank.ctypes.data_as(N.PI32),
            path.ctypes.data_as(N.PI32))
    lw = C.c_size_t(0)
    N.check("band_rayleigh_ritz", L.band_rayleigh_ritz(*args, None, C.byref(lw), sh))
    ws = _workspace(None, lw, dev)
    lw2 = C.c_size_t(ws.numel())
    N.check("band_rayleigh_ritz", L.band_rayleigh_ritz(*args, C.c_void_p(ws.data_ptr()),
                                                       C.byref(lw2), sh))
    out = []
    for i in range(ns):
        k = int(rank[i])
        out.append(RitzResult(ev[i][:k].cpu().numpy(), rs[i][:k].cpu().numpy(), X[i], k,
                              int(path[i])))
    return out


def slice_plan(B, K, mode="equal_count", lo=float("nan"), hi=float("nan"), count_tol=0.05,
               cert_delta=1e-8, max_rounds=60, planner=None, seed=0, nev=0, targets=None,
               stream=None):
    """Slice boundaries (K+1), exact counts (K) and the number of inertia
    evaluations, by equal width, equal count (bisection) or equal count
    searched with the planner network's predicted distribution (``planner``:
    device weights tensor; None in "learned" mode = uniform prior).
    ``nev`` > 0 covers exactly the lowest nev eigenvalues above lo;
    ``targets`` gives one desired count per slice instead of equal counts."""
    B = _as_band(B)
    modes = {"equal_width": N.FB_PLAN_EQUAL_WIDTH, "equal_count": N.FB_PLAN_EQUAL_COUNT,
             "learned": N.FB_PLAN_LEARNED}
    wp = C.c_void_p(planner.data_ptr()) if planner is not None else None
    tg = None
    if targets is not None:
        tg = np.ascontiguousarray(np.asarray(targets, np.int32))
        if tg.shape != (K,):
            raise ValueError("targets needs one count per slice")
    o = N.fb_plan_opts(modes[mode], int(K), float(lo), float(hi), float(count_tol),
                       float(cert_delta), int(max_rounds), wp, int(seed), int(nev),
                       tg.ctypes.data_as(N.PI32) if tg is not None else None)
    bounds = np.zeros(K + 1, np.float64)
    counts = np.zeros(K, np.int32)
    nev = C.c_int32(0)
    bs = B.struct()
    L = N.lib()
    sh = C.c_void_p(_stream_handle(stream))
    args = (C.byref(bs), C.byref(o), bounds.ctypes.data_as(N.PD), counts.ctypes.data_as(N.PI32),
            C.byref(nev))
    lw = C.c_size_t(0)
    N.check("slice_plan", L.slice_plan(*args, None, C.byref(lw), sh))
    ws = _workspace(None, lw, B.data.device)
    lw2 = C.c_size_t(ws.numel())
    N.check("slice_plan", L.slice_plan(*args, C.c_void_p(ws.data_ptr()), C.byref(lw2), sh))
    return bounds, counts, int(nev.value)


def slice_plan_prev(B, prev, nev, K, alpha=1e-3, m1=6, cert_delta=1e-8, max_sweeps=100,
                    max_steps=1000, stream=None):
    """Slices for the lowest ``nev`` eigenvalues of B from the ascending
    eigenvalues ``prev`` of the previous matrix of a sequence: k-means
    boundaries, searched outer bounds, all certified.  Returns (bounds
    (K'+1), exact counts (K'), inertia evaluations), K' <= K."""
    B = _as_band(B)
    pv = np.ascontiguousarray(np.asarray(prev, np.float64))
    o = N.fb_prev_opts(int(K), int(nev), float(alpha), int(m1), float(cert_delta),
                       int(max_sweeps), int(max_steps))
    bounds = np.zeros(K + 1, np.float64)
    counts = np.zeros(K, np.int32)
    kout = C.c_int32(0)
    nev_ = C.c_int32(0)
    bs = B.struct()
    L = N.lib()
    sh = C.c_void_p(_stream_handle(stream))
    args = (C.byref(bs), pv.ctypes.data_as(N.PD), C.c_int64(pv.size), C.byref(o),
            bounds.ctypes.data_as(N.PD), counts.ctypes.data_as(N.PI32), C.byref(kout),
            C.byref(nev_))
    lw = C.c_size_t(0)
    N.check("slice_plan_prev", L.slice_plan_prev(*args, None, C.byref(lw), sh))
    ws = _workspace(None, lw, B.data.device)
    lw2 = C.c_size_t(ws.numel())
    N.check("slice_plan_prev", L.slice_plan_prev(*args, C.c_void_p(ws.data_ptr()), C.byref(lw2),
                                                 sh))
    k = int(kout.value)
    return bounds[:k + 1], counts[:k], int(nev_.value)


def m0_rule(m: int) -> int:
    """Subspace size for a slice of m eigenvalues (fb_m0_rule)."""
    return int(N.lib().fb_m0_rule(int(m)))


def slice_certify(B, bounds, cert_delta=1e-8, stream=None):
    """Certified copies of ``bounds`` on B (slice_certify): returns (bounds,
    n_-(bounds), exact counts, m0 per slice, inertia evaluations)."""
    B = _as_band(B)
    b = np.ascontiguousarray(np.asarray(bounds, np.float64).copy())
    nb = b.size
    neg = np.zeros(nb, np.int32)
    counts = np.zeros(max(nb - 1, 1), np.int32)
    m0 = np.zeros(max(nb - 1, 1), np.int32)
    nin = C.c_int32(0)
    bs = B.struct()
    L = N.lib()
    sh = C.c_void_p(_stream_handle(stream))
    args = (C.byref(bs), nb, b.ctypes.data_as(N.PD), float(cert_delta),
            neg.ctypes.data_as(N.PI32), counts.ctypes.data_as(N.PI32),
            m0.ctypes.data_as(N.PI32), C.byref(nin))
    lw = C.c_size_t(0)
    N.check("slice_certify", L.slice_certify(*args, None, C.byref(lw), sh))
    ws = _workspace(None, lw, B.data.device)
    lw2 = C.c_size_t(ws.numel())
    N.check("slice_certify", L.slice_certify(*args, C.c_void_p(ws.data_ptr()), C.byref(lw2), sh))
    return b, neg, counts[:nb - 1], m0[:nb - 1], int(nin.value)


@dataclass
class FilterResult:
    Q: list
    resid: np.ndarray | None
    passes: np.ndarray
    status: int


class FeastFilter:
    """Reusable filter application Q_i = r(B) Y_i over a fixed set of slices
    (workspace allocated once; each call factors and solves everything).
    graph=True replays the sweep from a HIP graph captured on the first call
    (batched, every pair in one launch, a stream other than the null one).
    workspace: a uint8 device tensor of at least workspace_bytes() bytes that
    filters run one after another may share."""

    def __init__(self, B, lo, hi, m, n_nodes=8, precision=0, ir_tol=1e-10, ir_max=4,
                 batched=True, with_resid=False, hbm_budget=0.0, pairs=0, rule="gauss",
                 ratio=1.0, graph=False, tune_cache=None, workspace=None, device="cuda"):
        self.B = _as_band(B)
        self.lo = np.ascontiguousarray(np.asarray(lo, np.float64).ravel())
        self.hi = np.ascontiguousarray(np.asarray(hi, np.float64).ravel())
        self.m = np.ascontiguousarray(np.asarray(m, np.int32).ravel())
        self.ns = len(self.lo)
        self.o = N.fb_feast_opts(n_nodes, 1e-10, 1, precision, ir_tol, ir_max,
                                 1 if batched else 0, float(hbm_budget), int(pairs),
                                 _RULES[rule], float(ratio),
                                 None if tune_cache is None else str(tune_cache).encode(),
                                 1 if graph else 0)
        self.with_resid = with_resid
        self.bs = self.B.struct()
        self.resid = np.zeros(self.ns, np.float64)
        self.passes = np.zeros(self.ns, np.int32)
        self._ws = workspace  # a uint8 device tensor shared with other filters, or None

    def _args(self, Y, Q):
        ldy = np.array([y.stride(1) if y.shape[1] > 1 else self.B.n for y in Y], np.int64)
        ldq = np.array([q.stride(1) if q.shape[1] > 1 else self.B.n for q in Q], np.int64)
        self._keep = (ldy, ldq)
        Yp = (C.c_void_p * self.ns)(*[y.data_ptr() for y in Y])
        Qp = (C.c_void_p * self.ns)(*[q.data_ptr() for q in Q])
        self._keep2 = (Yp, Qp)
        return (C.byref(self.bs), self.ns, self.lo.ctypes.data_as(N.PD),
                self.hi.ctypes.data_as(N.PD), self.m.ctypes.data_as(N.PI32), Yp,
                ldy.ctypes.data_as(N.PI64), Qp, ldq.ctypes.data_as(N.PI64),
                self.resid.ctypes.data_as(N.PD) if self.with_resid else None,
                self.passes.ctypes.data_as(N.PI32), C.byref(self.o))

    def workspace_bytes(self, Y, Q) -> int:
        lw = C.c_size_t(0)
        N.check("feast_filter", N.lib().feast_filter(*self._args(Y, Q), None, C.byref(lw), None))
        return int(lw.value)

    def __call__(self, Y, Q, stream=None) -> FilterResult:
        if self._ws is None:
            self._ws = torch.empty(max(self.workspace_bytes(Y, Q), 256), dtype=torch.uint8,
                                   device=self.B.data.device)
        if self._ws.numel() < self.workspace_bytes(Y, Q):
            raise ValueError("the filter's workspace is smaller than workspace_bytes()")
        lw = C.c_size_t(self._ws.numel())
        rc = N.lib().feast_filter(*self._args(Y, Q), C.c_void_p(self._ws.data_ptr()),
                                  C.byref(lw), C.c_void_p(_stream_handle(stream)))
        N.check("feast_filter", rc, allow_positive=True)
        return FilterResult(Q, self.resid.copy() if self.with_resid else None,
                            self.passes.copy(), rc)


def feast_filter(B, lo, hi, Y, Q=None, **kw) -> FilterResult:
    """One-shot filter application (see FeastFilter)."""
    B = _as_band(B)
    m = [y.shape[1] for y in Y]
    if Q is None:
        Q = [colmajor(B.n, mm, Y[0].dtype, B.data.device) for mm in m]
    return FeastFilter(B, lo, hi, m, **kw)(Y, Q)


def profile_enable(on: bool = True):
    N.check("fb_profile_enable", N.lib().fb_profile_enable(1 if on else 0))


def profile_read() -> dict:
    """{class: (launches, total ms, total algorithmic flops)} since enable."""
    out = {}
    for i, name in enumerate(N.PROF_CLASSES):
        L = C.c_int64(0)
        ms = C.c_double(0)
        w = C.c_double(0)
        N.check("fb_profile_read", N.lib().fb_profile_read(i, C.byref(L), C.byref(ms), C.byref(w)))
        out[name] = (int(L.value), float(ms.value), float(w.value))
    return out


def autotune(B, precision, nsys=8, m=256, cache_path=None, stream=None):
    """Time the block-solve variants on B's shape and keep the fastest for
    this precision for the rest of the process.  Returns (variant, ms)."""
    B = _as_band(B)
    bs = B.struct()
    L = N.lib()
    ch = C.c_int32(-1)
    ms = C.c_double(0)
    path = cache_path.encode() if cache_path else None
    sh = C.c_void_p(_stream_handle(stream))
    lw = C.c_size_t(0)
    N.check("fb_autotune", L.fb_autotune(C.byref(bs), precision, nsys, m, path, C.byref(ch),
                                         C.byref(ms), None, C.byref(lw), sh))
    ws = _workspace(None, lw, B.data.device)
    lw2 = C.c_size_t(ws.numel())
    N.check("fb_autotune", L.fb_autotune(C.byref(bs), precision, nsys, m, path, C.byref(ch),
                                         C.byref(ms), C.c_void_p(ws.data_ptr()), C.byref(lw2), sh))
    return int(ch.value), float(ms.value)


def tune_load(cache_path) -> int:
    return int(N.lib().fb_tune_load(cache_path.encode()))


def _query_run(name, call):
    lw = C.c_size_t(0)
    N.check(name, call(None, C.byref(lw)))
    return lw


def cheb_moments(B, K=16, P=20, seed=0, stream=None):
    """(P, K+1) Chebyshev moments and (g_lo, g_hi, ||B||_1)."""
    B = _as_band(B)
    bs = B.struct()
    mu = np.zeros(P * (K + 1))
    g = np.zeros(3)
    L = N.lib()
    sh = C.c_void_p(_stream_handle(stream))
    f = lambda w, lw: L.band_cheb_moments(C.byref(bs), K, P, seed, mu.ctypes.data_as(N.PD),
                                          g.ctypes.data_as(N.PD), w, lw, sh)
    lw = _query_run("band_cheb_moments", f)
    ws = _workspace(None, lw, B.data.device)
    lw2 = C.c_size_t(ws.numel())
    N.check("band_cheb_moments", f(C.c_void_p(ws.data_ptr()), C.byref(lw2)))
    return mu.reshape(P, K + 1), g


def band_features(B, seed=0, stream=None) -> np.ndarray:
    """The 80 planner features of B (float64)."""
    B = _as_band(B)
    bs = B.struct()
    feat = np.zeros(80)
    L = N.lib()
    sh = C.c_void_p(_stream_handle(stream))
    f = lambda w, lw: L.band_features(C.byref(bs), seed, feat.ctypes.data_as(N.PD), w, lw, sh)
    lw = _query_run("band_features", f)
    ws = _workspace(None, lw, B.data.device)
    lw2 = C.c_size_t(ws.numel())
    N.check("band_features", f(C.c_void_p(ws.data_ptr()), C.byref(lw2)))
    return feat


def planner_bytes() -> int:
    return int(N.lib().fb_planner_bytes())


def planner_forward(weights: torch.Tensor, x: torch.Tensor, stream=None) -> torch.Tensor:
    """Network outputs (batch, 64) for features x (batch, 80) float32 on the device."""
    x = x.contiguous().float()
    out = torch.empty((x.shape[0], 64), dtype=torch.float32, device=x.device)
    L = N.lib()
    sh = C.c_void_p(_stream_handle(stream))
    f = lambda w, lw: L.planner_forward(C.c_void_p(weights.data_ptr()), x.shape[0],
                                        C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()),
                                        w, lw, sh)
    lw = _query_run("planner_forward", f)
    ws = _workspace(None, lw, x.device)
    lw2 = C.c_size_t(ws.numel())
    N.check("planner_forward", f(C.c_void_p(ws.data_ptr()), C.byref(lw2)))
    return out


def planner_train_step(weights, opt_state, x, target, lr, t, grads=None, want_loss=True,
                       stream=None):
    """One Adam step (or gradients only when ``grads`` is given); returns the
    batch loss (float) when want_loss."""
    x = x.contiguous().float()
    target = target.contiguous().float()
    loss = C.c_float(0)
    L = N.lib()
    sh = C.c_void_p(_stream_handle(stream))
    gp = C.c_void_p(grads.data_ptr()) if grads is not None else None
    op = C.c_void_p(opt_state.data_ptr()) if opt_state is not None else None
    f = lambda w, lw: L.planner_train_step(C.c_void_p(weights.data_ptr()), op, x.shape[0],
                                           C.c_void_p(x.data_ptr()),
                                           C.c_void_p(target.data_ptr()), float(lr), int(t),
                                           C.byref(loss) if want_loss else None, gp, w, lw, sh)
    lw = _query_run("planner_train_step", f)
    ws = _workspace(None, lw, x.device)
    lw2 = C.c_size_t(ws.numel())
    N.check("planner_train_step", f(C.c_void_p(ws.data_ptr()), C.byref(lw2)))
    return float(loss.value) if want_loss else None
