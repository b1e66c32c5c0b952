"""C ABI checks that need no GPU: the library loads, exports every symbol the
header declares, rejects invalid arguments before launching anything, and
answers workspace queries."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "feastband.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b(\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def L():
    from paper_2012_00506_amd import _native as N
    return N.lib()


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert "band_inertia" in names and "feast_band_slice" in names and "slice_plan" in names
    for name in names:
        assert hasattr(L, name), f"{name} declared in feastband.h but not exported"


def test_python_signatures_cover_header():
    from paper_2012_00506_amd import _native as N
    for name in declared_functions():
        assert name in N.SIGNATURES, name


def _band(n=10, b=2, dtype=2, ldab=None, ptr=1):
    from paper_2012_00506_amd import _native as N
    return N.fb_band(n, b, dtype, ldab if ldab is not None else b + 1, C.c_void_p(ptr))


@pytest.mark.parametrize("kw", [dict(n=0), dict(b=-1), dict(b=10), dict(dtype=3), dict(ldab=2),
                                dict(ptr=0), dict(n=400, b=129)])
def test_invalid_band_rejected(L, kw):
    from paper_2012_00506_amd import _native as N
    bs = _band(**kw)
    lw = C.c_size_t(0)
    sh = (C.c_double * 1)(0.0)
    neg = (C.c_int32 * 1)()
    assert L.band_inertia(C.byref(bs), 1, sh, neg, None, None, None, C.byref(lw), None) == -1


def test_inertia_argument_errors_and_query(L):
    bs = _band()
    lw = C.c_size_t(0)
    sh = (C.c_double * 2)(0.0, 1.0)
    neg = (C.c_int32 * 2)()
    assert L.band_inertia(C.byref(bs), -1, sh, neg, None, None, None, C.byref(lw), None) == -2
    assert L.band_inertia(C.byref(bs), 2, None, neg, None, None, None, C.byref(lw), None) == -3
    assert L.band_inertia(C.byref(bs), 2, sh, None, None, None, None, C.byref(lw), None) == -4
    assert L.band_inertia(C.byref(bs), 2, sh, neg, None, None, None, None, None) == -8
    assert L.band_inertia(C.byref(bs), 2, sh, neg, None, None, None, C.byref(lw), None) == 0
    assert lw.value >= (2 + 1) * 10 * 16


def test_shifted_solve_argument_errors_and_query(L):
    from paper_2012_00506_amd import _native as N
    n = 100
    bs = _band(n=n, b=4)
    z = (C.c_double * 4)(0.1, 0.2, 0.3, 0.4)
    m = (C.c_int32 * 2)(5, 7)
    Y = (C.c_void_p * 2)(1, 1)
    X = (C.c_void_p * 2)(2, 3)
    ld = (C.c_int64 * 2)(n, n)
    o = N.fb_solve_opts(0, 1e-10, 4, 0)
    lw = C.c_size_t(0)
    args = [C.byref(bs), 2, z, m, Y, ld, X, None, ld, None, None, C.byref(o), None, C.byref(lw),
            None]
    assert L.band_shifted_solve(*args) == 0 and lw.value > 0
    bad = list(args)
    bad[1] = -1
    assert L.band_shifted_solve(*bad) == -2
    bad = list(args)
    bad[3] = (C.c_int32 * 2)(-1, 3)
    assert L.band_shifted_solve(*bad) == -4
    bad = list(args)
    bad[5] = (C.c_int64 * 2)(n - 1, n)
    assert L.band_shifted_solve(*bad) == -5
    bad = list(args)
    bad[11] = C.byref(N.fb_solve_opts(2, 1e-10, 4, 0))
    assert L.band_shifted_solve(*bad) == -12
    bad = list(args)
    bad[2] = (C.c_double * 4)(float("nan"), 0, 0, 0)
    assert L.band_shifted_solve(*bad) == -3
    # residuals need their own buffers: asking for them grows the workspace
    lw1 = C.c_size_t(0)
    args1 = list(args)
    args1[9] = (C.c_double * 2)()
    args1[13] = C.byref(lw1)
    assert L.band_shifted_solve(*args1) == 0 and lw1.value > lw.value
    lw2 = C.c_size_t(0)
    args2 = list(args)
    args2[11] = C.byref(N.fb_solve_opts(1, 1e-10, 4, 0))
    args2[13] = C.byref(lw2)
    assert L.band_shifted_solve(*args2) == 0 and lw2.value > 0


def test_strerror(L):
    assert b"pivot" in L.fb_strerror(-2001)
    assert L.fb_strerror(0) == b"success"
    assert b"invalid" in L.fb_strerror(-3)


def test_slice_plan_prev_argument_errors_and_query(L):
    from paper_2012_00506_amd import _native as N
    bs = _band(n=50, b=3)
    prev = np.arange(20, dtype=np.float64)
    pp = prev.ctypes.data_as(N.PD)
    bounds = np.zeros(9)
    counts = np.zeros(8, np.int32)
    bp, cp = bounds.ctypes.data_as(N.PD), counts.ctypes.data_as(N.PI32)
    lw = C.c_size_t(0)

    def call(p=pp, n=20, o=None, b=bp, c=cp, lwp=C.byref(lw)):
        o = o or N.fb_prev_opts(8, 10, 1e-3, 6, 1e-8, 100, 1000)
        return L.slice_plan_prev(C.byref(bs), p, n, C.byref(o), b, c, None, None, None, lwp, None)

    assert call(p=None) == -2
    unsorted = prev[::-1].copy()
    assert call(p=unsorted.ctypes.data_as(N.PD)) == -2
    assert call(o=N.fb_prev_opts(0, 10, 1e-3, 6, 1e-8, 100, 1000)) == -4
    assert call(o=N.fb_prev_opts(8, 21, 1e-3, 6, 1e-8, 100, 1000)) == -4  # nev > nprev
    assert call(o=N.fb_prev_opts(8, 10, -1.0, 6, 1e-8, 100, 1000)) == -4
    assert call(b=None) == -5
    assert call(c=None) == -6
    assert call(lwp=None) == -10
    assert call() == 0 and lw.value > 0


def test_slice_certify_argument_errors_and_query(L):
    from paper_2012_00506_amd import _native as N
    bs = _band(n=50, b=3)
    bounds = np.array([-1.0, 0.0, 2.0])
    neg = np.zeros(3, np.int32)
    counts = np.zeros(2, np.int32)
    lw = C.c_size_t(0)

    def call(nb=3, b=bounds, d=1e-8, ng=neg, c=counts, lwp=C.byref(lw)):
        bp = None if b is None else b.ctypes.data_as(N.PD)
        return L.slice_certify(C.byref(bs), nb, bp, d, None if ng is None else
                               ng.ctypes.data_as(N.PI32), None if c is None else
                               c.ctypes.data_as(N.PI32), None, None, None, lwp, None)

    assert call(nb=0) == -2
    assert call(b=None) == -3
    assert call(b=np.array([0.0, -1.0, 2.0])) == -3     # not ascending
    assert call(b=np.array([0.0, np.nan, 2.0])) == -3
    assert call(d=-1.0) == -4
    assert call(ng=None) == -5
    assert call(c=None) == -6
    assert call(lwp=None) == -10
    assert call() == 0 and lw.value > 0


@pytest.mark.parametrize("m", [0, 1, 7, 19, 20, 21, 100, 1023])
def test_m0_rule(L, m):
    import math
    assert L.fb_m0_rule(m) == max(math.ceil(1.5 * m), m + 10)


def test_feast_filter_contour_options_checked(L):
    from paper_2012_00506_amd import _native as N
    n = 100
    bs = _band(n=n, b=4)
    lo = (C.c_double * 1)(-1.0)
    hi = (C.c_double * 1)(1.0)
    m = (C.c_int32 * 1)(5)
    Y = (C.c_void_p * 1)(1)
    Q = (C.c_void_p * 1)(2)
    ld = (C.c_int64 * 1)(n)
    lw = C.c_size_t(0)

    def call(rule=0, ratio=1.0, nodes=8):
        o = N.fb_feast_opts(nodes, 1e-10, 1, 0, 1e-12, 4, 1, 0.0, 0, rule, ratio)
        return L.feast_filter(C.byref(bs), 1, lo, hi, m, Y, ld, Q, ld, None, None, C.byref(o),
                              None, C.byref(lw), None)

    assert call() == 0 and lw.value > 0
    assert call(rule=1, ratio=0.3, nodes=16) == 0
    assert call(ratio=0.0) == 0          # 0 stands for the circle
    assert call(rule=2, ratio=0.9) == 0   # Zolotarev, inner fraction 0.9
    assert call(rule=2) == -12             # ratio 1 is no inner fraction
    assert call(rule=3) == -12
    assert call(ratio=-0.5) == -12
    assert call(ratio=float("inf")) == -12
    assert call(nodes=65) == -12


@pytest.mark.parametrize("rule,ratio,k", [("gauss", 1.0, 8), ("gauss", 0.4, 16),
                                          ("trapezoid", 0.6, 12), ("zolotarev", 0.9, 8),
                                          ("zolotarev", 0.95, 16), ("zolotarev", 0.6, 3),
                                          ("zolotarev", 0.5, 1), ("zolotarev", 0.99, 64)])
def test_contour_nodes_match_oracle(rule, ratio, k):
    """The library's nodes and weights (host code, no GPU) against the
    oracle's for every rule; for the Zolotarev rule this also pins the
    library's elliptic functions."""
    from oracle import quadrature as oq
    from paper_2012_00506_amd.api import contour_nodes
    lo, hi = -2.5, 4.0
    z, w = contour_nodes(lo, hi, k, rule, ratio)
    zo, wo = oq.contour(lo, hi, k, rule, ratio)
    assert np.abs(z - zo).max() <= 1e-13 * (hi - lo)
    assert np.abs(w - wo).max() <= 1e-12 * np.abs(wo).max()
    x = np.linspace(lo - 3, hi + 3, 301)
    np.testing.assert_allclose(oq.filter_value(x, z, w), oq.filter_value(x, zo, wo),
                               rtol=0, atol=1e-12)


def test_contour_argument_errors(L):
    from paper_2012_00506_amd import _native as N
    z = np.zeros(16)
    w = np.zeros(16)
    zp, wp = z.ctypes.data_as(N.PD), w.ctypes.data_as(N.PD)
    assert L.fb_contour(0.0, 1.0, 8, 2, 0.9, zp, wp) == 0
    assert L.fb_contour(float("nan"), 1.0, 8, 0, 1.0, zp, wp) == -1
    assert L.fb_contour(1.0, 1.0, 8, 0, 1.0, zp, wp) == -2
    assert L.fb_contour(0.0, 1.0, 0, 0, 1.0, zp, wp) == -3
    assert L.fb_contour(0.0, 1.0, 8, 3, 1.0, zp, wp) == -4
    assert L.fb_contour(0.0, 1.0, 8, 2, 1.0, zp, wp) == -5
    assert L.fb_contour(0.0, 1.0, 8, 2, 0.0, zp, wp) == -5
    assert L.fb_contour(0.0, 1.0, 8, 0, -1.0, zp, wp) == -5
    assert L.fb_contour(0.0, 1.0, 8, 0, 1.0, None, wp) == -6
    assert L.fb_contour(0.0, 1.0, 8, 0, 1.0, zp, None) == -7


def test_inertia_noalloc_rejects_before_launch(L):
    # argument errors and problems beyond the fixed scratch return before any
    # device work (the band pointer here is never dereferenced)
    from paper_2012_00506_amd import _native as N
    sh = (C.c_double * 2)(0.0, 1.0)
    neg = (C.c_int32 * 2)()
    bad = _band(n=0)
    assert L.band_inertia_noalloc(C.byref(bad), 2, sh, neg, None, None, None) == -1
    bs = _band()
    assert L.band_inertia_noalloc(C.byref(bs), -1, sh, neg, None, None, None) == -2
    assert L.band_inertia_noalloc(C.byref(bs), 2, None, neg, None, None, None) == -3
    assert L.band_inertia_noalloc(C.byref(bs), 2, sh, None, None, None, None) == -4
    nan = (C.c_double * 2)(0.0, float("nan"))
    assert L.band_inertia_noalloc(C.byref(bs), 2, nan, neg, None, None, None) == -3
    big = _band(n=70000, b=64)   # 73 MB band copy > 64 MiB scratch
    assert L.band_inertia_noalloc(C.byref(big), 2, sh, neg, None, None, None) == -2007
    assert b"scratch" in L.fb_strerror(-2007)


def test_tune_file_parsing(L, tmp_path):
    """fb_tune_load reads only well-formed choices and skips the rest (the
    autotuner's per-variant timing lines, truncated or out-of-range lines)."""
    p = tmp_path / "tune.jsonl"
    p.write_text('{"timed": 1, "rsize": 4, "nb": 64, "variant": 0, "ms": 1.0}\n'
                 '{"rsize": 4, "nb": 64, "variant": 3, "ms": 2.0, "n": 100, "m": 8}\n'
                 '{"rsize": 8, "nb": 48, "variant": 1}\n'
                 '{"rsize": 4, "nb": 64, "variant": 99}\n'
                 '{"rsize": 3, "nb": 64, "variant": 1}\n'
                 '{"rsize": 4, "nb": 65, "variant": 1}\n'
                 '{"rsize": 4, "nb"\n'
                 + "x" * 2000 + "\n")
    assert L.fb_tune_load(str(p).encode()) == 2
    assert L.fb_tune_load(str(tmp_path / "missing").encode()) == -1
    assert L.fb_tune_load(None) == -1
