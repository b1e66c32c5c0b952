"""GPU parity of the inertia counts and the shifted band solves against the
CPU oracle, through the C ABI.

Tolerances:
* inertia counts: bit-exact at shifts farther than 1e-8 ||B||_1 from every
  eigenvalue (both sides are FP64 LDL^H; they may differ only within
  rounding distance of an eigenvalue);
* complex128 solves: both are backward-stable band LU solves, so
  ||x_gpu - x_oracle|| / ||x|| <= kappa * O(n eps); with kappa <~ 1e3 here,
  1e-11 is used, and the GPU residual ||y - A x|| / ||y|| <= 1e-13;
* complex64 + FP64 refinement: residual <= ir_tol per column, so
  ||x_gpu - x_oracle|| / ||x|| <= kappa * ir_tol (kappa <~ 1e3).
"""
import math

import numpy as np
import pytest

import synth
from oracle import band as oband
from oracle import bandlu as olu
from oracle import inertia as oin
from oracle import quadrature as oq

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2012_00506_amd as fb
    return fb


def certified_shifts(ab, k, seed):
    ev = np.linalg.eigvalsh(oband.dense_from_band(ab)) if ab.shape[1] <= 1500 else None
    lo, hi = oband.gershgorin(ab)
    rng = np.random.default_rng(seed)
    out = []
    delta = 1e-8 * oband.norm1(ab)
    while len(out) < k:
        s = rng.uniform(lo - 1, hi + 1)
        if ev is not None and np.min(np.abs(ev - s)) <= delta:
            continue
        out.append(s)
    return np.array(out)


@pytest.mark.parametrize("n,b,cplx", [(300, 7, True), (257, 16, False), (97, 64, True),
                                      (130, 128, True), (40, 0, False), (1, 0, True),
                                      (150, 33, False), (200, 90, True)])
def test_inertia_parity(fb, n, b, cplx):
    print(f"inertia n={n} b={b} cplx={cplx}", flush=True)
    ab = synth.band_matrix(n, b, 100 + n, cplx, -10, 10)
    shifts = certified_shifts(ab, 9, n)
    neg, zero, pos = fb.band_inertia(ab, shifts)
    for i, s in enumerate(shifts):
        ref = oin.inertia(ab, s)
        assert (neg[i], zero[i], pos[i]) == ref, (s, (neg[i], zero[i], pos[i]), ref)


def test_inertia_many_shifts_cfg1(fb):
    cfg = synth.CONFIGS["real-n2048-b32"]
    ab = cfg.matrix()
    shifts = np.array([-1.0, 1.0, -12.5, 0.0, 7.25, 13.5])
    neg, _, _ = fb.band_inertia(ab, shifts)
    ref = [oin.inertia(ab, s)[0] for s in shifts]
    assert list(neg) == ref
    assert neg[1] - neg[0] == 202


def _solve_case(fb, n, b, cplx, m, precision, z=None, seed=0, want_h=True, ab=None):
    if ab is None:
        ab = synth.band_matrix(n, b, 200 + n + b, cplx, -10, 10)
    if z is None:
        z, _ = oq.contour(-1.0, 1.0, 8)
        z = z[[0, 3, 7]]
    Yh = synth.rhs_block(n, m, seed + 7, True)
    Y = fb.to_colmajor(Yh)
    r = fb.band_shifted_solve(ab, z, [Y] * len(z), want_h=want_h, precision=precision,
                              ir_tol=1e-12, ir_max=6)
    torch.cuda.synchronize()
    return ab, z, Yh, r


def _check_against_oracle(ab, z, Yh, r, tol_x, tol_res, want_h=True, cols=None):
    cols = np.arange(Yh.shape[1]) if cols is None else cols
    for s, zs in enumerate(z):
        F = olu.shifted_band_lu(ab, zs)
        Xr = olu.lu_solve(F, Yh[:, cols])
        Xg = r.X[s].cpu().numpy()[:, cols]
        err = np.linalg.norm(Xg - Xr, axis=0) / np.linalg.norm(Xr, axis=0)
        assert err.max() <= tol_x, (s, err.max())
        res = olu.shifted_residual(ab, zs, Xg, Yh[:, cols])
        assert res.max() <= tol_res, (s, res.max())
        if want_h:
            XHr = olu.lu_solve_h(F, Yh[:, cols])
            XHg = r.XH[s].cpu().numpy()[:, cols]
            err = np.linalg.norm(XHg - XHr, axis=0) / np.linalg.norm(XHr, axis=0)
            assert err.max() <= tol_x, ("H", s, err.max())
            res = olu.shifted_residual(ab, zs, XHg, Yh[:, cols], herm=True)
            assert res.max() <= tol_res, ("H", s, res.max())


CASES = [(1000, 16, True, 70), (700, 64, True, 40), (50, 40, False, 33), (40, 0, True, 5),
         (333, 1, False, 17), (400, 128, True, 20), (129, 64, False, 1),
         # every other block size of the factor blocks (32, 80, 96, 112 rows)
         (300, 30, True, 24), (350, 70, False, 19), (410, 90, True, 21), (460, 100, True, 18)]


@pytest.mark.parametrize("n,b,cplx,m", CASES)
def test_solve_fp64_parity(fb, n, b, cplx, m):
    print(f"solve fp64 n={n} b={b} cplx={cplx} m={m}", flush=True)
    ab, z, Yh, r = _solve_case(fb, n, b, cplx, m, 0)
    assert r.status == 0
    assert r.resid.max() <= 1e-13
    _check_against_oracle(ab, z, Yh, r, 1e-11, 1e-13)


@pytest.mark.parametrize("n,b,cplx,m", CASES)
def test_solve_fp32_refined_parity(fb, n, b, cplx, m):
    print(f"solve c64+IR n={n} b={b} cplx={cplx} m={m}", flush=True)
    ab, z, Yh, r = _solve_case(fb, n, b, cplx, m, 1)
    assert r.status == 0, r.resid
    assert r.resid.max() <= 1e-12
    assert r.passes.max() >= 1
    _check_against_oracle(ab, z, Yh, r, 1e-9, 1e-12)


def test_solve_pivoting_heavy(fb):
    # weak diagonal: many row interchanges in every block
    n, b = 600, 12
    ab = synth.band_matrix(n, b, 5, True, 0.0, 0.0) * 10
    ab[0] = 0.0
    z = np.array([0.01 + 0.01j, 0.3 + 0.2j])
    F = olu.shifted_band_lu(ab, z[0])
    assert (F.ipiv != np.arange(n)).sum() > n // 4
    for prec, tx, tr in ((0, 1e-9, 1e-13), (1, 1e-7, 1e-12)):
        _, _, Yh, r = _solve_case(fb, n, b, True, 37, prec, z=z, ab=ab)
        _check_against_oracle(ab, z, Yh, r, tx, tr)


def test_solve_diagonal_closed_form(fb):
    n = 77
    d = np.linspace(-3, 3, n)
    ab = np.zeros((1, n))
    ab[0] = d
    z = np.array([0.5 + 0.25j])
    Yh = synth.rhs_block(n, 9, 3, True)
    r = fb.band_shifted_solve(ab, z, [fb.to_colmajor(Yh)], precision=0)
    assert np.allclose(r.X[0].cpu().numpy(), Yh / (z[0] - d)[:, None], rtol=1e-14, atol=0)
    assert np.allclose(r.XH[0].cpu().numpy(), Yh / np.conj(z[0] - d)[:, None], rtol=1e-14, atol=0)


def test_solve_cfg2_shape_sampled(fb):
    """Full cfg2 shape (n=16384, b=64, complex) on one node, sampled columns."""
    cfg = synth.CONFIGS["cplx-n16384-b64"]
    ab = cfg.matrix()
    lo, hi = cfg.slices[7]
    z, _ = oq.contour(lo, hi, 8)
    zs = z[[0]]
    Yh = synth.rhs_block(cfg.n, 40, cfg.seed, True)
    for prec in (0, 1):
        r = fb.band_shifted_solve(ab, zs, [fb.to_colmajor(Yh)], precision=prec, ir_tol=1e-12)
        assert r.status == 0
        assert r.resid.max() <= (1e-13 if prec == 0 else 1e-12)
        _check_against_oracle(ab, zs, Yh, r, 1e-10, 1e-12, cols=np.array([0, 17, 39]))


@pytest.mark.parametrize("b", [64, 40, 9])
@pytest.mark.parametrize("precision", [0, 1])
def test_every_solve_variant_parity(fb, precision, b, tmp_path):
    """Each block-solve variant the autotuner may pick gives oracle-parity
    solutions (ragged n and tile tails; N and H; blocks of 64, 48, 16)."""
    n, m = 700, 45
    nb = (b + 15) // 16 * 16
    rsize = 4 if precision == 1 else 8
    tol_x, tol_r = (1e-9, 1e-12) if precision else (1e-11, 1e-13)
    for v in range(10):  # 6, 7: registers for three waves per SIMD; 8, 9: streamed products
        tile = 32 if (2 <= v < 6 or v == 9) else 16
        lds = ((2 * nb * 4 + 15) // 16) * 16 + 3 * nb * (tile + 1) * 2 * rsize
        if lds > 160 * 1024 or (nb > 64 and v >= 2 and v != 8):
            continue
        path = tmp_path / f"tune{v}.json"
        path.write_text(f'{{"rsize": {rsize}, "nb": {nb}, "variant": {v}, "ms": 0}}\n')
        assert fb.tune_load(str(path)) == 1
        ab, z, Yh, r = _solve_case(fb, n, b, True, m, precision)
        assert r.status == 0
        _check_against_oracle(ab, z, Yh, r, tol_x, tol_r)


def test_autotune_picks_a_variant(fb):
    ab = synth.band_matrix(2000, 64, 9, True, -10, 10)
    for prec in (0, 1):
        v, ms = fb.autotune(ab, prec, nsys=4, m=64)
        assert 0 <= v < 10 and ms > 0
