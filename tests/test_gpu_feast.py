"""GPU FEAST (feast_band_slice through the C ABI) against the CPU oracle.

Bars: eigenvalue counts bit-exact (equal to the inertia count); eigenvalues
within 1e-12 ||B||_1 of the oracle's; every returned pair has
||Bx - lx|| / ||B||_1 <= 1e-10; the converged vectors are orthonormal to
1e-12 and span the oracle's eigenvectors (|x_gpu^H x_oracle| = 1 to 1e-8 for
eigenvalues separated by more than 1e-3, the phase being free).
"""
import math

import numpy as np
import pytest
from scipy.linalg import eigvals_banded

import synth
from oracle import band as oband
from oracle import feast as ofeast
from oracle import inertia as oin

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2012_00506_amd as fb
    return fb


def m0_rule(m):
    return max(math.ceil(1.5 * m), m + 10)


def start_block(fb, n, m0, seed, cplx):
    Yh = synth.rhs_block(n, m0, seed, cplx)
    return Yh, fb.to_colmajor(Yh)


def check_slice(r, ab, lo, hi, ref_lam, ora=None):
    nrm = oband.norm1(ab)
    m = len(ref_lam)
    assert r.info == 0, (r.info, r.m_found, m)
    assert r.m_found == m
    lam = r.lam
    assert np.all(np.diff(lam) >= 0)
    assert np.abs(lam - ref_lam).max() <= 1e-12 * nrm
    assert r.resid[:m].max() <= 1e-10
    X = r.X.cpu().numpy()
    G = X.conj().T @ X
    assert np.abs(G - np.eye(m)).max() <= 1e-12
    # independent residual check with the oracle's band product
    R = oband.band_matmul(ab, X) - X * lam[None, :]
    assert (np.linalg.norm(R, axis=0) / nrm).max() <= 1e-10
    if ora is not None:
        assert np.abs(lam - ora.lam).max() <= 1e-12 * nrm
        gaps = np.diff(np.concatenate([[-np.inf], ref_lam, [np.inf]]))
        iso = np.minimum(gaps[:-1], gaps[1:]) > 1e-3
        ov = np.abs(np.sum(np.conj(X) * ora.X, axis=0))
        assert np.all(np.abs(ov[iso] - 1.0) <= 1e-8)


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("precision", [0, 1])
def test_feast_small_against_oracle(fb, cplx, precision):
    print(f"feast small cplx={cplx} precision={precision}", flush=True)
    n = 300
    ab = synth.band_matrix(n, 6, 12, cplx, -8, 8)
    lam_all = np.linalg.eigvalsh(oband.dense_from_band(ab))
    lo, hi = -1.3, 2.1
    ref = lam_all[(lam_all >= lo) & (lam_all < hi)]
    m0 = m0_rule(len(ref))
    Yh, Y = start_block(fb, n, m0, 12, cplx)
    ora = ofeast.feast_slice(ab, lo, hi, Yh)
    [r] = fb.feast_band_slice(ab, [lo], [hi], [Y], precision=precision)
    check_slice(r, ab, lo, hi, ref, ora)


@pytest.mark.parametrize("precision", [0, 1])
def test_feast_bandwidth_90(fb, precision):
    """FEAST at b = 90 (factor blocks of 96 rows, which 64-column panels do
    not divide) against the dense eigenvalues, in both precisions."""
    print(f"feast b=90 precision={precision}", flush=True)
    n = 600
    ab = synth.band_matrix(n, 90, 91, True, -10, 10)
    lam_all = np.linalg.eigvalsh(oband.dense_from_band(ab))
    lo, hi = -1.5, 1.0
    ref = lam_all[(lam_all >= lo) & (lam_all < hi)]
    _, Y = start_block(fb, n, m0_rule(len(ref)), 91, True)
    [r] = fb.feast_band_slice(ab, [lo], [hi], [Y], precision=precision)
    check_slice(r, ab, lo, hi, ref)


def test_feast_several_slices_batched_equals_unbatched(fb):
    n = 500
    ab = synth.band_matrix(n, 9, 31, True, -10, 10)
    edges = [-6.0, -3.5, -1.0, 2.5]
    lam_all = np.linalg.eigvalsh(oband.dense_from_band(ab))
    res = {}
    for batched in (True, False):
        Ys = []
        for i in range(3):
            m = oin.count_in(ab, edges[i], edges[i + 1])
            Ys.append(start_block(fb, n, m0_rule(m), 40 + i, True)[1])
        res[batched] = fb.feast_band_slice(ab, edges[:-1], edges[1:], Ys, batched=batched)
    for i in range(3):
        lo, hi = edges[i], edges[i + 1]
        ref = lam_all[(lam_all >= lo) & (lam_all < hi)]
        check_slice(res[True][i], ab, lo, hi, ref)
        # identical launches per tile: bit-identical results
        assert np.array_equal(res[True][i].evals, res[False][i].evals)
        assert torch.equal(res[True][i].Y, res[False][i].Y)


@pytest.mark.parametrize("ir_from", [0.0, 1e-4, 1.0])
def test_feast_coarse_start_iterations(fb, ir_from):
    """precision 1 with ir_from: unrefined complex64 sweeps while the slices
    are far from converged (1.0: every slice starts that way, capped at 3
    iterations), then refined ones.  The result meets the same bars as the
    refined run from the first iteration, within one more iteration."""
    print(f"feast coarse start ir_from={ir_from}", flush=True)
    n = 1500
    ab = synth.band_matrix(n, 12, 55, True, -10, 10)
    edges = [-4.0, -1.5, 1.0]
    lam_all = np.linalg.eigvalsh(oband.dense_from_band(ab))
    Ys, refs = [], []
    for i in range(2):
        ref = lam_all[(lam_all >= edges[i]) & (lam_all < edges[i + 1])]
        refs.append(ref)
        Ys.append(start_block(fb, n, m0_rule(len(ref)), 70 + i, True)[1])
    Y0 = [y.clone() for y in Ys]
    base = fb.feast_band_slice(ab, edges[:-1], edges[1:], Y0, precision=1, ir_tol=1e-10,
                               ir_from=0.0)
    res = fb.feast_band_slice(ab, edges[:-1], edges[1:], Ys, precision=1, ir_tol=1e-10,
                              ir_from=ir_from)
    for i in range(2):
        check_slice(res[i], ab, edges[i], edges[i + 1], refs[i])
        assert res[i].iters <= base[i].iters + 1
        if ir_from == 0.0:  # the same run
            assert np.array_equal(res[i].evals, base[i].evals)


def test_feast_m0_below_count_flagged(fb):
    n = 200
    ab = synth.band_matrix(n, 4, 14, True, -6, 6)
    m = oin.count_in(ab, -2.0, 2.0)
    _, Y = start_block(fb, n, m - 5, 14, True)
    [r] = fb.feast_band_slice(ab, [-2.0], [2.0], [Y], rerun=False)
    assert r.info == 5 and r.m_found == 0


def test_feast_m0_below_count_rerun_once(fb):
    """info 5 (m0 < m) triggers one rerun with ceil(1.5 m) + 10 columns, whose
    result matches the dense eigenvalues."""
    n = 200
    ab = synth.band_matrix(n, 4, 14, True, -6, 6)
    lam = np.linalg.eigvalsh(oband.dense_from_band(ab))
    ref = lam[(lam >= -2.0) & (lam < 2.0)]
    m = len(ref)
    _, Y = start_block(fb, n, m - 5, 14, True)
    [r] = fb.feast_band_slice(ab, [-2.0], [2.0], [Y])
    assert r.info == 0 and r.m_found == m
    assert r.Y.shape[1] == math.ceil(1.5 * m) + 10
    assert np.abs(r.lam - ref).max() <= 1e-12 * oband.norm1(ab)


@pytest.mark.parametrize("precision", [0, 1])
def test_feast_real_n2048_b32(fb, precision):
    """The n=2048, b=32 real workload in full: one slice [-1, 1], 202 eigenvalues."""
    cfg = synth.CONFIGS["real-n2048-b32"]
    ab = cfg.matrix()
    ev = eigvals_banded(ab, lower=True)
    ref = ev[(ev >= -1.0) & (ev < 1.0)]
    assert len(ref) == 202
    Yh, Y = start_block(fb, cfg.n, m0_rule(202), cfg.seed, False)
    [r] = fb.feast_band_slice(ab, [-1.0], [1.0], [Y], precision=precision)
    print(f"real n2048 precision={precision}: iters={r.iters} info={r.info}", flush=True)
    check_slice(r, ab, -1.0, 1.0, ref)
    assert r.iters <= 6


@pytest.mark.parametrize("cplx", [True, False])
@pytest.mark.parametrize("precision", [0, 1])
def test_filter_against_oracle_and_pair_grouping(fb, cplx, precision):
    """feast_filter: Q = r(B) Y against the oracle's node sum, and bit-identical
    Q whether the (node, direction) pairs run one, three or all per launch or
    one slice at a time (the node sum is taken in pair order in every case).
    Oracle bar: FP64 solves agree to kappa n eps (kappa ~ 1e2 here); the
    refined complex64 solves to kappa * ir_tol each, summed over 16 terms of
    size |w_j| / Im z_j <= 0.4 ||Y||: 1e-8 relative to ||Q||."""
    from oracle import bandlu as olu
    from oracle import quadrature as oq
    n, b = 700, 11
    print(f"filter cplx={cplx} precision={precision}", flush=True)
    ab = synth.band_matrix(n, b, 61, cplx, -12, 12)
    edges = [-9.0, -4.0, 0.5, 3.0]
    ms = [37, 20, 45]
    Yh = [synth.rhs_block(n, m, 70 + i, cplx) for i, m in enumerate(ms)]
    Y = [fb.to_colmajor(y) for y in Yh]
    out = {}
    for key, kw in (("all", {}), ("one", {"pairs": 1}), ("three", {"pairs": 3}),
                    ("plain", {"batched": False})):
        r = fb.feast_filter(ab, edges[:-1], edges[1:], Y, precision=precision, ir_tol=1e-12,
                            with_resid=True, **kw)
        assert r.status == 0
        out[key] = [q.cpu().numpy() for q in r.Q]
    for key in ("one", "three", "plain"):
        for i in range(3):
            assert np.array_equal(out[key][i], out["all"][i]), (key, i)
    tol = 1e-11 if precision == 0 else 1e-8
    for i in range(3):
        z, w = oq.contour(edges[i], edges[i + 1], 8)
        F = [olu.shifted_band_lu(ab, zj) for zj in z]
        Qr = ofeast.filter_apply(ab, F, w, Yh[i])
        err = np.linalg.norm(out["all"][i] - Qr) / np.linalg.norm(Qr)
        assert err <= tol, (i, err)


def test_feast_block_jacobi_sizes(fb):
    """A slice whose search space (m0 = 420) takes the multi-workgroup block
    Jacobi for both reduced eigenproblems, complex Hermitian B."""
    n, b = 3000, 12
    ab = synth.band_matrix(n, b, 77, True, -20, 20)
    ev = eigvals_banded(ab, lower=True)
    lo, hi = -3.0, 1.5
    ref = ev[(ev >= lo) & (ev < hi)]
    m0 = m0_rule(len(ref))
    assert m0 > 256
    Yh, Y = start_block(fb, n, m0, 77, True)
    [r] = fb.feast_band_slice(ab, [lo], [hi], [Y], precision=1)
    print(f"block-Jacobi slice: m={len(ref)} m0={m0} iters={r.iters} info={r.info}", flush=True)
    check_slice(r, ab, lo, hi, ref)


def test_feast_waves_equal_one_wave(fb):
    """A budget that admits one slice at a time (three waves) gives the same
    results bit for bit as all slices in one wave (the pairs per launch held
    fixed)."""
    n = 600
    ab = synth.band_matrix(n, 7, 45, True, -10, 10)
    edges = [-7.0, -4.0, -1.5, 1.0]
    ms = [m0_rule(oin.count_in(ab, edges[i], edges[i + 1])) for i in range(3)]
    res = {}
    for key, budget in (("one", 0.0), ("waves", 1.0)):
        Ys = [start_block(fb, n, ms[i], 50 + i, True)[1] for i in range(3)]
        res[key] = fb.feast_band_slice(ab, edges[:-1], edges[1:], Ys, hbm_budget=budget, pairs=2)
    for i in range(3):
        assert res["one"][i].info == 0
        assert np.array_equal(res["one"][i].evals, res["waves"][i].evals)
        assert torch.equal(res["one"][i].Y, res["waves"][i].Y)


@pytest.mark.parametrize("rule,ratio,nodes", [("gauss", 0.5, 8), ("trapezoid", 1.0, 8),
                                              ("trapezoid", 0.6, 12), ("gauss", 1.0, 16),
                                              ("zolotarev", 0.9, 8)])
def test_feast_contour_variants_against_oracle(fb, rule, ratio, nodes):
    """Other contours and rules (an ellipse through the slice ends, the
    midpoint rule, 16 nodes, the Zolotarev filter): the same bars as the
    default half circle."""
    print(f"feast contour {rule} ratio={ratio} nodes={nodes}", flush=True)
    n = 300
    ab = synth.band_matrix(n, 6, 12, True, -8, 8)
    lam_all = np.linalg.eigvalsh(oband.dense_from_band(ab))
    lo, hi = -1.3, 2.1
    ref = lam_all[(lam_all >= lo) & (lam_all < hi)]
    Yh, Y = start_block(fb, n, m0_rule(len(ref)), 13, True)
    ora = ofeast.feast_slice(ab, lo, hi, Yh, n_nodes=nodes, rule=rule, ratio=ratio)
    [r] = fb.feast_band_slice(ab, [lo], [hi], [Y], n_nodes=nodes, rule=rule, ratio=ratio)
    print(f"  iters gpu {r.iters} oracle {ora.iters}", flush=True)
    check_slice(r, ab, lo, hi, ref, ora)
    assert r.iters <= ora.iters + 1


@pytest.mark.parametrize("rule,ratio", [("trapezoid", 0.6), ("gauss", 2.0), ("zolotarev", 0.85)])
def test_filter_contour_variants_against_oracle(fb, rule, ratio):
    """feast_filter with another contour: Q against the oracle's node sum
    (FP64 solves: kappa n eps)."""
    from oracle import bandlu as olu
    from oracle import quadrature as oq
    n, b = 500, 7
    ab = synth.band_matrix(n, b, 62, True, -12, 12)
    lo, hi = -3.0, 1.5
    Yh = synth.rhs_block(n, 21, 77, True)
    r = fb.feast_filter(ab, [lo], [hi], [fb.to_colmajor(Yh)], n_nodes=10, rule=rule, ratio=ratio)
    assert r.status == 0
    z, w = oq.contour(lo, hi, 10, rule, ratio)
    F = [olu.shifted_band_lu(ab, zj) for zj in z]
    Qr = ofeast.filter_apply(ab, F, w, Yh)
    err = np.linalg.norm(r.Q[0].cpu().numpy() - Qr) / np.linalg.norm(Qr)
    assert err <= 1e-11, err


@pytest.mark.parametrize("cplx,precision", [(False, 0), (True, 1), (False, 1)])
def test_feast_zolotarev_real_and_mixed(fb, cplx, precision):
    """The Zolotarev rule on a real symmetric band (N solves only) and in the
    complex64 + FP64 refinement path: the same eigenvalues as the dense
    solver, and as the oracle run with the same filter."""
    print(f"zolotarev cplx={cplx} precision={precision}", flush=True)
    n = 400
    ab = synth.band_matrix(n, 8, 31, cplx, -6, 6)
    lam_all = np.linalg.eigvalsh(oband.dense_from_band(ab))
    lo, hi = -0.9, 1.4
    ref = lam_all[(lam_all >= lo) & (lam_all < hi)]
    Yh, Y = start_block(fb, n, m0_rule(len(ref)), 17, cplx)
    ora = ofeast.feast_slice(ab, lo, hi, Yh, n_nodes=8, rule="zolotarev", ratio=0.9)
    [r] = fb.feast_band_slice(ab, [lo], [hi], [Y], n_nodes=8, rule="zolotarev", ratio=0.9,
                              precision=precision)
    print(f"  m={len(ref)} iters gpu {r.iters} oracle {ora.iters}", flush=True)
    check_slice(r, ab, lo, hi, ref, ora)
    assert r.iters <= ora.iters + 1
