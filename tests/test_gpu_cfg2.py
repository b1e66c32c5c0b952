"""FEAST on the whole n = 16384, b = 64 complex Hermitian workload (16 equal
slices of [-50, 50), 8 Gauss nodes, m0 = max(ceil(1.5 m), m + 10), the
benchmark's seeded start blocks), in complex64 with FP64 refinement and, for
one slice, in FP64.  At this size the checks are those that hold at any
size: the slice counts against the oracle's inertia at all 17 boundaries
(bit-exact), every returned pair inside its slice with residual <= 1e-10,
orthonormal eigenvectors, sampled residuals recomputed with the oracle's band
product, and every eigenvalue within 1e-12 ||B||_1 of an exact one by the
Kato-Temple bound ||r||^2 / gap (the gap to the next eigenvalue bounded below
by the neighbouring Ritz values and their residual intervals)."""
import math

import numpy as np
import pytest

import synth
from kt_bound import kato_temple as _kato_temple
from oracle import band as oband
from oracle import inertia as oin

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CFG = "cplx-n16384-b64"


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2012_00506_amd as fb
    cfg = synth.CONFIGS[CFG]
    ab = cfg.matrix()
    B = fb.DeviceBand.from_band(ab)
    edges = [cfg.slices[0][0]] + [s[1] for s in cfg.slices]
    neg, _, _ = fb.band_inertia(B, edges)
    print("oracle inertia at 17 boundaries", flush=True)
    neg_o = np.array([oin.inertia(ab, float(e))[0] for e in edges])
    assert np.array_equal(neg, neg_o)
    counts = np.diff(neg_o)
    return fb, cfg, ab, B, edges, counts


def _start(fb, cfg, m0, i):
    y = synth.rhs_block_device(cfg.n, m0, cfg.seed * 1000 + i, True)
    return y if y.stride(0) == 1 else y.contiguous().t().contiguous().t()


def test_cfg2_all_slices_mixed_precision(setup):
    fb, cfg, ab, B, edges, counts = setup
    nrm = oband.norm1(ab)
    m0 = [max(math.ceil(1.5 * int(c)), int(c) + 10) for c in counts]
    Y = [_start(fb, cfg, m, i) for i, m in enumerate(m0)]
    print("feast 16 slices c64 + refinement", flush=True)
    res = fb.feast_band_slice(B, edges[:-1], edges[1:], Y, precision=1, ir_tol=1e-10)
    lam_all, res_all = [], []
    rng = np.random.default_rng(4)
    for i, r in enumerate(res):
        assert r.info in (0, 3), (i, r.info, r.m_found)  # 3: complex128 fallback, a warning
        assert r.m_found == counts[i]
        assert r.iters <= 6
        lam = r.lam
        assert np.all((lam >= edges[i]) & (lam < edges[i + 1]))
        assert np.all(np.diff(lam) >= 0)
        assert r.resid[: r.m_found].max() <= 1e-10
        X = r.X
        G = X.conj().T @ X
        G -= torch.eye(r.m_found, dtype=G.dtype, device=G.device)
        assert float(G.abs().max()) <= 1e-12
        if i in (0, 7, 15):
            pick = rng.choice(r.m_found, 16, replace=False)
            Xs = X[:, pick].cpu().numpy()
            R = oband.band_matmul(ab, Xs) - Xs * lam[pick][None, :]
            got = np.linalg.norm(R, axis=0) / nrm
            assert np.allclose(got, r.resid[pick], rtol=1e-6, atol=1e-15)
        lam_all.append(lam)
        res_all.append(r.resid[: r.m_found] * nrm)
    lam_all = np.concatenate(lam_all)
    res_all = np.concatenate(res_all)
    assert len(lam_all) == counts.sum() == 16135
    kt = _kato_temple(lam_all, res_all, edges[0], edges[-1])
    print(f"max Kato-Temple bound {kt.max() / nrm:.3e} ||B||_1", flush=True)
    assert kt.max() <= 1e-12 * nrm


def test_cfg2_one_slice_fp64_agrees(setup):
    fb, cfg, ab, B, edges, counts = setup
    nrm = oband.norm1(ab)
    i = 7
    m0 = max(math.ceil(1.5 * int(counts[i])), int(counts[i]) + 10)
    out = {}
    for prec in (0, 1):
        Y = [_start(fb, cfg, m0, i)]
        print(f"feast slice {i} precision {prec}", flush=True)
        [r] = fb.feast_band_slice(B, [edges[i]], [edges[i + 1]], Y, precision=prec,
                                  ir_tol=1e-10 if prec else 1e-12)
        assert r.info in (0, 3) and r.m_found == counts[i]
        assert r.resid[: r.m_found].max() <= 1e-10
        out[prec] = r.lam
    assert np.abs(out[0] - out[1]).max() <= 1e-12 * nrm


def test_cfg2_interior_slice_zolotarev(setup):
    """Zolotarev's rational filter (8 nodes, inner fraction 0.9) on the
    interior slice [-6.25, 0) with m0 = 1.5 m: converges within the
    iterations of the Gauss rule, in both precisions, to the same eigenvalues
    (1e-12 ||B||_1).  The mixed-precision runs refine from the first
    iteration (ir_from = 0), so that the iteration counts compare the
    filters and not the coarse-start schedule, which switches on residual
    levels that the filters reach at different iterations."""
    fb, cfg, ab, B, edges, counts = setup
    nrm = oband.norm1(ab)
    i = 7
    assert (edges[i], edges[i + 1]) == (-6.25, 0.0)
    m = int(counts[i])
    m0 = max(math.ceil(1.5 * m), m + 10)
    out = {}
    for rule, ratio, prec in (("gauss", 1.0, 1), ("zolotarev", 0.9, 1), ("zolotarev", 0.9, 0)):
        Y = [_start(fb, cfg, m0, i)]
        print(f"interior slice {rule} precision {prec}", flush=True)
        [r] = fb.feast_band_slice(B, [edges[i]], [edges[i + 1]], Y, m_expected=[m],
                                  precision=prec, rule=rule, ratio=ratio,
                                  ir_tol=1e-10 if prec else 1e-12, rerun=False, ir_from=0.0)
        assert r.info in (0, 3) and r.m_found == m
        assert r.resid[:m].max() <= 1e-10
        out[(rule, prec)] = r
    g = out[("gauss", 1)]
    for key in (("zolotarev", 1), ("zolotarev", 0)):
        assert out[key].iters <= g.iters
        assert np.abs(out[key].lam - g.lam).max() <= 1e-12 * nrm
