"""GPU parity of the planner path (Chebyshev moments, features, network
forward/backward, Adam) against the oracle, and the exactness and gain of the
learned slice plan.

Tolerances:
* moments and features: both sides are FP64; the Chebyshev recurrence loses
  at most O(k^2) eps per step, so 1e-12 absolute on moments bounded by 1 and
  1e-10 on the O(1) features;
* network outputs: identical BF16 operands, FP32 (GPU) vs FP64 (oracle)
  accumulation over <= 256 terms gives ~1e-5 relative on pre-activations; a
  hidden value whose BF16 rounding flips moves by one BF16 ulp (2^-8
  relative), which happens for a small fraction of entries: 2e-3 of the
  output scale;
* gradients: the same argument, norm-wise per parameter tensor, 2e-3;
* Adam: FP32 vs FP64 arithmetic on the same gradient, 1e-6 of the step.
The trained weights themselves are not compared (stochastic training); what
is checked is that any weights, even corrupted ones, give an exact plan.
"""
import numpy as np
import pytest

import synth
from oracle import band as oband
from oracle import chebyshev as och
from oracle import inertia as oin
from oracle import mlp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2012_00506_amd as fb
    return fb


@pytest.fixture(scope="module")
def pl(fb):
    from paper_2012_00506_amd import planner
    return planner


def unpack(w):
    w = w.detach().cpu().double().numpy()
    p, o = {}, 0
    for l in range(3):
        fi, fo = mlp.SIZES[l], mlp.SIZES[l + 1]
        p[f"W{l + 1}"] = w[o:o + fi * fo].reshape(fi, fo)
        o += fi * fo
        p[f"b{l + 1}"] = w[o:o + fo]
        o += fo
    assert o == w.size
    return p


def random_weights(pl, seed):
    w = pl.init_weights(seed)
    rng = np.random.default_rng(seed + 50)
    p = unpack(w)
    off = 0
    for l in range(3):
        fi, fo = mlp.SIZES[l], mlp.SIZES[l + 1]
        off += fi * fo
        w[off:off + fo] = torch.as_tensor(rng.uniform(-0.2, 0.2, fo), dtype=torch.float32,
                                          device=w.device)
        off += fo
    return w


MATS = [(300, 7, True), (257, 16, False), (97, 64, True), (1000, 0, False), (2049, 128, True)]


@pytest.mark.parametrize("n,b,cplx", MATS)
def test_cheb_moments_parity(fb, n, b, cplx):
    print(f"moments n={n} b={b} cplx={cplx}", flush=True)
    ab = synth.band_matrix(n, b, 300 + n, cplx, -10, 10)
    mu, g = fb.cheb_moments(ab, K=16, P=20, seed=5)
    ref = och.cheb_moments(ab, 16, 20, 5)
    assert np.abs(mu - ref).max() <= 1e-12
    lo, hi = oband.gershgorin(ab)
    assert abs(g[0] - lo) <= 1e-12 * abs(lo) and abs(g[1] - hi) <= 1e-12 * abs(hi)
    assert abs(g[2] - oband.norm1(ab)) <= 1e-12 * g[2]


@pytest.mark.parametrize("n,b,cplx", MATS)
def test_features_parity(fb, n, b, cplx):
    ab = synth.band_matrix(n, b, 310 + n, cplx, -30, 20)
    f = fb.band_features(ab, seed=7)
    ref = och.planner_features(ab, seed=7)
    assert f.shape == (80,)
    err = np.abs(f - ref)
    assert err.max() <= 1e-10, (int(err.argmax()), f[err.argmax()], ref[err.argmax()])


def test_features_diagonal_cdf_exact(fb):
    # diagonal B: the moments are exact, the damped estimate follows the
    # counts up to the Jackson kernel's smoothing
    n = 4096
    ab = np.zeros((1, n))
    ab[0] = np.linspace(-5, 5, n)
    f = fb.band_features(ab, seed=0)
    assert np.allclose(f[2:18], och.planner_features(ab, seed=0)[2:18], atol=1e-12)
    assert np.abs(f[18:34]).max() <= 1e-12        # spread over probes is zero
    assert np.abs(f[34:66] - (np.arange(32) + 0.5) / 32).max() < 0.03


@pytest.mark.parametrize("batch", [1, 37, 64])
def test_mlp_forward_parity(fb, pl, batch):
    w = random_weights(pl, batch)
    rng = np.random.default_rng(batch)
    X = rng.standard_normal((batch, 80)).astype(np.float32)
    Y = fb.planner_forward(w, torch.as_tensor(X, device="cuda")).cpu().double().numpy()
    ref, _ = mlp.forward(unpack(w), X.astype(np.float64), rounding=True)
    scale = max(1.0, np.abs(ref).max())
    assert np.abs(Y - ref).max() <= 2e-3 * scale


@pytest.mark.parametrize("batch", [5, 64])
def test_mlp_gradient_parity(fb, pl, batch):
    w = random_weights(pl, 10 + batch)
    rng = np.random.default_rng(20 + batch)
    X = rng.standard_normal((batch, 80)).astype(np.float32)
    T = rng.uniform(0, 1, (batch, 64)).astype(np.float32)
    g = torch.empty(fb.planner_bytes() // 4, dtype=torch.float32, device="cuda")
    loss = fb.planner_train_step(w, None, torch.as_tensor(X, device="cuda"),
                                 torch.as_tensor(T, device="cuda"), 0.0, 0, grads=g)
    lref, gref = mlp.backward(unpack(w), X.astype(np.float64), T.astype(np.float64), rounding=True)
    assert abs(loss - lref) <= 2e-3 * lref
    gg = unpack(g)
    for k in gref:
        err = np.linalg.norm(gg[k] - gref[k]) / np.linalg.norm(gref[k])
        assert err <= 2e-3, (k, err)


def test_adam_parity(fb, pl):
    w = random_weights(pl, 3)
    rng = np.random.default_rng(3)
    X = torch.as_tensor(rng.standard_normal((16, 80)).astype(np.float32), device="cuda")
    T = torch.as_tensor(rng.uniform(0, 1, (16, 64)).astype(np.float32), device="cuda")
    nparam = fb.planner_bytes() // 4
    opt = torch.zeros(2 * nparam, dtype=torch.float32, device="cuda")
    p = unpack(w)
    state = {}
    lr = 1e-3
    for t in (1, 2):
        g = torch.empty(nparam, dtype=torch.float32, device="cuda")
        fb.planner_train_step(w, None, X, T, 0.0, 0, grads=g)   # the gradient Adam will see
        fb.planner_train_step(w, opt, X, T, lr, t)
        mlp.adam_step(p, unpack(g), state, t=t, lr=lr)
        got = unpack(w)
        for k in p:
            assert np.abs(got[k] - p[k]).max() <= 1e-6 * lr + 1e-7 * np.abs(p[k]).max(), (t, k)
        p = got                      # continue from the GPU's FP32 weights


def test_training_lowers_loss(fb, pl):
    make = lambda i: synth.planner_matrix(i, scale=16)[0]
    X, Y = pl.build_dataset(range(96), make)
    Xv, Yv = pl.build_dataset(range(96, 112), make)
    assert np.all((Y >= 0) & (Y <= 1)) and np.all(np.diff(Y, axis=1) >= 0)
    w0 = pl.init_weights(0)
    mse0 = float(np.mean((pl.predict(w0, Xv) - Yv) ** 2))
    w, hist = pl.train(X, Y, epochs=150, batch=32)
    mse = float(np.mean((pl.predict(w, Xv) - Yv) ** 2))
    print(f"train mse {hist[0]:.3e} -> {hist[-1]:.3e}; held-out {mse0:.3e} -> {mse:.3e}")
    assert hist[-1] < 0.25 * hist[0]
    assert mse < 0.25 * mse0


def _check_plan(ab, K, bounds, counts, count_tol, delta_rel=1e-8):
    nrm = oband.norm1(ab)
    delta = delta_rel * nrm
    neg = []
    for s in bounds:
        a, b_ = oin.inertia(ab, s - delta)[0], oin.inertia(ab, s + delta)[0]
        assert a == b_, ("uncertified boundary", s)
        neg.append(oin.inertia(ab, s)[0])
    assert list(np.diff(neg)) == list(counts)
    total = neg[-1] - neg[0]
    tol = int(np.floor(count_tol * total / K))
    for i in range(1, K):
        target = neg[0] + int(round(i * total / K))
        assert abs(neg[i] - target) <= tol, (i, neg[i], target, tol)


@pytest.mark.parametrize("kind", ["uniform", "random", "nan"])
def test_learned_plan_exact_whatever_the_network(fb, pl, kind):
    ab = synth.band_matrix(900, 12, 77, True, -20, 20)
    w = None if kind == "uniform" else random_weights(pl, 4)
    if kind == "nan":
        w[:] = float("nan")
    for K in (1, 7, 16):
        bounds, counts, nev = fb.slice_plan(ab, K, "learned", planner=w, count_tol=0.05, seed=1)
        assert np.all(np.diff(bounds) > 0) and nev >= 2
        _check_plan(ab, K, bounds, counts, 0.05)


def test_learned_plan_diagonal_repeated_eigenvalues(fb, pl):
    # eigenvalues of multiplicity 30 at the integers: every boundary must be
    # moved off them (certification) and counts stay exact
    d = np.repeat(np.arange(-10.0, 10.0), 30)
    ab = np.zeros((3, d.size))
    ab[0] = d
    bounds, counts, _ = fb.slice_plan(ab, 8, "learned", planner=None, count_tol=0.2)
    _check_plan(ab, 8, bounds, counts, 0.2)
    for s in bounds[1:-1]:
        assert np.min(np.abs(d - s)) > 1e-8 * oband.norm1(ab)


def test_learned_planner_gain(fb, pl):
    """Trained on part of the (scaled-down) planner family, the learned
    search needs fewer inertia evaluations than bisection on held-out
    matrices, with plans that pass the same exactness checks."""
    make = lambda i: synth.planner_matrix(i, scale=8)[0]
    X, Y = pl.build_dataset(range(240), make)
    w, _ = pl.train(X, Y, epochs=200, batch=32)
    held = [(i, make(i)) for i in range(240, 264)]
    rows = pl.gain(w, held, K_list=(16, 64))
    for K in (16, 64):
        r = [x for x in rows if x["K"] == K]
        nb = np.mean([x["bisection"] for x in r])
        nl = np.mean([x["learned"] for x in r])
        nu = np.mean([x["uniform"] for x in r])
        print(f"K={K}: inertia evaluations bisection {nb:.1f}, uniform prior {nu:.1f}, "
              f"learned {nl:.1f}")
        assert nl < nb
    i, ab = held[0]
    bounds, counts, _ = fb.slice_plan(ab, 16, "learned", planner=w, seed=i)
    _check_plan(ab, 16, bounds, counts, 0.05)


@pytest.mark.parametrize("n,b,cplx,K", [(700, 9, True, 8), (1200, 30, False, 16), (400, 3, True, 1)])
def test_slice_plan_parity(fb, n, b, cplx, K):
    """Equal width and equal count (bisection) against the oracle: the same
    boundaries, counts and number of inertia evaluations."""
    from oracle import planner as opl
    ab = synth.band_matrix(n, b, 900 + n, cplx, -15, 15)
    e, c, ne = fb.slice_plan(ab, K, "equal_count", count_tol=0.05)
    re, rc, rne = opl.plan_equal_count(ab, K, count_tol=0.05)
    assert np.array_equal(e, re) and np.array_equal(c, rc) and ne == rne
    lo, hi = oband.gershgorin(ab)
    e, c, ne = fb.slice_plan(ab, K, "equal_width", lo=lo, hi=hi)
    re, rc, rne = opl.plan_equal_width(ab, K, lo, hi)
    assert np.array_equal(e, re) and np.array_equal(c, rc) and ne == rne


@pytest.mark.parametrize("mode", ["equal_count", "learned"])
def test_slice_plan_lowest_nev(fb, pl, mode):
    """nev: [lo, hi) holds exactly the lowest nev eigenvalues (the paper's
    lowest-part convention), split into equal counts; every boundary
    certified."""
    ab = synth.band_matrix(1100, 10, 91, True, -30, 30)
    nev, K = 333, 8
    bounds, counts, _ = fb.slice_plan(ab, K, mode, nev=nev, count_tol=0.05)
    assert counts.sum() == nev
    ev = np.linalg.eigvalsh(oband.dense_from_band(ab))
    assert np.sum(ev < bounds[-1]) == nev and np.sum(ev < bounds[0]) == 0
    _check_plan(ab, K, bounds, counts, 0.05)


def test_slice_plan_given_targets(fb):
    ab = synth.band_matrix(900, 8, 92, False, -25, 25)
    targets = np.array([43, 120, 341, 60, 77])
    bounds, counts, _ = fb.slice_plan(ab, len(targets), "equal_count", targets=targets,
                                      count_tol=0.05)
    assert counts.sum() == targets.sum()
    tol = int(np.floor(0.05 * targets.sum() / len(targets)))
    cum = np.cumsum(counts)[:-1]
    assert np.all(np.abs(cum - np.cumsum(targets)[:-1]) <= tol)
    delta = 1e-8 * oband.norm1(ab)
    for s_ in bounds:
        assert oin.inertia(ab, s_ - delta)[0] == oin.inertia(ab, s_ + delta)[0]


@pytest.mark.parametrize("n,b,cplx,nev,K", [(700, 9, True, 300, 8), (1200, 30, False, 500, 16),
                                            (400, 3, True, 50, 1), (300, 4, False, 6, 9)])
def test_slice_plan_prev_parity(fb, n, b, cplx, nev, K):
    """Slices from previous eigenvalues (k-means, bound searches,
    certification) against the oracle: the same boundaries, counts, number
    of slices and number of inertia evaluations."""
    from oracle import planner as opl
    ab = synth.band_matrix(n, b, 950 + n, cplx, -15, 15)
    E = synth.hermitian_perturbation(n, b, 951 + n, cplx)
    prev = np.linalg.eigvalsh(oband.dense_from_band(ab + 3e-2 * E))
    e, c, ne = fb.slice_plan_prev(ab, prev, nev, K)
    re, rc, rk, rne = opl.plan_prev(ab, prev, nev, K)
    print(f"n={n} K'={len(c)} counts {list(c)[:6]} inertias {ne}", flush=True)
    assert len(c) == rk <= K
    assert np.array_equal(e, re) and np.array_equal(c, rc) and ne == rne
    assert c.sum() >= nev


def test_slice_certify_parity_and_moves(fb):
    """slice_certify: counts equal the oracle's inertia at the certified
    boundaries; a boundary placed exactly on an eigenvalue (diagonal B) is
    moved off it by 2 delta k, the rest stay; m0 follows fb_m0_rule."""
    n = 300
    d = np.linspace(-5.0, 5.0, n)
    ab = np.zeros((3, n), np.complex128)
    ab[0] = d
    nrm = oband.norm1(ab)
    bounds = np.array([-4.0, d[100], 0.01, d[250], 4.9])
    b2, neg, counts, m0, nin = fb.slice_certify(ab, bounds, cert_delta=1e-8)
    delta = 1e-8 * nrm
    assert b2[0] == bounds[0] and b2[2] == bounds[2] and b2[4] == bounds[4]
    for i in (1, 3):
        assert b2[i] != bounds[i] and abs(b2[i] - bounds[i]) <= 2 * delta * 32
        assert np.abs(d - b2[i]).min() > delta
    neg_o = np.array([oin.inertia(ab, float(s))[0] for s in b2])
    assert np.array_equal(neg, neg_o)
    assert np.array_equal(counts, np.diff(neg_o))
    assert [int(v) for v in m0] == [fb.m0_rule(int(c)) for c in counts]
    assert nin >= 2 * len(bounds)
    # a random Hermitian band: certified boundaries keep the oracle's counts
    ab = synth.band_matrix(700, 9, 61, True, -6, 6)
    bounds = np.linspace(-5.0, 5.0, 9)
    b2, neg, counts, _, _ = fb.slice_certify(ab, bounds)
    assert np.array_equal(neg, [oin.inertia(ab, float(s))[0] for s in b2])
