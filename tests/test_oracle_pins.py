"""Pins of the CPU oracle against facts outside itself.

Each check compares the oracle with a closed form, a published table, a
library routine used only here, brute force on tiny inputs, or an invariant
of the mathematics, so that a dropped term, a wrong sign or conjugation, a
transposed operand or an off-by-one in a band index fails at least one test.
"""
import math
import os

import numpy as np
import pytest
from scipy.linalg import eigvals_banded, solve_banded

import synth
from oracle import band, bandlu, feast, inertia, jacobi, planner, quadrature

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_band(n, b, seed, cplx, lo=-5.0, hi=5.0):
    return synth.band_matrix(n, b, seed, cplx, lo, hi)


# ---------------------------------------------------------------- band helpers
@pytest.mark.parametrize("n,b,cplx", [(1, 0, False), (9, 3, True), (40, 7, False), (33, 32, True)])
def test_band_expand_product_norm(n, b, cplx):
    ab = rand_band(n, b, 3, cplx)
    B = band.dense_from_band(ab)
    assert np.allclose(B, B.conj().T, atol=0)
    X = synth.rhs_block(n, 5, 3, True)
    assert np.allclose(band.band_matmul(ab, X), B @ X, rtol=1e-13, atol=1e-13)
    assert math.isclose(band.norm1(ab), np.linalg.norm(B, 1), rel_tol=1e-13)
    ev = np.linalg.eigvalsh(B)
    g_lo, g_hi = band.gershgorin(ab)
    assert g_lo <= ev.min() + 1e-12 and ev.max() <= g_hi + 1e-12


# ---------------------------------------------------------------- Jacobi
@pytest.mark.parametrize("m,cplx", [(1, False), (2, True), (9, True), (40, False), (60, True)])
def test_jacobi_against_eigh(m, cplx):
    rng = np.random.default_rng(m)
    A = rng.standard_normal((m, m)) + (1j * rng.standard_normal((m, m)) if cplx else 0)
    A = 0.5 * (A + A.conj().T)
    w, V = jacobi.jacobi_eigh(A)
    assert np.allclose(w, np.linalg.eigvalsh(A), atol=1e-12 * max(1, np.abs(w).max()))
    assert np.abs(V.conj().T @ V - np.eye(m)).max() < 1e-13
    assert np.abs(A @ V - V * w).max() < 1e-12 * max(1, np.abs(w).max())


def test_jacobi_degenerate():
    A = np.diag([2.0, 2.0, 2.0, -1.0])
    A[0, 1] = A[1, 0] = 0.0
    w, V = jacobi.jacobi_eigh(A)
    assert np.allclose(w, [-1, 2, 2, 2])
    Q = np.linalg.qr(np.random.default_rng(0).standard_normal((5, 5)))[0]
    A = Q @ np.diag([1.0, 1.0, 3.0, 3.0, 3.0]) @ Q.T
    w, V = jacobi.jacobi_eigh(A)
    assert np.allclose(w, [1, 1, 3, 3, 3], atol=1e-13)


# ---------------------------------------------------------------- quadrature
def test_gauss_legendre_golden_table():
    ref = np.loadtxt(os.path.join(GOLDEN, "gauss_legendre_8.txt"))
    x, w = quadrature.gauss_legendre(8)
    assert np.allclose(x, ref[:, 0], atol=2e-15)
    assert np.allclose(w, ref[:, 1], atol=2e-15)


@pytest.mark.parametrize("k", [1, 2, 5, 8, 16])
def test_gauss_legendre_library_and_exactness(k):
    x, w = quadrature.gauss_legendre(k)
    xr, wr = np.polynomial.legendre.leggauss(k)
    assert np.allclose(x, xr, atol=1e-14) and np.allclose(w, wr, atol=1e-14)
    assert math.isclose(w.sum(), 2.0, rel_tol=1e-14)
    for deg in range(2 * k):
        exact = 0.0 if deg % 2 else 2.0 / (deg + 1)
        assert abs(np.sum(w * x ** deg) - exact) < 1e-13


@pytest.mark.parametrize("lo,hi", [(-1.0, 1.0), (2.0, 8.25), (-50.0, -43.75)])
def test_filter_closed_forms(lo, hi):
    z, w = quadrature.contour(lo, hi, 8)
    c, r = 0.5 * (lo + hi), 0.5 * (hi - lo)
    assert np.all(z.imag > 0)
    assert abs(quadrature.filter_value(c, z, w) - 1.0) < 1e-14
    assert abs(quadrature.filter_value(c + r, z, w) - 0.5) < 1e-14
    assert abs(quadrature.filter_value(c - r, z, w) - 0.5) < 1e-14
    t = np.linspace(0, 3 * r, 17)
    assert np.allclose(quadrature.filter_value(c + t, z, w), quadrature.filter_value(c - t, z, w),
                       atol=1e-14)
    # a filter: close to 1 deep inside, small far outside
    assert abs(quadrature.filter_value(c + 0.5 * r, z, w) - 1.0) < 1e-4
    assert abs(quadrature.filter_value(c + 2.0 * r, z, w)) < 1e-4


# ---------------------------------------------------------------- inertia
def test_inertia_diagonal():
    d = np.array([-3.0, 1.5, 0.25, 7.0, -0.5, 2.0])
    ab = np.zeros((3, 6))
    ab[0] = d
    for s in [-4, -1, 0.0, 0.3, 1.5, 10]:
        neg, zero, pos = inertia.inertia(ab, s)
        assert neg == int((d < s).sum()) and zero == int((d == s).sum())
        assert neg + zero + pos == 6


def test_inertia_toeplitz_closed_form():
    n, a, c = 57, 0.3, -1.1 + 0.4j
    ab = np.zeros((2, n), dtype=complex)
    ab[0] = a
    ab[1, : n - 1] = c
    lam = a + 2 * abs(c) * np.cos(np.arange(1, n + 1) * np.pi / (n + 1))
    for s in np.linspace(-2.5, 3.0, 23):
        assert inertia.inertia(ab, s)[0] == int((lam < s).sum())


@pytest.mark.parametrize("n,b,cplx", [(60, 5, True), (90, 11, False), (31, 30, True)])
def test_inertia_dense_counts_and_invariants(n, b, cplx):
    ab = rand_band(n, b, 21, cplx)
    ev = np.linalg.eigvalsh(band.dense_from_band(ab))
    g_lo, g_hi = band.gershgorin(ab)
    prev = -1
    for s in np.linspace(g_lo - 1, g_hi + 1, 41):
        if np.min(np.abs(ev - s)) < 1e-9:
            continue
        neg, zero, pos = inertia.inertia(ab, s)
        assert neg == int((ev < s).sum())
        assert neg + zero + pos == n
        assert neg >= prev
        prev = neg
    assert inertia.inertia(ab, g_lo - 1e-9)[0] == 0
    assert inertia.inertia(ab, g_hi + 1e-9)[0] == n


def test_inertia_direct_sum():
    a1 = rand_band(20, 3, 1, True)
    a2 = rand_band(25, 3, 2, True)
    ab = np.zeros((4, 45), dtype=complex)
    ab[:, :20] = a1
    ab[:, 20:] = a2
    ab[1:, 17:20] = 0.0       # no coupling between the two blocks
    a1c = ab[:, :20].copy()
    for s in [-3.0, 0.1, 2.2]:
        assert inertia.inertia(ab, s)[0] == inertia.inertia(a1c, s)[0] + inertia.inertia(a2, s)[0]


# ---------------------------------------------------------------- band LU
@pytest.mark.parametrize("n,b,cplx,z", [
    (1, 0, False, 0.4 + 0.1j), (7, 6, True, 1 + 1j), (50, 3, True, 0.3 + 0.05j),
    (67, 8, False, -2 + 0.2j), (130, 16, True, 0.1 + 0.01j), (64, 16, True, 4 + 0.5j)])
def test_band_lu_against_dense(n, b, cplx, z):
    ab = rand_band(n, b, 5 + n, cplx)
    A = z * np.eye(n) - band.dense_from_band(ab)
    Y = synth.rhs_block(n, 6, 9, True)
    F = bandlu.shifted_band_lu(ab, z)
    X = bandlu.lu_solve(F, Y)
    XH = bandlu.lu_solve_h(F, Y)
    assert np.allclose(X, np.linalg.solve(A, Y), rtol=1e-11, atol=1e-12)
    assert np.allclose(XH, np.linalg.solve(A.conj().T, Y), rtol=1e-11, atol=1e-12)
    eps = np.finfo(float).eps
    for Xs, M in ((X, A), (XH, A.conj().T)):
        be = np.linalg.norm(Y - M @ Xs, axis=0) / (np.linalg.norm(M, 2) * np.linalg.norm(Xs, axis=0))
        assert be.max() <= 10 * n * eps


def test_band_lu_pivots_happen():
    # zI - B with a weak diagonal forces row exchanges
    ab = rand_band(80, 6, 4, True, 0.0, 0.0) * 10
    ab[0] = 0.0
    F = bandlu.shifted_band_lu(ab, 0.01 + 0.01j)
    assert (F.ipiv != np.arange(80)).sum() > 10
    A = (0.01 + 0.01j) * np.eye(80) - band.dense_from_band(ab)
    Y = synth.rhs_block(80, 3, 4, True)
    assert np.allclose(bandlu.lu_solve(F, Y), np.linalg.solve(A, Y), rtol=1e-10, atol=1e-10)
    assert np.allclose(bandlu.lu_solve_h(F, Y), np.linalg.solve(A.conj().T, Y), rtol=1e-10, atol=1e-10)


def test_band_lu_diagonal_closed_form():
    d = np.linspace(-2, 2, 30)
    ab = np.zeros((4, 30))
    ab[0] = d
    z = 0.25 + 0.5j
    Y = synth.rhs_block(30, 4, 2, True)
    F = bandlu.shifted_band_lu(ab, z)
    assert np.allclose(bandlu.lu_solve(F, Y), Y / (z - d)[:, None], rtol=1e-15, atol=0)
    assert np.allclose(bandlu.lu_solve_h(F, Y), Y / np.conj(z - d)[:, None], rtol=1e-15, atol=0)


def test_band_lu_against_solve_banded_cfg1_shape():
    ab = synth.CONFIGS["real-n2048-b32"].matrix()
    z, _ = quadrature.contour(-1.0, 1.0, 8)
    n, b = ab.shape[1], 32
    Y = synth.rhs_block(n, 4, 1, False).astype(complex)
    full = np.zeros((2 * b + 1, n), dtype=complex)   # scipy (l, u) = (b, b) band of zI - B
    Bd = band.dense_from_band(ab)
    for zj in (z[0], z[7]):
        A_band = np.zeros_like(full)
        for k in range(-b, b + 1):
            dgl = np.diagonal(Bd, offset=k)
            if k >= 0:
                A_band[b - k, k:] = -dgl
            else:
                A_band[b - k, : n + k] = -dgl
        A_band[b] += zj
        ref = solve_banded((b, b), A_band, Y)
        X = bandlu.lu_solve(bandlu.shifted_band_lu(ab, zj), Y)
        assert np.allclose(X, ref, rtol=1e-11, atol=1e-12)


# ---------------------------------------------------------------- filter / FEAST
def test_filter_diagonal_closed_form():
    d = np.linspace(-3, 3, 40)
    ab = np.zeros((3, 40))
    ab[0] = d
    z, w = quadrature.contour(-1.0, 1.0, 8)
    Y = synth.rhs_block(40, 5, 3, False)
    Q = feast.filter_apply(ab, feast.factor_nodes(ab, z), w, Y)
    assert np.allclose(Q, quadrature.filter_value(d, z, w)[:, None] * Y, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("cplx", [False, True])
def test_filter_spectral_brute_force(cplx):
    n = 48
    ab = rand_band(n, 4, 8, cplx, -3, 3)
    lam, V = jacobi.jacobi_eigh(band.dense_from_band(ab))
    z, w = quadrature.contour(-1.0, 0.5, 8)
    Y = synth.rhs_block(n, 7, 8, cplx)
    Q = feast.filter_apply(ab, feast.factor_nodes(ab, z), w, Y)
    ref = V @ (quadrature.filter_value(lam, z, w)[:, None] * (V.conj().T @ Y))
    assert np.allclose(Q, ref, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("cplx", [False, True])
def test_feast_small_against_dense(cplx):
    n = 200
    ab = rand_band(n, 6, 12, cplx, -8, 8)
    lam_all = np.linalg.eigvalsh(band.dense_from_band(ab))
    lo, hi = -1.3, 2.1
    ref = lam_all[(lam_all >= lo) & (lam_all < hi)]
    m = len(ref)
    m0 = max(math.ceil(1.5 * m), m + 10)
    r = feast.feast_slice(ab, lo, hi, synth.rhs_block(n, m0, 12, cplx))
    assert r.info == 0 and r.m == m and len(r.lam) == m
    nrm = band.norm1(ab)
    assert np.abs(r.lam - ref).max() <= 1e-12 * nrm
    assert r.res.max() <= 1e-10
    assert np.abs(r.X.conj().T @ r.X - np.eye(m)).max() < 1e-12


def test_feast_full_spectrum_invariants():
    n = 60
    ab = rand_band(n, 5, 33, True, -4, 4)
    g_lo, g_hi = band.gershgorin(ab)
    B = band.dense_from_band(ab)
    r = feast.feast_slice(ab, g_lo - 0.5, g_hi + 0.5, synth.rhs_block(n, n, 33, True))
    assert r.info == 0 and len(r.lam) == n
    assert abs(r.lam.sum() - np.trace(B).real) < 1e-10
    assert abs((r.lam ** 2).sum() - np.linalg.norm(B) ** 2) < 1e-9


def test_feast_count_mismatch_flag():
    n = 120
    ab = rand_band(n, 4, 14, True, -6, 6)
    lo, hi = -2.0, 2.0
    m = inertia.count_in(ab, lo, hi)
    r = feast.feast_slice(ab, lo, hi, synth.rhs_block(n, m - 5, 14, True), max_iter=4)
    assert r.info == 2 and len(r.lam) < m


@pytest.fixture(scope="module")
def cfg1_result():
    cfg = synth.CONFIGS["real-n2048-b32"]
    ab = cfg.matrix()
    m = inertia.count_in(ab, -1.0, 1.0)
    m0 = max(math.ceil(1.5 * m), m + 10)
    return ab, feast.feast_slice(ab, -1.0, 1.0, synth.rhs_block(cfg.n, m0, cfg.seed, False))


@pytest.mark.slow
def test_feast_cfg1_against_lapack(cfg1_result):
    ab, r = cfg1_result
    ev = eigvals_banded(ab, lower=True)
    ref = ev[(ev >= -1.0) & (ev < 1.0)]
    assert r.info == 0 and r.m == 202 == len(ref)
    assert np.abs(r.lam - ref).max() <= 1e-12 * band.norm1(ab)
    assert r.res.max() <= 1e-10
    assert feast.orthogonality(r.X) < 1e-13


# ---------------------------------------------------------------- planner
def test_planner_equal_count_exact_counts():
    ab = rand_band(300, 8, 3, True, -20, 20)
    ev = np.linalg.eigvalsh(band.dense_from_band(ab))
    edges, counts, nev = planner.plan_equal_count(ab, 6, count_tol=0.05)
    assert np.all(np.diff(edges) > 0)
    for i in range(6):
        assert counts[i] == int(((ev >= edges[i]) & (ev < edges[i + 1])).sum())
    assert counts.sum() == 300
    assert np.abs(counts - 50).max() <= math.floor(0.05 * 50)
    delta = 1e-8 * band.norm1(ab)
    for e in edges:
        assert np.min(np.abs(ev - e)) > delta


def test_planner_certification_moves_boundary():
    d = np.arange(10, dtype=float)
    ab = np.zeros((2, 10))
    ab[0] = d
    edges, counts, _ = planner.plan_equal_width(ab, 3, 0.0, 9.0)
    assert np.all(np.min(np.abs(d[None, :] - edges[:, None]), axis=1) > 0)
    assert counts.sum() == int(((d >= edges[0]) & (d < edges[-1])).sum())


def test_planner_whole_spectrum_when_gershgorin_is_tight():
    # diagonal B: the Gershgorin bounds are eigenvalues (multiplicity 5); the
    # default interval must still hold all of them
    d = np.repeat(np.arange(-4.0, 4.0), 5)
    ab = np.zeros((2, d.size))
    ab[0] = d
    edges, counts, _ = planner.plan_equal_count(ab, 4, count_tol=0.0)
    assert counts.sum() == d.size
    assert list(counts) == [10, 10, 10, 10]
    assert np.all(np.min(np.abs(d[None, :] - edges[:, None]), axis=1) > 1e-8 * 4)


def test_orthonormalise_ill_conditioned_block():
    # a block whose Gram matrix spans 14 orders of magnitude, like a filtered
    # FEAST block: the result is orthonormal to rounding and spans the kept
    # directions
    rng = np.random.default_rng(5)
    n, m = 400, 60
    U, _ = np.linalg.qr(rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m)))
    W, _ = np.linalg.qr(rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))
    Q = U @ np.diag(10.0 ** -np.linspace(0, 7, m)) @ W
    Qo, k = feast.orthonormalise(Q)
    assert k == m
    assert np.abs(Qo.conj().T @ Qo - np.eye(k)).max() < 1e-13
    # same span as Q: projecting Q onto span(Qo) leaves nothing
    R = Q - Qo @ (Qo.conj().T @ Q)
    assert np.linalg.norm(R) < 1e-12 * np.linalg.norm(Q)


def test_orthonormalise_keeps_directions_below_gram_resolution():
    # singular values down to 3e-9 (Gram eigenvalues down to 1e-17, below
    # what FP64 resolves in Q^H Q): every direction is kept, the result is
    # orthonormal, and the smallest singular direction lies in its span
    rng = np.random.default_rng(11)
    n, m = 300, 40
    U, _ = np.linalg.qr(rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m)))
    W, _ = np.linalg.qr(rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))
    sv = np.concatenate([np.ones(m - 4), [1e-7, 3e-8, 1e-8, 3e-9]])
    Q = U @ np.diag(sv) @ W
    Qo, k = feast.orthonormalise(Q)
    assert k == m
    assert np.abs(Qo.conj().T @ Qo - np.eye(k)).max() < 1e-13
    for j in range(m - 4, m):
        u = U[:, j]
        assert np.linalg.norm(u - Qo @ (Qo.conj().T @ u)) < 1e-6
    # an exactly rank-deficient block: the null directions are dropped
    Z = np.concatenate([Q[:, :10], Q[:, :10] @ rng.standard_normal((10, 5))], axis=1)
    _, k2 = feast.orthonormalise(Z)
    assert k2 == 10


def test_cholqr_orthonormal_same_span_and_fallback():
    # Cholesky QR twice on the column-equilibrated block: orthonormal to
    # rounding, the same span as Q, and column order kept (the basis is
    # upper-triangular in Q: U = Q T, so the first j columns of U span the
    # first j columns of Q); a block whose equilibrated Gram matrix has a
    # pivot at or below 1e-12 is refused (the eigen passes take over)
    rng = np.random.default_rng(7)
    n, m = 500, 50
    U0, _ = np.linalg.qr(rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m)))
    W, _ = np.linalg.qr(rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))
    Q = U0 @ np.diag(10.0 ** -np.linspace(0, 5, m)) @ W
    Qo = feast.orthonormalise_cholqr(Q)
    assert Qo is not None
    assert np.abs(Qo.conj().T @ Qo - np.eye(m)).max() < 1e-14
    R = Q - Qo @ (Qo.conj().T @ Q)
    assert np.linalg.norm(R) < 1e-11 * np.linalg.norm(Q)
    T = np.linalg.lstsq(Q, Qo, rcond=None)[0]
    assert np.abs(np.tril(T, -1)).max() < 1e-6 * np.abs(T).max()
    # against Householder QR: same columns up to unit phases
    Qh, Rh = np.linalg.qr(Q)
    ph = np.diag(Qh.conj().T @ Qo)
    assert np.allclose(np.abs(ph), 1.0, atol=1e-8)
    # a column that repeats an earlier one: refused
    Z = np.concatenate([Q[:, :10], Q[:, 3:4]], axis=1)
    assert feast.orthonormalise_cholqr(Z) is None
    # a zero column: refused
    Z2 = Q[:, :5].copy()
    Z2[:, 2] = 0
    assert feast.orthonormalise_cholqr(Z2) is None


def test_rayleigh_ritz_paths_agree():
    # the Cholesky QR and eigen-decomposition paths give the same Ritz values
    # on a full-rank block (the basis differs by a unitary, the Ritz values
    # not), and Rayleigh-Ritz on an invariant subspace returns eigenvalues
    import synth
    n = 300
    ab = synth.band_matrix(n, 6, 9, True, -10, 10)
    rng = np.random.default_rng(1)
    Q = rng.standard_normal((n, 40)) + 1j * rng.standard_normal((n, 40))
    st = {}
    lam_c, X_c, k_c = feast.rayleigh_ritz(ab, Q, st)
    assert st == {"cholqr": 1} and k_c == 40
    Qe, k_e = feast.orthonormalise(Q)
    A = Qe.conj().T @ band.band_matmul(ab, Qe)
    lam_e = np.linalg.eigvalsh(0.5 * (A + A.conj().T))
    assert np.abs(lam_c - lam_e).max() < 1e-12 * band.norm1(ab)
    lam_all, V = np.linalg.eigh(band.dense_from_band(ab))
    lam_v, _, _ = feast.rayleigh_ritz(ab, V[:, 100:130] @ W30(rng))
    assert np.abs(lam_v - lam_all[100:130]).max() < 1e-12 * band.norm1(ab)


def W30(rng):
    W, _ = np.linalg.qr(rng.standard_normal((30, 30)) + 1j * rng.standard_normal((30, 30)))
    return W @ np.diag(10.0 ** -np.linspace(0, 3, 30))
