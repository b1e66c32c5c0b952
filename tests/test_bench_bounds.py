"""Host-side error bounds of bench.py's end-to-end report: the Kato-Temple
bound per Ritz pair and the bound of one run's Ritz values through a
reference run's (triangle inequality), on small hand-made spectra whose
figures follow from the definitions."""
import numpy as np

import bench


def test_kato_temple_inner_and_outer_pairs():
    lam = np.array([0.0, 1.0, 3.0, 6.0])
    r = np.array([1e-3, 1e-4, 2e-4, 1e-3])
    kt = bench.kato_temple(lam, r)
    # outermost pairs keep their residual
    assert kt[0] == 1e-3 and kt[3] == 1e-3
    # lam = 1: gaps 1 - 0 - 1e-3 and 3 - 1 - 2e-4
    assert np.isclose(kt[1], 1e-8 / (1.0 - 1e-3))
    # lam = 3: gaps 3 - 1 - 1e-4 and 6 - 3 - 1e-3
    assert np.isclose(kt[2], 4e-8 / (2.0 - 1e-4))
    # unsorted input gives the same bounds per pair
    p = np.array([2, 0, 3, 1])
    assert np.allclose(bench.kato_temple(lam[p], r[p]), kt[p])


def test_bound_via_reference_takes_the_smaller():
    lam_ref = np.array([0.0, 1.0, 3.0, 6.0])
    r_ref = np.array([1e-9, 1e-9, 1e-9, 1e-9])
    lam = lam_ref + np.array([1e-11, -2e-11, 0.0, 3e-11])
    r = np.array([1e-6, 1e-9, 1e-9, 1e-6])
    nrm = 2.0
    via = bench.bound_via_reference(lam[::-1].copy(), r[::-1].copy(), lam_ref, r_ref, nrm)
    own = bench.kato_temple(lam, r) / nrm
    ref = bench.kato_temple(lam_ref, r_ref) / nrm
    d = np.abs(lam - lam_ref) / nrm
    assert np.allclose(via, np.minimum(own, d + ref))
    # the outer pairs (residual 1e-6) are bounded through the reference
    assert via[0] < 1e-8 and via[3] < 1e-8
