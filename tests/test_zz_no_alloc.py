"""band_inertia_noalloc (the entry point for callers that cannot allocate):
through the C ABI, its counts equal band_inertia's bit for bit and the
oracle's, on two calls in a row, the second with a smaller problem."""
import ctypes as C
import sys

import numpy as np
import pytest

import synth
from oracle import inertia as oinertia

pytestmark = pytest.mark.gpu


def _counts_noalloc(B, shifts):
    from paper_2012_00506_amd import _native as N
    import torch
    sh = np.ascontiguousarray(np.asarray(shifts, np.float64))
    k = len(sh)
    neg, zero, pos = (np.full(k, -7, np.int32) for _ in range(3))
    bs = B.struct()
    rc = N.lib().band_inertia_noalloc(C.byref(bs), k, sh.ctypes.data_as(N.PD),
                                      neg.ctypes.data_as(N.PI32), zero.ctypes.data_as(N.PI32),
                                      pos.ctypes.data_as(N.PI32),
                                      C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, N.lib().fb_strerror(rc)
    return neg, zero, pos


@pytest.mark.parametrize("order", ["large_then_small"])
def test_noalloc_matches_band_inertia_twice(order):
    import torch
    import paper_2012_00506_amd as fb
    cases = [(6000, 48, True, 11, 37), (700, 5, False, 12, 9)]
    for n, b, cplx, seed, ns in cases:
        print(f"noalloc case n={n} b={b} cplx={cplx} seed={seed} shifts={ns}", flush=True)
        ab = synth.band_matrix(n, b, seed, cplx, -30, 30)
        B = fb.DeviceBand.from_band(ab)
        rng = np.random.default_rng(seed)
        shifts = np.sort(rng.uniform(-40, 40, ns))
        got = _counts_noalloc(B, shifts)
        torch.cuda.synchronize()
        ref = fb.band_inertia(B, shifts)
        for g, r in zip(got, ref):
            assert np.array_equal(g, r)
        assert np.all(got[0] + got[1] + got[2] == n)
        # the oracle at a few shifts (FP64 band LDL^H, same count rule)
        for s in shifts[:: max(1, ns // 4)]:
            assert int(oinertia.inertia(ab, float(s))[0]) == int(got[0][list(shifts).index(s)])
