"""The filter sweep replayed from a HIP graph (feast_filter with graph = 1 on
a non-null stream) against the same sweep launched directly: identical
kernels on identical job tables, so the outputs are compared bit for bit on
every replay, with new start blocks and other stream work between replays.
A refinement forced to fail inside the graph is redone by the direct sweep
with the complex128 fallback (passes -1), again equal to the direct call."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2012_00506_amd as fb
    return fb


def _blocks(fb, n, ms, seed, cplx):
    return [fb.to_colmajor(synth.rhs_block(n, m, seed + i, cplx)) for i, m in enumerate(ms)]


@pytest.mark.parametrize("cplx,precision", [(True, 1), (True, 0), (False, 1)])
def test_graph_replays_equal_direct(fb, cplx, precision):
    n, b = 1800, 12
    ab = synth.band_matrix(n, b, 41, cplx, -6, 6)
    B = fb.DeviceBand.from_band(ab)
    lo, hi, ms = [-2.0, 0.5], [0.5, 2.5], [40, 33]
    kw = dict(precision=precision, ir_tol=1e-10, ir_max=4, with_resid=True)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = fb.FeastFilter(B, lo, hi, ms, graph=True, **kw)
        d = fb.FeastFilter(B, lo, hi, ms, graph=False, **kw)
        dt = torch.complex128 if cplx else torch.float64
        Qg = [fb.colmajor(n, m, dt) for m in ms]
        Qd = [fb.colmajor(n, m, dt) for m in ms]
        Y = _blocks(fb, n, ms, 100, cplx)   # same buffers: the graph is replayed
        for rep in range(3):
            for y, y2 in zip(Y, _blocks(fb, n, ms, 100 + 7 * rep, cplx)):
                y.copy_(y2)
            print(f"graph replay {rep} cplx={cplx} precision={precision}", flush=True)
            rg = g(Y, Qg, stream=s)
            junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64).sum()
            rd = d(Y, Qd, stream=s)
            s.synchronize()
            assert float(junk) == float(junk)
            assert rg.status == rd.status == 0
            for a, c in zip(Qg, Qd):
                assert torch.equal(a, c)
            assert np.array_equal(rg.passes, rd.passes)
            assert np.array_equal(rg.resid, rd.resid)


def test_graph_stagnation_redone_directly(fb):
    n, b = 1200, 10
    ab = synth.band_matrix(n, b, 42, True, -6, 6)
    B = fb.DeviceBand.from_band(ab)
    lo, hi, ms = [-1.0], [1.0], [30]
    kw = dict(precision=1, ir_tol=1e-300, ir_max=1, with_resid=True)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = fb.FeastFilter(B, lo, hi, ms, graph=True, **kw)
        d = fb.FeastFilter(B, lo, hi, ms, graph=False, **kw)
        Qg = [fb.colmajor(n, ms[0])]
        Qd = [fb.colmajor(n, ms[0])]
        Y = _blocks(fb, n, ms, 300, True)
        for rep in range(2):
            Y[0].copy_(_blocks(fb, n, ms, 300 + rep, True)[0])
            print(f"graph stagnation replay {rep}", flush=True)
            rg = g(Y, Qg, stream=s)
            rd = d(Y, Qd, stream=s)
            s.synchronize()
            assert rg.status == rd.status
            assert rg.passes[0] == rd.passes[0] == -1
            assert torch.equal(Qg[0], Qd[0])
            assert np.array_equal(rg.resid, rd.resid)
