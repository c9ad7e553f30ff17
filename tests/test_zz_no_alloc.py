"""The allocation-free chain entry point (sat_run_static) against sat_run
through the C ABI (MI355X): the same bits on two calls in a row, the second
on a smaller input."""
import numpy as np
import pytest

from test_gpu_sat import _slice

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_1411_4622_amd as P
    P.load()
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return P


def _run_both(P, sl, prm, dtype):
    geom = P.Geometry(sl.N, sl.angles, sl.K, sl.mask, dtype)
    pl = P.pila_build(geom)
    sino = torch.from_numpy(sl.sino).cuda()
    a = torch.from_numpy(sl.f0.copy()).cuda()
    st_a, tr_a = P.sat_run(pl, sino, prm, a, trace=True)
    b = torch.from_numpy(sl.f0.copy()).cuda()
    st_b, tr_b = P.sat_run_static(pl, sino, prm, b, trace=True)
    torch.cuda.synchronize()
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    for k in ("m_star", "accept", "dC"):
        assert torch.equal(tr_a[k], tr_b[k]), k
    for k in ("accepts", "accepts_nonzero", "resyncs", "status", "body", "sse_final", "T0_used",
              "max_drift_r"):
        assert st_a[k] == st_b[k], k
    return st_b


def test_static_matches_sat_run_twice(P):
    # first call: FP32 residual in global memory (segmented, slot words in the
    # array), then a smaller FP64 chain whose residual lives in LDS
    big = _slice(192, 180, 272, seed=4, masked=True, I0=1e4)
    prm = P.SatParams(n_steps=20000, seed=3, chain_id=1, m_cand=8, T0=None, q_auto=40,
                      precision="f32", resync_every=512, n_stages=40)
    st = _run_both(P, big, prm, "f32")
    assert st["body"] & P._binding.BODY_SEGMENTED and st["resyncs"] >= 2
    small = _slice(24, 30, 35, seed=6, masked=True, I0=1e4)
    prm = P.SatParams(n_steps=4000, seed=8, chain_id=2, m_cand=4, T0=None, q_auto=30, n_stages=20)
    st = _run_both(P, small, prm, "f64")
    assert st["body"] & 0xff == P._binding.BODY_PIPED
