"""GPU parity of the paper's variants against the oracle (MI355X): the
exponential and cubic cooling schedules of section III-C, and Eq. 3 as
printed (a proposal outside the range is drawn again)."""
import numpy as np
import pytest

from test_gpu_sat import _compare_fp64, _gpu_chain, _oracle_chain, _slice

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_1411_4622_amd as P
    P.load()
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return P


def _oracle(sl, prm):
    # the oracle wrapper takes the schedule and proposal by name as well
    return _oracle_chain(sl, prm, schedule=prm.schedule, proposal=prm.proposal)


@pytest.mark.parametrize("schedule", ["exp", "cubic"])
@pytest.mark.parametrize("N,U,K,M", [(32, 45, 47, 16), (128, 120, 182, 8)])
def test_schedules_fp64_match_oracle(P, schedule, N, U, K, M):
    sl = _slice(N, U, K, seed=N + M, masked=True, I0=1e4)
    prm = P.SatParams(n_steps=12000, seed=3, chain_id=M, n_stages=60, m_cand=M, T0=None,
                      q_auto=50, delta_max=0.05, schedule=schedule)
    print("fp64 schedule %s N=%d" % (schedule, N), flush=True)
    g = _gpu_chain(P, sl, "f64", prm)
    assert g[1]["body"] & 15 == P._binding.BODY_PIPED
    _compare_fp64(g, _oracle(sl, prm))


@pytest.mark.parametrize("N,U,K,M,schedule", [(24, 30, 35, 4, "linear"), (64, 180, 91, 8, "exp")])
def test_redraw_fp64_matches_oracle(P, N, U, K, M, schedule):
    sl = _slice(N, U, K, seed=2 * N, masked=True, I0=1e4)
    prm = P.SatParams(n_steps=6000, seed=11, chain_id=1, n_stages=30, m_cand=M, T0=None,
                      q_auto=40, delta_max=0.2, proposal="redraw", schedule=schedule)
    print("fp64 redraw N=%d" % N, flush=True)
    g = _gpu_chain(P, sl, "f64", prm)
    assert g[1]["body"] & 15 == P._binding.BODY_GENERAL
    _compare_fp64(g, _oracle(sl, prm))
    moved = g[0][sl.mask != 0] != sl.f0[sl.mask != 0]
    assert moved.any() and not np.any(np.isin(g[0][sl.mask != 0][moved], [0.0, 1.0]))


def test_redraw_fp32_batch_equals_alone(P):
    sl = _slice(40, 36, 57, seed=9, masked=True, I0=1e4)
    prm = P.SatParams(n_steps=5000, seed=2, m_cand=8, T0=None, q_auto=30, precision="f32",
                      resync_every=256, n_stages=20, proposal="redraw", schedule="cubic")
    a = _gpu_chain(P, sl, "f32", prm, trace=False)
    geom = P.Geometry(sl.N, sl.angles, sl.K, sl.mask, "f32")
    pl = P.pila_build(geom)
    img = torch.from_numpy(sl.f0.copy()).cuda()
    st = P.sat_run_batch([P.Job(pl, torch.from_numpy(sl.sino).cuda(), img, prm)],
                         waves_per_chain=8, chains_per_cu=1)
    assert np.array_equal(img.cpu().numpy(), a[0])
    assert st[0]["accepts"] == a[1]["accepts"] and st[0]["body"] & 15 == P._binding.BODY_GENERAL
