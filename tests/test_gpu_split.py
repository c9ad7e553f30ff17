"""GPU parity of the split chain body (MI355X): one chain over several
workgroups, which sat_run takes when the residual lives in global memory and
a step scores many long rows (M times the mean row of at least 12288
entries).  Compared with the FP64 oracle (clamped and redrawn proposals, M
spread evenly and unevenly over the workgroups), and bit for bit with the
general body that a batch runs for the same chain (FP32 residual with
resyncs, FP32 and one-byte lengths).  A wait limit of zero ends the chain
with PILA_ETIMEDOUT instead of waiting."""
import os
import subprocess
import sys

import numpy as np
import pytest

from test_gpu_sat import _compare_fp64, _gpu_chain, _oracle_chain, _slice

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

LDS_BUDGET = 160 * 1024
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def P():
    import paper_1411_4622_amd as P
    P.load()
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return P


def _split_body(P, st, M):
    b = st["body"]
    return (b & 15 == P._binding.BODY_SPLIT and b & P._binding.BODY_GLOBAL_R
            and (b >> 8) & 0xff == max(2, min(16, M // 4)))


# M = 32 and 64: 8 and 16 workgroups of 4 estimates; M = 22: 5 workgroups
# of 5 or 4 estimates
@pytest.mark.parametrize("N,U,K,M", [(48, 600, 68, 32), (40, 720, 57, 22), (32, 900, 46, 64)])
def test_split_fp64_matches_oracle(P, N, U, K, M):
    assert U * K * 8 > LDS_BUDGET
    sl = _slice(N, U, K, seed=N + U, masked=True, I0=1e4)
    prm = P.SatParams(n_steps=2000, seed=5, chain_id=M, n_stages=40, m_cand=M, T0=None,
                      q_auto=50, delta_max=0.05)
    print("fp64 split N=%d U=%d K=%d M=%d" % (N, U, K, M), flush=True)
    g = _gpu_chain(P, sl, "f64", prm)
    assert _split_body(P, g[1], M), g[1]["body"]
    assert g[1]["accepts_nonzero"] > 100
    _compare_fp64(g, _oracle_chain(sl, prm))


def test_split_redraw_fp64_matches_oracle(P):
    N, U, K, M = 40, 720, 57, 24
    sl = _slice(N, U, K, seed=3, masked=True, I0=1e4)
    prm = P.SatParams(n_steps=2000, seed=11, chain_id=1, n_stages=30, m_cand=M, T0=None,
                      q_auto=40, delta_max=0.2, proposal="redraw", schedule="exp")
    print("fp64 split redraw N=%d U=%d M=%d" % (N, U, M), flush=True)
    g = _gpu_chain(P, sl, "f64", prm)
    assert _split_body(P, g[1], M), g[1]["body"]
    _compare_fp64(g, _oracle_chain(sl, prm, schedule=prm.schedule, proposal=prm.proposal))
    moved = g[0][sl.mask != 0] != sl.f0[sl.mask != 0]
    assert moved.any() and not np.any(np.isin(g[0][sl.mask != 0][moved], [0.0, 1.0]))


@pytest.mark.parametrize("dtype", ["f32", "u8"])
def test_split_fp32_equals_batch_general_body(P, dtype):
    """FP32 residual, resyncs every 300 nonzero changes: the split chain
    (segments, grid-wide resyncs, copies refreshed) and the general body in
    a batch (resyncs inside the workgroup) give the same bits."""
    N, U, K, M = 64, 600, 91, 32
    sl = _slice(N, U, K, seed=12, masked=True, I0=1e4)
    prm = P.SatParams(n_steps=6000, seed=9, chain_id=3, m_cand=M, T0=None, q_auto=40,
                      precision="f32", resync_every=300, n_stages=30, delta_max=0.05)
    geom = P.Geometry(N, sl.angles, K, sl.mask, dtype)
    pl = P.pila_build(geom)
    sino = torch.from_numpy(sl.sino).cuda()
    print("fp32 split vs batch %s N=%d U=%d M=%d" % (dtype, N, U, M), flush=True)
    img_a = torch.from_numpy(sl.f0.copy()).cuda()
    st_a, _ = P.sat_run(pl, sino, prm, img_a)
    assert _split_body(P, st_a, M) and st_a["body"] & P._binding.BODY_SEGMENTED, st_a["body"]
    assert st_a["resyncs"] >= 2 and st_a["status"] == 0
    img_b = torch.from_numpy(sl.f0.copy()).cuda()
    st_b = P.sat_run_batch([P.Job(pl, sino, img_b, prm)], waves_per_chain=16, chains_per_cu=1)
    assert st_b[0]["body"] & 15 == P._binding.BODY_GENERAL
    torch.cuda.synchronize()
    assert np.array_equal(img_a.cpu().numpy(), img_b.cpu().numpy())
    for k in ("accepts", "accepts_nonzero", "resyncs"):
        assert st_a[k] == st_b[0][k], k
    assert st_a["max_drift_r"] <= 1e-3


def test_split_full_size_equals_general_body(P):
    """The large-slice workload's chain (1024 x 1024, 720 angles, 1449 bins,
    M = 32, its seeds and schedule), 2000 steps with resyncs every 500
    nonzero changes: split over eight workgroups as sat_run runs it (the
    launch the benchmark times) and on one workgroup in a batch give the same
    bits; the FP32 residual stays within 1e-3 of the FP64 rebuilds."""
    import datagen
    c = datagen.CONFIGS["c4"]
    sl = datagen.config_slice("c4")
    prm = P.SatParams(n_steps=2000, seed=c["chain_seed"], chain_id=0, n_stages=c["n_stages"],
                      m_cand=c["M"], T0=None, q_auto=c["q_auto"], tn_ratio=c["tn_ratio"],
                      delta_max=c["delta_max"], precision="f32", resync_every=500)
    pl = P.pila_build(P.Geometry(sl.N, sl.angles, sl.K, sl.mask, "f32"))
    sino = torch.from_numpy(sl.sino).cuda()
    print("fp32 split full size 1024x1024 U=720 M=32", flush=True)
    img_a = torch.from_numpy(sl.f0.copy()).cuda()
    st_a, _ = P.sat_run(pl, sino, prm, img_a)
    assert _split_body(P, st_a, 32) and (st_a["body"] >> 8) & 0xff == 8, st_a["body"]
    assert st_a["resyncs"] >= 2 and st_a["status"] == 0
    img_b = torch.from_numpy(sl.f0.copy()).cuda()
    st_b = P.sat_run_batch([P.Job(pl, sino, img_b, prm)], waves_per_chain=16, chains_per_cu=1)
    assert st_b[0]["body"] & 15 == P._binding.BODY_GENERAL
    torch.cuda.synchronize()
    assert torch.equal(img_a, img_b)
    for k in ("accepts", "accepts_nonzero", "resyncs"):
        assert st_a[k] == st_b[0][k], k
    assert st_a["max_drift_r"] <= 1e-3


def test_split_wait_limit_ends_chain(P):
    """With a wait limit of zero a workgroup gives up as soon as a sum it
    needs has not arrived: the chain ends with PILA_ETIMEDOUT and every
    workgroup exits (run in a child process that sets the limit)."""
    r = subprocess.run([sys.executable, os.path.join(HERE, "split_wait_child.py")],
                       env=dict(os.environ, PILA_SPLIT_WAIT_MS="0"), capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    line = [x for x in r.stdout.splitlines() if x.startswith("status")][-1]
    status, body = (int(v) for v in line.split()[1:3])
    assert body & 15 == P._binding.BODY_SPLIT, body
    assert status == P._binding.PILA_ETIMEDOUT, line
