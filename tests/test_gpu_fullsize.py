"""GPU parity on the paths the full-size workloads take (MI355X).

The residual sinograms of the batch, large-slice and serving workloads do not
fit in LDS, so their chains run the bodies' global-memory modes: the
pipelined body with part of the residual in LDS and a patch table, the
long-row body, and the general body.  Each is compared here with the FP64
oracle at a size whose residual exceeds the LDS budget (the body that ran is
asserted from the chain's statistics).  FP32 chains at such sizes must end
within 1% of the oracle's FP64 chain in RMSE against the phantom, alone
(segments with grid-wide resyncs) and batched (resyncs inside the
workgroup).  SIRT is compared where the forward projection runs in several
image bands.
"""
import numpy as np
import pytest

import datagen
import oracle
from test_gpu_sat import _compare_fp64, _gpu_chain, _oracle_chain, _slice

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

LDS_BUDGET = 160 * 1024


@pytest.fixture(scope="module")
def P():
    import paper_1411_4622_amd as P
    P.load()
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return P


def _body(P, kind):
    return kind | P._binding.BODY_GLOBAL_R


@pytest.mark.parametrize("name,N,U,K,M,steps,kind", [
    # pipelined body, rows <= 256 in registers, residual partly in LDS + patch table
    ("piped", 128, 120, 182, 8, 20000, 1),
    # long-row body: rows of more than 512 entries
    ("long", 80, 420, 114, 6, 4000, 2),
    # general body: M = 40 is above the pipelined and long-row bodies' limits
    ("general", 40, 180, 121, 40, 3000, 3),
])
def test_fp64_global_residual_bodies_match_oracle(P, name, N, U, K, M, steps, kind):
    assert U * K * 8 > LDS_BUDGET
    sl = _slice(N, U, K, seed=N + U, masked=True, I0=1e4)
    prm = P.SatParams(n_steps=steps, seed=31, chain_id=M, n_stages=40, m_cand=M, T0=None,
                      q_auto=50, delta_max=0.05)
    print("fp64 %s body N=%d U=%d K=%d M=%d" % (name, N, U, K, M), flush=True)
    g = _gpu_chain(P, sl, "f64", prm)
    assert g[1]["body"] & 0xff == _body(P, kind), g[1]["body"]
    _compare_fp64(g, _oracle_chain(sl, prm))


def test_fp64_chain_c2_geometry_matches_oracle(P):
    """The 256 x 256, 180-angle, 367-bin geometry at M = 16 in FP64 (the
    benchmark's FP64 reference chain), 2e5 steps, T0 from Eq. 8."""
    sl = datagen.config_slice("c2")
    c = datagen.CONFIGS["c2"]
    prm = P.SatParams(n_steps=200_000, seed=c["chain_seed"], chain_id=0, n_stages=c["n_stages"],
                      m_cand=c["M"], T0=None, q_auto=c["q_auto"], delta_max=c["delta_max"])
    print("fp64 c2 geometry chain, 2e5 steps", flush=True)
    g = _gpu_chain(P, sl, "f64", prm)
    assert g[1]["body"] & P._binding.BODY_GLOBAL_R
    _compare_fp64(g, _oracle_chain(sl, prm))


# 192^2 x 180: pipelined body; 128^2 x 360 (rows up to 524 entries): long-row body
@pytest.mark.parametrize("N,U,K,M,kind", [(192, 180, 272, 8, 1), (128, 360, 182, 8, 2)])
def test_fp32_rmse_within_one_percent_of_oracle_fp64(P, N, U, K, M, kind):
    """FP32 residual with FP64 resyncs, residual in global memory: the final
    RMSE against the phantom is within 1% of the oracle's FP64 chain with the
    same seeds, alone (segmented, grid-wide resyncs) and in a batch (in-group
    resyncs); both GPU runs give the same bits."""
    assert U * K * 4 > LDS_BUDGET
    sl = _slice(N, U, K, seed=5 + N, masked=True, I0=1e4, n_ell=8)
    P_sup = int(sl.mask.sum())
    steps = 40 * P_sup
    base = dict(n_steps=steps, seed=77, chain_id=1, m_cand=M, T0=None, q_auto=100, n_stages=200,
                delta_max=0.05)
    print("fp32 vs oracle fp64 N=%d U=%d steps=%d" % (N, U, steps), flush=True)
    f32, s32, _ = _gpu_chain(P, sl, "f32", P.SatParams(precision="f32", resync_every=2048, **base),
                             trace=False)
    assert s32["resyncs"] >= 2
    assert s32["body"] & 0xff == kind | P._binding.BODY_GLOBAL_R | P._binding.BODY_SEGMENTED, s32["body"]
    f_o, s_o, _ = _oracle_chain(sl, P.SatParams(precision="f64", **base))
    r32 = datagen.rmse(f32, sl.truth)
    r64 = datagen.rmse(f_o, sl.truth)
    print("rmse fp32 gpu %.6f, fp64 oracle %.6f, drift %.3g" % (r32, r64, s32["max_drift_r"]),
          flush=True)
    assert abs(r32 / r64 - 1.0) <= 0.01
    assert s32["max_drift_r"] <= 1e-3
    geom = P.Geometry(sl.N, sl.angles, sl.K, sl.mask, "f32")
    pl = P.pila_build(geom)
    img = torch.from_numpy(sl.f0.copy()).cuda()
    st = P.sat_run_batch([P.Job(pl, torch.from_numpy(sl.sino).cuda(), img,
                                P.SatParams(precision="f32", resync_every=2048, **base))],
                         waves_per_chain=8, chains_per_cu=1)
    assert np.array_equal(img.cpu().numpy(), f32)
    assert st[0]["accepts"] == s32["accepts"] and st[0]["resyncs"] == s32["resyncs"]


# N = 300 and 520 give 2 and 3 image bands in the forward projection (bands of
# 256 and 248 rows), the last one ragged
@pytest.mark.parametrize("N,U,K,masked", [(300, 24, 425, True), (300, 16, 425, False),
                                          (520, 12, 736, True)])
def test_sirt_multiband_matches_oracle(P, N, U, K, masked):
    ell = datagen.random_ellipses(N + U, N, 8)
    sl = datagen.make_slice(N, U, K, ell, masked=masked, I0=1e4, noise_seed=3)
    iters, lam = 5, 0.1
    csr = oracle.pila(N, U, K, sl.angles, sl.mask)
    f_o, c_o = oracle.sirt_run(N, U, K, csr, sl.sino, sl.f0, iters, lam)
    sino = torch.from_numpy(sl.sino).cuda()
    print("sirt multiband N=%d U=%d" % (N, U), flush=True)
    pl = P.pila_build(P.Geometry(N, sl.angles, K, sl.mask, "f64"))
    img = torch.from_numpy(sl.f0.copy()).cuda()
    cost = P.sirt_run(pl, sino, iters, lam, img)
    f_g = img.cpu().numpy()
    assert np.max(np.abs(f_g - f_o)) <= 1e-10 * max(1.0, np.max(np.abs(f_o)))
    assert np.max(np.abs(cost - c_o) / c_o) <= 1e-12
    # FP32 lengths: the same iteration with the lengths rounded to float (the
    # oracle run on those lengths accumulates in FP64 as the GPU does; a
    # length whose two FP64 computations straddle a float rounding boundary
    # may differ by one float unit, which moves the image by ~1e-10)
    csr32 = (csr[0], csr[1], csr[2].astype(np.float32).astype(np.float64))
    f_o32, c_o32 = oracle.sirt_run(N, U, K, csr32, sl.sino, sl.f0, iters, lam)
    pl32 = P.pila_build(P.Geometry(N, sl.angles, K, sl.mask, "f32"))
    img32 = torch.from_numpy(sl.f0.copy()).cuda()
    cost32 = P.sirt_run(pl32, sino, iters, lam, img32)
    f_g32 = img32.cpu().numpy()
    assert np.max(np.abs(f_g32 - f_o32)) <= 1e-8 * max(1.0, np.max(np.abs(f_o32)))
    assert np.max(np.abs(cost32 - c_o32) / c_o32) <= 1e-9
    # and against the FP64-length oracle: a relative length error of at most
    # 2^-24 moves each iteration's update by a few units of that size
    assert np.max(np.abs(f_g32 - f_o)) <= 64 * 2.0 ** -24 * iters * max(1.0, np.max(np.abs(f_o)))
