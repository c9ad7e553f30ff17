"""GPU parity with one-byte lengths (section II-B: a length l is stored as
round(180 l) and read back as q / 180).

The PILA build must give the oracle's bytes; projections and FP64 chains on
one-byte lengths must give the oracle's results on the dequantized lengths
(the float q / 180 widened to double, as the oracle defines it) to the FP64
bars of the exact-length tests; FP32 chains on one-byte lengths must give the
same bits alone and batched, and end within 1% in RMSE of the same chain on
FP32 lengths.
"""
import numpy as np
import pytest

import datagen
import oracle
from test_gpu_sat import _compare_fp64, _slice

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

LDS_BUDGET = 160 * 1024


@pytest.fixture(scope="module")
def P():
    import paper_1411_4622_amd as P
    P.load()
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return P


def _q_matches(got, ln):
    """got == round(180 l) for every entry, except where 180 l lies within the
    FP64 length tolerance of a half-integer (either neighbour is then right)."""
    want = oracle.quantize_u8(ln)
    x = 180.0 * ln
    tie = np.abs(x - np.floor(x) - 0.5) <= 180.0 * 1e-12
    bad = (got != want) & ~(tie & (np.abs(got.astype(np.int32) - want.astype(np.int32)) == 1))
    assert not bad.any(), "byte %d: gpu %d oracle %d (180 l = %r)" % (
        int(np.flatnonzero(bad)[0]), got[bad][0], want[bad][0], x[bad][0])


def _dq_csr(csr):
    rp, col, ln = csr
    return rp, col, oracle.dequantize_u8(oracle.quantize_u8(ln))


@pytest.mark.parametrize("N,U,K,masked", [(256, 180, 367, True), (100, 77, 143, True), (9, 36, 13, False)])
def test_pila_u8_bytes_match_oracle(P, N, U, K, masked):
    ang = datagen.angles_deg(U)
    mask = datagen.circle_mask(N) if masked else None
    print("u8 pila N=%d U=%d K=%d" % (N, U, K), flush=True)
    pl = P.pila_build(P.Geometry(N, ang, K, mask, "u8"))
    (rp, col, ln), (off, pix, rl) = oracle.pila(N, U, K, ang, mask, with_rays=True)
    assert pl.len.dtype == torch.uint8
    assert np.array_equal(pl.row_ptr.cpu().numpy(), rp)
    assert np.array_equal(pl.col.cpu().numpy(), col)
    _q_matches(pl.len.cpu().numpy(), ln)
    rid = np.repeat(np.arange(U * K), np.diff(off))
    order = np.lexsort((pix, rid))
    assert np.array_equal(pl.t_col.cpu().numpy(), pix[order])
    _q_matches(pl.t_len.cpu().numpy(), rl[order])
    # the quantisation bound of section II-B, on the lengths the device stored
    dq = oracle.dequantize_u8(pl.len.cpu().numpy())
    assert np.max(np.abs(dq - ln), initial=0.0) <= 1.0 / 360.0 + 1e-7


def test_projections_u8_match_oracle_on_dequantized_lengths(P):
    N, U, K = 96, 60, 137
    ang, mask = datagen.angles_deg(U), datagen.circle_mask(N)
    pl = P.pila_build(P.Geometry(N, ang, K, mask, "u8"))
    csr = _dq_csr(oracle.pila(N, U, K, ang, mask))
    rng = np.random.default_rng(5)
    f, y = rng.random((N, N)), rng.standard_normal((U, K))
    pf = P.pila_forward(pl, torch.from_numpy(f).cuda()).cpu().numpy()
    of = oracle.forward(N, U, K, csr, f)
    assert np.all(np.abs(pf - of) <= 1e-12 * oracle.forward(N, U, K, csr, np.abs(f)) + 1e-300)
    pb = P.pila_backproject(pl, torch.from_numpy(y).cuda()).cpu().numpy()
    ob = oracle.backward(N, csr, y)
    assert np.all(np.abs(pb - ob) <= 1e-12 * oracle.backward(N, csr, np.abs(y)) + 1e-300)


def _run(P, sl, dtype, prm, trace=True):
    pl = P.pila_build(P.Geometry(sl.N, sl.angles, sl.K, sl.mask, dtype))
    img = torch.from_numpy(sl.f0.copy()).cuda()
    st, tr = P.sat_run(pl, torch.from_numpy(sl.sino).cuda(), prm, img, trace=trace)
    torch.cuda.synchronize()
    if tr is not None:
        tr = {k: v.cpu().numpy() for k, v in tr.items()}
    return (img.cpu().numpy(), st, tr), pl


def _oracle(sl, prm):
    csr = _dq_csr(oracle.pila(sl.N, sl.U, sl.K, sl.angles, sl.mask))
    return oracle.sat_run(sl.N, sl.U, sl.K, csr, sl.sino, sl.f0, mask=sl.mask, seed=prm.seed,
                          chain_id=prm.chain_id, n_steps=prm.n_steps, n_stages=prm.n_stages,
                          m_cand=prm.m_cand, T0=prm.T0, TN=prm.TN, q_auto=prm.q_auto,
                          delta_max=prm.delta_max, precision="f64", schedule=prm.schedule,
                          proposal=prm.proposal)


@pytest.mark.parametrize("N,U,K,M,steps", [(32, 45, 47, 16, 20000), (64, 120, 91, 4, 20000)])
def test_fp64_chain_u8_matches_oracle(P, N, U, K, M, steps):
    """FP64 residual on one-byte lengths, alone and batched: the oracle's
    decisions on the dequantized lengths, step for step."""
    sl = _slice(N, U, K, seed=N + M, masked=True, I0=1e4)
    prm = P.SatParams(n_steps=steps, seed=19, chain_id=M, n_stages=40, m_cand=M, T0=None, q_auto=50,
                      delta_max=0.05)
    print("fp64 u8 chain N=%d U=%d M=%d" % (N, U, M), flush=True)
    g, pl = _run(P, sl, "u8", prm)
    _compare_fp64(g, _oracle(sl, prm))
    img = torch.from_numpy(sl.f0.copy()).cuda()
    st = P.sat_run_batch([P.Job(pl, torch.from_numpy(sl.sino).cuda(), img, prm)], waves_per_chain=4,
                         chains_per_cu=2)
    assert np.array_equal(img.cpu().numpy(), g[0])
    assert st[0]["accepts"] == g[1]["accepts"]


# residual in LDS (pipelined body), in global memory (pipelined body with
# slot words; long-row body for rows of more than 512 entries)
@pytest.mark.parametrize("N,U,K,M,kind,glob", [(64, 90, 91, 8, 1, False), (192, 180, 272, 8, 1, True),
                                               (128, 360, 182, 8, 2, True)])
def test_fp32_chain_u8_batch_equals_alone_and_rmse(P, N, U, K, M, kind, glob):
    assert (U * K * 4 > LDS_BUDGET) == glob
    sl = _slice(N, U, K, seed=5 + N, masked=True, I0=1e4, n_ell=8)
    steps = 40 * int(sl.mask.sum())
    base = dict(n_steps=steps, seed=77, chain_id=1, m_cand=M, T0=None, q_auto=100, n_stages=200,
                delta_max=0.05, precision="f32", resync_every=2048)
    print("fp32 u8 chain N=%d U=%d K=%d steps=%d" % (N, U, K, steps), flush=True)
    (fq, sq, _), pl = _run(P, sl, "u8", P.SatParams(**base), trace=False)
    want = kind | (P._binding.BODY_GLOBAL_R | P._binding.BODY_SEGMENTED if glob else 0)
    assert sq["body"] & 0xff == want, sq["body"]
    assert sq["max_drift_r"] <= 1e-3
    img = torch.from_numpy(sl.f0.copy()).cuda()
    st = P.sat_run_batch([P.Job(pl, torch.from_numpy(sl.sino).cuda(), img, P.SatParams(**base))],
                         waves_per_chain=8, chains_per_cu=1)
    assert np.array_equal(img.cpu().numpy(), fq)
    assert st[0]["accepts"] == sq["accepts"]
    (f4, s4, _), _ = _run(P, sl, "f32", P.SatParams(**base), trace=False)
    rq, r4 = datagen.rmse(fq, sl.truth), datagen.rmse(f4, sl.truth)
    print("rmse u8 %.6f f32 %.6f" % (rq, r4), flush=True)
    assert abs(rq / r4 - 1.0) <= 0.01


def test_sirt_u8_matches_oracle_on_dequantized_lengths(P):
    N, U, K = 64, 90, 91
    sl = _slice(N, U, K, seed=3, masked=True, I0=1e4)
    pl = P.pila_build(P.Geometry(N, sl.angles, K, sl.mask, "u8"))
    csr = _dq_csr(oracle.pila(N, U, K, sl.angles, sl.mask))
    img = torch.from_numpy(sl.f0.copy()).cuda()
    cost = P.sirt_run(pl, torch.from_numpy(sl.sino).cuda(), 20, 1.0, img)
    fo, co = oracle.sirt_run(N, U, K, csr, sl.sino, sl.f0, 20, 1.0)
    assert np.max(np.abs(img.cpu().numpy() - fo)) <= 1e-10 * max(1.0, np.max(np.abs(fo)))
    assert np.max(np.abs(cost - co) / co) <= 1e-12
