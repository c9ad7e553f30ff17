"""GPU parity of the annealing chains against the oracle (MI355X).

FP64 chains must reproduce the oracle's accept/reject sequence and BoME
choices exactly, Delta C within 1e-12 (relative to |Delta C| plus the
rounding scale of its sum), and the final image within 1e-9 max-abs.
"""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_1411_4622_amd as P
    P.load()
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return P


def _slice(N, U, K, seed, n_ell=6, masked=True, I0=None):
    ell = datagen.random_ellipses(seed, N, n_ell)
    return datagen.make_slice(N, U, K, ell, masked=masked, I0=I0, noise_seed=seed + 7)


def _gpu_chain(P, sl, dtype, params, trace=True):
    geom = P.Geometry(sl.N, sl.angles, sl.K, sl.mask, dtype)
    pl = P.pila_build(geom)
    img = torch.from_numpy(sl.f0.copy()).cuda()
    sino = torch.from_numpy(sl.sino).cuda()
    st, tr = P.sat_run(pl, sino, params, img, trace=trace)
    torch.cuda.synchronize()
    out = img.cpu().numpy()
    if tr is not None:
        tr = {k: v.cpu().numpy() for k, v in tr.items()}
    return out, st, tr


def _oracle_chain(sl, params, **extra):
    csr = oracle.pila(sl.N, sl.U, sl.K, sl.angles, sl.mask)
    kw = dict(seed=params.seed, chain_id=params.chain_id, n_steps=params.n_steps,
              n_stages=params.n_stages, m_cand=params.m_cand, T0=params.T0, TN=params.TN,
              q_auto=params.q_auto, tn_ratio=params.tn_ratio, delta_max=params.delta_max,
              f_min=params.f_min, f_max=params.f_max, precision=params.precision,
              resync_every=params.resync_every)
    kw.update(extra)
    return oracle.sat_run(sl.N, sl.U, sl.K, csr, sl.sino, sl.f0, mask=sl.mask, **kw)


def _compare_fp64(g, o):
    f_g, st_g, tr_g = g
    f_o, st_o, tr_o = o
    mism = np.flatnonzero((tr_g["m_star"] != tr_o["m_star"]) | (tr_g["accept"] != tr_o["accept"]))
    if len(mism):
        s = int(mism[0])
        raise AssertionError("decision differs first at step %d: gpu (m=%d, acc=%d, dC=%r) oracle "
                             "(m=%d, acc=%d, dC=%r)" % (s, tr_g["m_star"][s], tr_g["accept"][s],
                                                        tr_g["dC"][s], tr_o["m_star"][s],
                                                        tr_o["accept"][s], tr_o["dC"][s]))
    err = np.abs(tr_g["dC"] - tr_o["dC"])
    bound = 1e-12 * (np.abs(tr_o["dC"]) + tr_o["scale"]) + 1e-300
    worst = int(np.argmax(err / bound))
    assert np.all(err <= bound), "dC step %d: %r vs %r" % (worst, tr_g["dC"][worst], tr_o["dC"][worst])
    assert np.max(np.abs(f_g - f_o)) <= 1e-9
    assert st_g["accepts"] == st_o["accepts"]
    assert st_g["accepts_nonzero"] == st_o["accepts_nonzero"]
    assert abs(st_g["T0_used"] - st_o["T0_used"]) <= 1e-12 * st_o["T0_used"]
    assert abs(st_g["sse_final"] - st_o["sse_final"]) <= 1e-9 * st_o["sse_final"]


def test_fp64_chain_c1_full(P):
    """The 64 x 64, 90-angle, 64-bin single chain, 2e5 steps, M=1, T0=1e-2, TN=1e-6."""
    c = datagen.CONFIGS["c1"]
    sl = datagen.config_slice("c1")
    prm = P.SatParams(n_steps=c["n_steps"], seed=c["chain_seed"], chain_id=0, n_stages=c["n_stages"],
                      m_cand=c["M"], T0=c["T0"], TN=c["TN"], delta_max=c["delta_max"])
    print("fp64 c1 chain", flush=True)
    g = _gpu_chain(P, sl, "f64", prm)
    o = _oracle_chain(sl, prm)
    _compare_fp64(g, o)
    assert 0 < g[1]["accepts"] < c["n_steps"]


@pytest.mark.parametrize("M,N,U,K,steps", [(16, 32, 45, 47, 20000), (7, 24, 30, 35, 20000),
                                           (64, 16, 12, 23, 3000), (32, 40, 60, 57, 6000)])
def test_fp64_chain_bome_masked(P, M, N, U, K, steps):
    sl = _slice(N, U, K, seed=M + N, masked=True, I0=1e4)
    prm = P.SatParams(n_steps=steps, seed=77, chain_id=M, n_stages=50, m_cand=M, T0=None,
                      q_auto=50, delta_max=0.1)
    print("fp64 bome M=%d N=%d" % (M, N), flush=True)
    _compare_fp64(_gpu_chain(P, sl, "f64", prm), _oracle_chain(sl, prm))


def test_fp64_chain_auto_t0_eq8(P):
    sl = _slice(48, 60, 68, seed=3, masked=True)
    prm = P.SatParams(n_steps=5000, seed=5, chain_id=2, n_stages=20, m_cand=4, T0=None, q_auto=200,
                      delta_max=0.05)
    g = _gpu_chain(P, sl, "f64", prm)
    o = _oracle_chain(sl, prm)
    _compare_fp64(g, o)
    assert g[1]["T0_used"] > 0 and abs(g[1]["TN_used"] - g[1]["T0_used"] / 1e3) <= 1e-18


def test_edge_cases(P):
    sl = _slice(16, 12, 23, seed=11, masked=True)
    # zero steps: image untouched, stats sane
    prm = P.SatParams(n_steps=0, T0=1e-2, TN=1e-6)
    f, st, _ = _gpu_chain(P, sl, "f64", prm, trace=False)
    assert np.array_equal(f, sl.f0) and st["accepts"] == 0
    # zero step width: every change is zero, every step accepted, image untouched
    prm = P.SatParams(n_steps=500, T0=1e-2, TN=1e-6, delta_max=0.0, m_cand=3)
    f, st, tr = _gpu_chain(P, sl, "f64", prm)
    assert np.array_equal(f, sl.f0) and st["accepts"] == 500 and st["accepts_nonzero"] == 0
    assert np.all(tr["m_star"] == 0)
    # single-pixel image
    one = datagen.Slice(1, 3, 1, datagen.angles_deg(3), None, np.full((3, 1), 0.5), np.ones((1, 1)),
                        np.full((1, 1), 0.2))
    prm = P.SatParams(n_steps=300, T0=1e-3, TN=1e-6, delta_max=0.2, n_stages=10)
    g = _gpu_chain(P, one, "f64", prm)
    o = _oracle_chain(one, prm)
    _compare_fp64(g, o)


def test_empty_support_is_rejected(P):
    N, U, K = 8, 4, 11
    geom = P.Geometry(N, datagen.angles_deg(U), K, np.zeros((N, N), np.uint8), "f64")
    pl = P.pila_build(geom)
    assert pl.n_support == 0 and pl.nnz == 0
    img = torch.zeros(N, N, dtype=torch.float64, device="cuda")
    sino = torch.zeros(U, K, dtype=torch.float64, device="cuda")
    with pytest.raises(P.PilaError) as e:
        P.sat_run(pl, sino, P.SatParams(n_steps=10, T0=1e-2, TN=1e-6), img)
    assert e.value.code == -1


def test_deterministic_and_launch_independent(P):
    sl = _slice(40, 36, 57, seed=21, masked=True, I0=1e4)
    prm = P.SatParams(n_steps=8000, seed=9, m_cand=8, T0=None, q_auto=50, precision="f32",
                      resync_every=256, n_stages=40)
    a = _gpu_chain(P, sl, "f32", prm, trace=True)
    b = _gpu_chain(P, sl, "f32", prm, trace=True)
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[2]["m_star"], b[2]["m_star"]) and np.array_equal(a[2]["dC"], b[2]["dC"])
    # same chain through the batched kernel with other launch shapes
    geom = P.Geometry(sl.N, sl.angles, sl.K, sl.mask, "f32")
    pl = P.pila_build(geom)
    sino = torch.from_numpy(sl.sino).cuda()
    for waves in (1, 2, 4, 8, 16):
        img = torch.from_numpy(sl.f0.copy()).cuda()
        st = P.sat_run_batch([P.Job(pl, sino, img, prm)], waves_per_chain=waves, chains_per_cu=2)
        assert np.array_equal(img.cpu().numpy(), a[0]), waves
        assert st[0]["accepts"] == a[1]["accepts"]


def test_fp32_residual_drift_and_quality(P):
    """FP32 residual with FP64 resync: bounded drift, cost close to FP64."""
    sl = _slice(64, 90, 91, seed=31, masked=True, I0=1e4, n_ell=8)
    base = dict(n_steps=300_000, seed=41, m_cand=8, T0=None, q_auto=100, n_stages=100,
                delta_max=0.05)
    f64, s64, _ = _gpu_chain(P, sl, "f64", P.SatParams(precision="f64", **base), trace=False)
    f32, s32, _ = _gpu_chain(P, sl, "f32", P.SatParams(precision="f32", resync_every=1024, **base),
                             trace=False)
    assert s32["resyncs"] >= 1
    assert s32["max_drift_r"] <= 1e-3
    assert s32["max_drift_sse"] <= 1e-3
    r64 = datagen.rmse(f64, sl.truth)
    r32 = datagen.rmse(f32, sl.truth)
    print("rmse fp64 %.6f fp32 %.6f" % (r64, r32), flush=True)
    assert abs(r32 - r64) <= 0.01 * r64
    # the FP64 chain against the oracle's FP64 chain on the same input
    o = _oracle_chain(sl, P.SatParams(precision="f64", **base))
    assert np.max(np.abs(f64 - o[0])) <= 1e-9


def test_batch_matches_single_and_oracle(P):
    specs = [(16, 12, 23, "f64", 1), (24, 30, 35, "f32", 4), (32, 45, 47, "f64", 8),
             (20, 18, 29, "f32", 16), (12, 8, 17, "f64", 3), (28, 36, 40, "f32", 8)]
    jobs, singles, slices = [], [], []
    for q, (N, U, K, dt, M) in enumerate(specs):
        sl = _slice(N, U, K, seed=100 + q, masked=True, I0=1e4)
        prm = P.SatParams(n_steps=3000 + 500 * q, seed=1234, chain_id=q, m_cand=M, T0=None,
                          q_auto=40, n_stages=30, precision=dt,
                          resync_every=128 if dt == "f32" else 0)
        geom = P.Geometry(N, sl.angles, K, sl.mask, dt)
        pl = P.pila_build(geom)
        img = torch.from_numpy(sl.f0.copy()).cuda()
        jobs.append(P.Job(pl, torch.from_numpy(sl.sino).cuda(), img, prm))
        slices.append((sl, prm))
        singles.append(_gpu_chain(P, sl, dt, prm, trace=False))
    stats = P.sat_run_batch(jobs, waves_per_chain=4, chains_per_cu=2)
    torch.cuda.synchronize()
    for q, job in enumerate(jobs):
        got = job.image.cpu().numpy()
        assert np.array_equal(got, singles[q][0]), "batch result differs from the lone chain %d" % q
        assert stats[q]["accepts"] == singles[q][1]["accepts"]
        sl, prm = slices[q]
        if prm.precision == "f64":
            o = _oracle_chain(sl, prm)
            assert np.max(np.abs(got - o[0])) <= 1e-9


def test_segmented_general_body_matches_in_group(P):
    """An FP32 chain the pipelined body cannot take (M = 40, 360 angles) with a
    residual too large for LDS: sat_run runs it in segments with grid-wide
    resyncs (on one workgroup with the smallest workspace, else split over
    ten), the general batch kernel resyncs inside its workgroup; all must
    give the same bits."""
    sl = _slice(96, 360, 136, seed=61, masked=True, I0=1e4)
    assert 360 * 136 * 4 > 160 * 1024
    prm = P.SatParams(n_steps=3000, seed=17, m_cand=40, T0=None, q_auto=30, precision="f32",
                      resync_every=200, n_stages=20)
    geom = P.Geometry(sl.N, sl.angles, sl.K, sl.mask, "f32")
    pl = P.pila_build(geom)
    sino = torch.from_numpy(sl.sino).cuda()
    # the smallest workspace leaves no room for a split chain's copies
    img_seg = torch.from_numpy(sl.f0.copy()).cuda()
    st_seg, _ = P.sat_run(pl, sino, prm, img_seg, workspace=P.sat_workspace(geom, prm, minimal=True))
    f_seg = img_seg.cpu().numpy()
    assert st_seg["body"] & 0xff == (P._binding.BODY_GENERAL | P._binding.BODY_GLOBAL_R
                                     | P._binding.BODY_SEGMENTED), st_seg["body"]
    assert st_seg["resyncs"] >= 2 and st_seg["chain_launches"] > 1
    # with room for them the chain is split over workgroups: same bits
    f_split, st_split, _ = _gpu_chain(P, sl, "f32", prm, trace=False)
    assert st_split["body"] & 15 == P._binding.BODY_SPLIT, st_split["body"]
    assert np.array_equal(f_split, f_seg) and st_split["accepts"] == st_seg["accepts"]
    img = torch.from_numpy(sl.f0.copy()).cuda()
    st = P.sat_run_batch([P.Job(pl, torch.from_numpy(sl.sino).cuda(), img, prm)],
                         waves_per_chain=16, chains_per_cu=1)
    assert np.array_equal(img.cpu().numpy(), f_seg)
    assert st[0]["accepts"] == st_seg["accepts"] and st[0]["resyncs"] == st_seg["resyncs"]


@pytest.mark.parametrize("U,K", [(420, 23), (720, 22)])
def test_long_rows_fp64_match_oracle(P, U, K):
    """420 angles: rows of more than 512 entries, which the long-row body
    (one estimate per wavefront, rows in registers) takes; 720 angles with an
    even bin count: the central pixels' rows (1050 entries) go past the
    registers' 1024 and their last entries are read in place."""
    sl = _slice(16, U, K, seed=71, masked=True, I0=1e4)
    if U == 720:
        geom = P.Geometry(sl.N, sl.angles, sl.K, sl.mask, "f64")
        assert P.pila_build(geom).max_row > 1024
    prm = P.SatParams(n_steps=4000, seed=19, chain_id=3, m_cand=6, T0=None, q_auto=30,
                      n_stages=40, delta_max=0.05)
    g = _gpu_chain(P, sl, "f64", prm)
    assert g[1]["chain_launches"] == 1
    _compare_fp64(g, _oracle_chain(sl, prm))


@pytest.mark.parametrize("U,K", [(420, 114), (720, 114)])
def test_long_rows_fp32_alone_batched_served_agree(P, U, K):
    """FP32 long rows with the residual partly in LDS: alone (segments with
    grid-wide resyncs), in a batch and served (in-workgroup resyncs) give the
    same bits; at 720 angles and an even bin count some rows are longer than
    the registers hold."""
    sl = _slice(80, U, K, seed=73, masked=True, I0=1e4)
    assert U * K * 4 > 160 * 1024
    prm = P.SatParams(n_steps=6000, seed=23, chain_id=1, m_cand=8, T0=None, q_auto=30,
                      precision="f32", resync_every=300, n_stages=30)
    f_alone, st_alone, _ = _gpu_chain(P, sl, "f32", prm, trace=False)
    assert st_alone["resyncs"] >= 2 and st_alone["chain_launches"] > 1
    geom = P.Geometry(sl.N, sl.angles, sl.K, sl.mask, "f32")
    pl = P.pila_build(geom)
    assert pl.max_row > (1024 if U == 720 else 512)
    sino = torch.from_numpy(sl.sino).cuda()
    img = torch.from_numpy(sl.f0.copy()).cuda()
    st = P.sat_run_batch([P.Job(pl, sino, img, prm)], waves_per_chain=8, chains_per_cu=1)
    assert np.array_equal(img.cpu().numpy(), f_alone)
    assert st[0]["accepts"] == st_alone["accepts"]
    img2 = torch.from_numpy(sl.f0.copy()).cuda()
    torch.cuda.current_stream().synchronize()
    with P.Server(mem_budget=1 << 30, max_slots=6, idle_us=5000) as srv:
        t = srv.submit(geom, sino, img2, prm)
        assert t is not None and t & 3 == 2, "long-row queue"
        while srv.poll(t) is None:
            pass
    assert np.array_equal(img2.cpu().numpy(), f_alone)


@pytest.mark.parametrize("U,K,steps", [(300, 151, 5000), (240, 201, 5000)])
def test_slot_words_match_computed_slots(P, U, K, steps):
    """The pipelined body that loads precomputed slot words (batches always;
    sat_run up to 256 angles) gives the bits of the one that forms them per
    entry (sat_run above 256 angles), and the FP32 chain stays within the
    drift bound of its FP64 resyncs."""
    sl = _slice(64, U, K, seed=81, masked=True, I0=1e4)
    assert U * K * 4 > 160 * 1024  # residual partly in global memory
    prm = P.SatParams(n_steps=steps, seed=29, chain_id=2, m_cand=8, T0=None, q_auto=30,
                      precision="f32", resync_every=400, n_stages=30)
    f_alone, st_alone, _ = _gpu_chain(P, sl, "f32", prm, trace=False)
    geom = P.Geometry(sl.N, sl.angles, sl.K, sl.mask, "f32")
    pl = P.pila_build(geom)
    assert pl.max_row <= 512  # the pipelined body
    sino = torch.from_numpy(sl.sino).cuda()
    img = torch.from_numpy(sl.f0.copy()).cuda()
    st = P.sat_run_batch([P.Job(pl, sino, img, prm)], waves_per_chain=8, chains_per_cu=1)
    torch.cuda.synchronize()
    assert np.array_equal(img.cpu().numpy(), f_alone)
    assert st[0]["accepts"] == st_alone["accepts"] and st[0]["resyncs"] == st_alone["resyncs"] >= 2
    assert st_alone["max_drift_r"] < 1e-3
