"""HIP graphs of chains and batches against the eager calls (MI355X).

A graph captured from sat_run (a segmented FP32 chain: hundreds of launches;
chains on one workgroup and split over several)
or from sat_run_batch (several groups on forked streams) is replayed several
times, with other eager work and synchronisations between the replays, and
every replay must give the eager call's bits."""
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


def _eager_noise():
    # unrelated eager work between replays, with a synchronisation
    a = torch.randn(1 << 20, device="cuda")
    (a * 2.0 + 1.0).sum().item()
    torch.cuda.synchronize()


# the last two: chains split over eight workgroups (their exchange words are
# cleared by a kernel at the start of every replay)
@pytest.mark.parametrize("dt,N,U,K,M,every", [("f32", 192, 180, 272, 8, 256), ("f64", 40, 36, 57, 16, 0),
                                              ("f32", 64, 600, 91, 32, 300), ("f64", 48, 600, 68, 32, 0)])
def test_chain_graph_replays_match_eager(P, dt, N, U, K, M, every):
    sl = _slice(N, U, K, seed=N + 1, masked=True, I0=1e4)
    prm = P.SatParams(n_steps=12000, seed=5, chain_id=2, m_cand=M, T0=None, q_auto=40, precision=dt,
                      resync_every=every, n_stages=30)
    geom = P.Geometry(N, sl.angles, K, sl.mask, dt)
    pl = P.pila_build(geom)
    sino = torch.from_numpy(sl.sino).cuda()
    f0 = torch.from_numpy(sl.f0).cuda()
    ref = f0.clone()
    st_ref, tr_ref = P.sat_run(pl, sino, prm, ref, trace=True)
    torch.cuda.synchronize()
    if dt == "f32":
        assert st_ref["chain_launches"] > 20  # a segmented chain: many launches
    img = f0.clone()
    tr = dict(m_star=torch.empty(prm.n_steps, dtype=torch.int32, device="cuda"),
              accept=torch.empty(prm.n_steps, dtype=torch.uint8, device="cuda"),
              dC=torch.empty(prm.n_steps, dtype=torch.float64, device="cuda"))
    g = P.sat_graph(pl, sino, prm, img, trace=tr)
    for rep in range(3):
        img.copy_(f0)
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(img, ref), rep
        for k in ("m_star", "accept", "dC"):
            assert torch.equal(tr[k], tr_ref[k]), (rep, k)
        st = g.stats()[0]
        for k in ("accepts", "accepts_nonzero", "resyncs", "sse_final", "body"):
            assert st[k] == st_ref[k], (rep, k)
        _eager_noise()
    g.close()


def test_batch_graph_replays_match_eager(P):
    specs = [(24, 30, 35, "f32", 8), (64, 360, 91, "f32", 8), (48, 60, 68, "f32", 4), (32, 45, 47, "f64", 8),
             (40, 90, 57, "f32", 16)]
    jobs, f0s = [], []
    for q, (N, U, K, dt, M) in enumerate(specs):
        sl = _slice(N, U, K, seed=200 + q, masked=True, I0=1e4)
        prm = P.SatParams(n_steps=2000 + 700 * q, seed=99, chain_id=q, m_cand=M, T0=None, q_auto=30,
                          n_stages=20, precision=dt, resync_every=128 if dt == "f32" else 0)
        pl = P.pila_build(P.Geometry(N, sl.angles, K, sl.mask, dt))
        f0 = torch.from_numpy(sl.f0).cuda()
        f0s.append(f0)
        jobs.append(P.Job(pl, torch.from_numpy(sl.sino).cuda(), f0.clone(), prm))
    groups = []
    st_ref = P.sat_run_batch(jobs, waves_per_chain=8, chains_per_cu=1, groups=groups)
    torch.cuda.synchronize()
    assert len(groups) >= 3  # several kernels on forked streams
    ref = [j.image.clone() for j in jobs]
    g = P.sat_batch_graph(jobs, waves_per_chain=8, chains_per_cu=1)
    for rep in range(3):
        for j, f0 in zip(jobs, f0s):
            j.image.copy_(f0)
        g.launch()
        torch.cuda.synchronize()
        for q, j in enumerate(jobs):
            assert torch.equal(j.image, ref[q]), (rep, q)
        st = g.stats()
        for q in range(len(jobs)):
            for k in ("accepts", "resyncs", "sse_final", "body"):
                assert st[q][k] == st_ref[q][k], (rep, q, k)
        _eager_noise()
    g.close()
