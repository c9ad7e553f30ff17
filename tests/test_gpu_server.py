"""The chain server (srv_* ABI) on the GPU.

A served chain must give exactly the image and counts of the same chain run
alone through sat_run (FP64 chains also match the oracle), whatever else the
server runs beside it; admission, cancellation, ring reuse and the resident
kernel's idle exit and relaunch are checked on small chains.
"""
import time

import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GiB = 1 << 30


@pytest.fixture(scope="module")
def P():
    import paper_1411_4622_amd as P
    P.load()
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return P


def _slice(N, U, K, seed, I0=1e4):
    ell = datagen.random_ellipses(seed, N, 6)
    return datagen.make_slice(N, U, K, ell, masked=True, I0=I0, noise_seed=seed + 7)


def _params(P, q, M, dt, steps):
    return P.SatParams(n_steps=steps, seed=4321, chain_id=q, m_cand=M, T0=None, q_auto=40,
                       n_stages=30, precision=dt, resync_every=256 if dt == "f32" else 0,
                       delta_max=0.05)


def _alone(P, sl, dt, prm):
    geom = P.Geometry(sl.N, sl.angles, sl.K, sl.mask, dt)
    pl = P.pila_build(geom)
    img = torch.from_numpy(sl.f0.copy()).cuda()
    st, _ = P.sat_run(pl, torch.from_numpy(sl.sino).cuda(), prm, img)
    torch.cuda.synchronize()
    return img.cpu().numpy(), st


def _wait(srv, ticket, timeout=120.0):
    t0 = time.time()
    while True:
        st = srv.poll(ticket)
        if st is not None:
            return st
        assert time.time() - t0 < timeout, "ticket %d not done after %.0f s" % (ticket, timeout)
        time.sleep(0.002)


# (N, U, K, precision, M): FP32 M <= 8 with short rows take the pipelined
# queue; M = 16 and FP64 take the general queue; 420 angles (rows of more
# than 512 entries) take the long-row queue
SPECS = [(24, 30, 35, "f32", 4), (32, 45, 47, "f32", 8), (20, 18, 29, "f64", 3),
         (28, 36, 40, "f32", 16), (40, 60, 57, "f32", 8), (16, 12, 23, "f64", 8),
         (24, 420, 35, "f32", 6)]


def _requests(P, specs, steps0=2000):
    out = []
    for q, (N, U, K, dt, M) in enumerate(specs):
        sl = _slice(N, U, K, seed=300 + q)
        out.append((sl, dt, _params(P, q, M, dt, steps0 + 300 * q)))
    return out


def _submit(P, srv, sl, dt, prm):
    geom = P.Geometry(sl.N, sl.angles, sl.K, sl.mask, dt)
    img = torch.from_numpy(sl.f0.copy()).cuda()
    sino = torch.from_numpy(sl.sino).cuda()
    # inputs ready before the request is published.  Only this stream: a
    # device-wide synchronisation would also wait for the server's resident
    # kernel, i.e. for every chain in flight
    torch.cuda.current_stream().synchronize()
    t = srv.submit(geom, sino, img, prm)
    assert t is not None
    return t, img


def test_served_chains_match_lone_chains(P):
    reqs = _requests(P, SPECS)
    with P.Server(mem_budget=GiB, max_slots=16, idle_us=5000) as srv:
        tickets = [_submit(P, srv, *r) for r in reqs]
        queues = {t & 3 for t, _ in tickets}
        assert queues == {0, 1, 2}, "all three queues are exercised"
        stats = [_wait(srv, t) for t, _ in tickets]
        for (sl, dt, prm), (t, img), st in zip(reqs, tickets, stats):
            print("ticket %d N=%d M=%d %s" % (t, sl.N, prm.m_cand, dt), flush=True)
            ref, rst = _alone(P, sl, dt, prm)
            got = img.cpu().numpy()
            assert st["status"] == 0
            assert np.array_equal(got, ref), "served chain %d differs from sat_run" % t
            assert st["accepts"] == rst["accepts"] and st["resyncs"] == rst["resyncs"]
            if dt == "f64":
                csr = oracle.pila(sl.N, sl.U, sl.K, sl.angles, sl.mask)
                o = oracle.sat_run(sl.N, sl.U, sl.K, csr, sl.sino, sl.f0, mask=sl.mask, trace=False,
                                   seed=prm.seed, chain_id=prm.chain_id, n_steps=prm.n_steps,
                                   n_stages=prm.n_stages, m_cand=prm.m_cand, T0=None,
                                   q_auto=prm.q_auto, tn_ratio=prm.tn_ratio,
                                   delta_max=prm.delta_max, f_min=prm.f_min, f_max=prm.f_max,
                                   precision="f64", resync_every=0)
                assert np.max(np.abs(got - o[0])) <= 1e-9
        s = srv.status()
        assert s["in_flight"] == 0 and s["reaped"] == len(SPECS)


def test_alone_and_in_a_mix_agree(P):
    target = _requests(P, [(36, 40, 51, "f32", 8)], steps0=4000)[0]
    with P.Server(mem_budget=GiB, max_slots=8, idle_us=5000) as srv:
        t, img = _submit(P, srv, *target)
        _wait(srv, t)
        alone = img.cpu().numpy()
    mix = _requests(P, SPECS * 3)
    with P.Server(mem_budget=GiB, max_slots=8, idle_us=5000) as srv:
        held = [_submit(P, srv, *r) for r in mix[:9]]
        t, img = _submit(P, srv, *target)
        held += [_submit(P, srv, *r) for r in mix[9:]]
        for tk, _ in held:
            _wait(srv, tk)
        _wait(srv, t)
        assert np.array_equal(img.cpu().numpy(), alone)


def test_ring_slots_are_reused(P):
    reqs = _requests(P, SPECS[:2] * 5, steps0=800)
    with P.Server(mem_budget=GiB, max_slots=4, ring_size=4, idle_us=5000) as srv:
        pending = []
        done = 0
        for r in reqs:
            while True:
                try:
                    pending.append(_submit(P, srv, *r) + (r,))
                    break
                except AssertionError:  # ring full: reap the oldest first
                    t, img, rr = pending.pop(0)
                    _wait(srv, t)
                    assert np.array_equal(img.cpu().numpy(), _alone(P, rr[0], rr[1], rr[2])[0])
                    done += 1
        for t, img, rr in pending:
            _wait(srv, t)
            assert np.array_equal(img.cpu().numpy(), _alone(P, rr[0], rr[1], rr[2])[0])
            done += 1
        assert done == len(reqs)
        assert srv.status()["submitted"] == len(reqs)


def test_cancel_waiting_and_running(P):
    sl = _slice(48, 60, 68, seed=77)
    long_prm = _params(P, 1, 8, "f32", 5_000_000)
    # three slots: one pipelined workgroup, one general, one long-row; the
    # second pipelined chain waits
    with P.Server(mem_budget=GiB, max_slots=3, idle_us=5000) as srv:
        t1, img1 = _submit(P, srv, sl, "f32", long_prm)
        t2, img2 = _submit(P, srv, sl, "f32", _params(P, 2, 8, "f32", 5_000_000))
        time.sleep(0.5)
        srv.cancel(t2)  # still waiting: the only pipelined workgroup runs t1
        srv.cancel(t1)  # running: stops at its next check, then t2 is taken and skipped
        st1 = _wait(srv, t1, timeout=60)
        assert st1["status"] == -5
        assert 0 < st1["steps"] < long_prm.n_steps and (st1["steps"] - 1) % 1024 == 0
        assert not np.array_equal(img1.cpu().numpy(), sl.f0)
        st2 = _wait(srv, t2, timeout=60)
        assert st2["status"] == -5 and st2["steps"] == 0
        assert np.array_equal(img2.cpu().numpy(), sl.f0)


def test_admission_against_the_budget(P):
    small = _slice(24, 30, 35, seed=5)
    big = _slice(128, 180, 183, seed=6)
    prm = _params(P, 0, 4, "f32", 3000)
    with P.Server(mem_budget=24 << 20, max_slots=4, idle_us=5000) as srv:
        with pytest.raises(P.PilaError) as e:
            srv.submit(P.Geometry(big.N, big.angles, big.K, big.mask, "f32"),
                       torch.from_numpy(big.sino).cuda(), torch.from_numpy(big.f0.copy()).cuda(), prm)
        assert e.value.code == -2  # could never fit
        t, img = _submit(P, srv, small, "f32", prm)
        _wait(srv, t)
        s = srv.status()
        assert s["pila_cached"] == 1 and s["bytes_used"] <= s["bytes_budget"]


def test_idle_exit_and_relaunch(P):
    sl = _slice(24, 30, 35, seed=9)
    prm = _params(P, 0, 4, "f32", 1500)
    with P.Server(mem_budget=GiB, max_slots=4, idle_us=2000) as srv:
        t, img = _submit(P, srv, sl, "f32", prm)
        _wait(srv, t)
        first = img.cpu().numpy()
        t0 = time.time()
        while srv.status()["kernel_running"]:
            assert time.time() - t0 < 10, "resident kernel did not exit when idle"
            time.sleep(0.01)
        t, img = _submit(P, srv, sl, "f32", prm)
        _wait(srv, t)
        assert np.array_equal(img.cpu().numpy(), first)
        assert srv.status()["launches"] == 2
