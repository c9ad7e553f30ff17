"""Pins of the oracle's annealing chain and SIRT (CPU only).

The chain is replayed step by step with an independent generator (numpy's
Philox4x64-10), an independent projector (dense brute-force clipping) and
the cost written from its definition (Eq. 4), so the incremental update
(Eq. 6-7), the BoME choice (section III-B), the cooling schedule (Eq. 2),
the acceptance rule (Step 4) and Eq. 8 are all checked against something
that is not the oracle's own arithmetic.  SIRT (Eq. 10-11, simultaneous
form) is pinned to dense preconditioned Landweber and to its fixed point.
"""
import math

import numpy as np
import pytest

import brute_clip
import datagen
from test_oracle_geometry import np_philox

TWO53 = 2.0 ** -53


def _problem(N=8, U=10, K=13, seed=5, masked=True, noise=None):
    ang = datagen.angles_deg(U)
    ell = datagen.random_ellipses(seed, N, 4)
    sino = datagen.radon_ellipses(ell, N, ang, K)
    if noise is not None:
        sino = datagen.poisson_noise(sino, N, noise, seed + 1)
    mask = datagen.circle_mask(N) if masked else None
    f0 = datagen.uniform_start(sino, mask, N)
    return ang, sino, mask, f0


def _cost(A, f, b, KU):
    r = A @ f.reshape(-1) - b.reshape(-1)
    return math.sqrt(float(r @ r) / KU)


def _estimate(key, ctr, support, f, dmax, fmin, fmax):
    w = np_philox(key, ctr)
    idx = (int(w[0]) * len(support)) >> 64
    p = int(support[idx])
    u1 = (int(w[1]) >> 11) * TWO53
    delta = dmax * (2.0 * u1 - 1.0)
    fn = min(max(f[p] + delta, fmin), fmax)
    return p, fn


@pytest.mark.parametrize("m_cand,masked", [(1, False), (4, True), (7, True)])
def test_chain_replay(oracle_lib, m_cand, masked):
    N, U, K = 8, 10, 13
    ang, sino, mask, f0 = _problem(N, U, K, masked=masked)
    A = brute_clip.dense_system(N, U, K, ang, mask)
    KU = float(K * U)
    prm = dict(seed=11, chain_id=3, n_steps=500, n_stages=7, m_cand=m_cand, T0=4e-3, TN=4e-6,
               delta_max=0.3, f_min=0.0, f_max=1.0, precision="f64")
    csr = oracle_lib.pila(N, U, K, ang, mask)
    f_or, st, tr = oracle_lib.sat_run(N, U, K, csr, sino, f0, mask=mask, **prm)

    support = np.flatnonzero(np.ones(N * N) if mask is None else mask.reshape(-1))
    key = [prm["seed"], prm["chain_id"]]
    f = f0.reshape(-1).copy()
    n_acc = 0
    n_margin = 0
    for s in range(prm["n_steps"]):
        n = (s * prm["n_stages"]) // prm["n_steps"]
        T = prm["T0"] - n * (prm["T0"] - prm["TN"]) / prm["n_stages"]
        assert abs(T - oracle_lib.temperature(s, prm["n_steps"], prm["n_stages"], prm["T0"], prm["TN"])) <= 1e-18
        C0 = _cost(A, f, sino, KU)
        costs, cands = [], []
        for m in range(m_cand):
            p, fn = _estimate(key, [s, m, 0, 0], support, f, prm["delta_max"], 0.0, 1.0)
            fm = f.copy()
            fm[p] = fn
            costs.append(_cost(A, fm, sino, KU))
            cands.append((p, fn))
        ms = int(tr["m_star"][s])
        tol = 1e-12 * max(C0, 1.0)
        assert costs[ms] <= min(costs) + tol, "chosen estimate is not the best"
        for m in range(ms):
            assert costs[m] > costs[ms] - tol or abs(costs[m] - costs[ms]) <= tol
            assert not (costs[m] < costs[ms] - tol)
        dC_full = costs[ms] - C0
        assert abs(tr["dC"][s] - dC_full) <= 1e-11 + 1e-9 * abs(dC_full)
        wa = np_philox(key, [s, 0, 1, 0])
        N1 = (int(wa[0]) >> 11) * TWO53
        dC = float(tr["dC"][s])
        thr = math.exp(-dC / T)
        if dC > 0 and abs(N1 - thr) < 1e-9:
            n_margin += 1
        else:
            assert bool(tr["accept"][s]) == (dC <= 0.0 or N1 < thr)
        if tr["accept"][s]:
            p, fn = cands[ms]
            f[p] = fn
            n_acc += 1
    assert n_margin == 0
    assert np.array_equal(f.reshape(N, N), f_or), "replayed image differs from the oracle's"
    assert st["accepts"] == n_acc
    # the run must have exercised both outcomes
    assert 0 < n_acc < prm["n_steps"]
    # running cost agrees with the definition at the end
    assert abs(st["cost_final"] - _cost(A, f_or, sino, KU)) <= 1e-12 * max(1.0, st["cost_final"])


def test_auto_t0_eq8(oracle_lib):
    N, U, K = 8, 10, 13
    ang, sino, mask, f0 = _problem(N, U, K, masked=True)
    A = brute_clip.dense_system(N, U, K, ang, mask)
    KU = float(K * U)
    prm = dict(seed=21, chain_id=0, n_steps=10, n_stages=5, m_cand=2, T0=None, TN=None,
               q_auto=20, tn_ratio=1e3, delta_max=0.2, precision="f64")
    csr = oracle_lib.pila(N, U, K, ang, mask)
    _, st, _ = oracle_lib.sat_run(N, U, K, csr, sino, f0, mask=mask, **prm)
    support = np.flatnonzero(mask.reshape(-1))
    f = f0.reshape(-1)
    C0 = _cost(A, f, sino, KU)
    ups = []
    q = 0
    while len(ups) < 20:
        p, fn = _estimate([21, 0], [q, 0, 2, 0], support, f, 0.2, 0.0, 1.0)
        fm = f.copy()
        fm[p] = fn
        d = _cost(A, fm, sino, KU) - C0
        if d > 0:
            ups.append(d)
        q += 1
    T0 = -sum(ups) / (20 * math.log(0.9))
    assert T0 > 0
    assert abs(st["T0_used"] - T0) <= 1e-10 * T0
    assert abs(st["TN_used"] - T0 / 1e3) <= 1e-10 * T0


def test_schedule_endpoints(oracle_lib):
    T0, TN, n_stages, n_steps = 1e-2, 1e-6, 1000, 200_000
    assert oracle_lib.temperature(0, n_steps, n_stages, T0, TN) == T0
    last = oracle_lib.temperature(n_steps - 1, n_steps, n_stages, T0, TN)
    assert abs(last - (TN + (T0 - TN) / n_stages)) <= 1e-18
    # 200 steps per stage: constant within a stage, strictly decreasing across
    assert oracle_lib.temperature(199, n_steps, n_stages, T0, TN) == T0
    assert oracle_lib.temperature(200, n_steps, n_stages, T0, TN) < T0


def test_fp32_residual_drift(oracle_lib):
    N, U, K = 16, 24, 23
    ang, sino, mask, f0 = _problem(N, U, K, masked=True, noise=1e4)
    csr = oracle_lib.pila(N, U, K, ang, mask)
    base = dict(seed=31, chain_id=0, n_steps=20_000, n_stages=50, m_cand=4, T0=None,
                q_auto=50, delta_max=0.05)
    f64, s64, _ = oracle_lib.sat_run(N, U, K, csr, sino, f0, mask=mask, trace=False,
                                     precision="f64", **base)
    f32, s32, _ = oracle_lib.sat_run(N, U, K, csr, sino, f0, mask=mask, trace=False,
                                     precision="f32", resync_every=256, **base)
    assert s32["resyncs"] >= 1
    rmax = float(np.max(np.abs(sino)))
    assert s32["max_drift_r"] <= 1e-4 * rmax
    assert s32["max_drift_sse"] <= 1e-3
    # both chains anneal to a similar cost
    assert abs(s32["cost_final"] - s64["cost_final"]) <= 0.05 * s64["cost_final"]


def _landweber(A, b, x, lam, U, n_iter):
    W = (A * A).sum(axis=1)
    winv = np.where(W > 0, 1.0 / np.where(W > 0, W, 1.0), 0.0)
    costs = []
    for _ in range(n_iter):
        r = b - A @ x
        costs.append(math.sqrt(float(r @ r) / A.shape[0]))
        x = x + (lam / U) * (A.T @ (winv * r))
    return x, np.array(costs)


@pytest.mark.parametrize("lam", [1.0, 0.1])
def test_sirt_equals_dense_landweber(oracle_lib, lam):
    N, U, K = 8, 12, 13
    ang, sino, mask, f0 = _problem(N, U, K, masked=True)
    A = brute_clip.dense_system(N, U, K, ang, mask)
    csr = oracle_lib.pila(N, U, K, ang, mask)
    f_or, cost = oracle_lib.sirt_run(N, U, K, csr, sino, f0, 30, lam)
    x, c_ref = _landweber(A, sino.reshape(-1), f0.reshape(-1).copy(), lam, U, 30)
    assert np.max(np.abs(f_or.reshape(-1) - x)) <= 1e-12
    assert np.max(np.abs(cost - c_ref)) <= 1e-12


def test_sirt_fixed_point_is_weighted_least_squares(oracle_lib):
    N, U, K = 8, 16, 13
    ang = datagen.angles_deg(U)
    mask = datagen.circle_mask(N)
    A = brute_clip.dense_system(N, U, K, ang, mask)
    sup = np.flatnonzero(mask.reshape(-1))
    assert np.linalg.matrix_rank(A[:, sup]) == len(sup)
    rng = np.random.default_rng(9)
    x_true = np.zeros(N * N)
    x_true[sup] = rng.random(len(sup))
    b = (A @ x_true).reshape(U, K)
    csr = oracle_lib.pila(N, U, K, ang, mask)
    f0 = datagen.uniform_start(b, mask, N)
    f, cost = oracle_lib.sirt_run(N, U, K, csr, b, f0, 30000, 1.0)
    # weighted least squares: minimise |W^-1/2 (A x - b)| over the support
    W = (A * A).sum(axis=1)
    w = np.where(W > 0, 1.0 / np.sqrt(np.where(W > 0, W, 1.0)), 0.0)
    sol, *_ = np.linalg.lstsq(w[:, None] * A[:, sup], w * b.reshape(-1), rcond=None)
    assert np.max(np.abs(sol - x_true[sup])) <= 1e-9
    assert np.max(np.abs(f.reshape(-1)[sup] - sol)) <= 1e-9
    # the weighted residual never increases (step inside the convergence range)
    r_w = []
    for it in range(1, 60):
        fi, _ = oracle_lib.sirt_run(N, U, K, csr, b, f0, it, 1.0)
        r = w * (A @ fi.reshape(-1) - b.reshape(-1))
        r_w.append(float(r @ r))
    assert all(r_w[i + 1] <= r_w[i] * (1 + 1e-12) for i in range(len(r_w) - 1))
