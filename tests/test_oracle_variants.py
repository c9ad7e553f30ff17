"""Pins of the oracle's paper variants (CPU only).

* Cooling schedules of section III-C: Eq. 2 (linear), the exponential one
  (the second Eq. 8) and the cubic one (Eq. 9), by their closed forms at
  special stages and their exact stage-to-stage steps, and inside the chain
  by a replay whose temperatures come from those closed forms.
* Eq. 3 as printed (the change is drawn again until the new value is in
  range), by a replay with an independent generator.
* Pixel-by-pixel SIRT (section III-D): one-pixel closed form, descent of the
  weighted residual at every single update, the weighted least-squares
  fixed point, and the running projections against a dense projection.
* The comparison projector of section III-A (DRT by bilinear
  interpolation): scipy's bilinear sampling of the same points, and the
  closed form of a constant image at 0 and 90 degrees; the SAT chain that
  uses it, by a replay against full costs computed with scipy.
* One-byte lengths (section II-B): |l - q/180| <= 1/360, q <= 255, and the
  projection error bound that follows.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import ndimage

import brute_clip
import datagen
from test_oracle_geometry import np_philox

TWO53 = 2.0 ** -53


# ---------------------------------------------------------------------------
# schedules
# ---------------------------------------------------------------------------

def test_exponential_schedule_closed_form(oracle_lib):
    T0, TN, S, n_steps = 2e-2, 3e-6, 1000, 100_000
    per = n_steps // S
    t = lambda n: oracle_lib.temperature(n * per, n_steps, S, T0, TN, "exp")
    assert t(0) == T0
    # half way the temperature is the geometric mean of the end points
    assert abs(t(S // 2) - math.sqrt(T0 * TN)) <= 1e-14 * T0
    # constant ratio between consecutive stages: (TN/T0)^(1/S)
    q = (TN / T0) ** (1.0 / S)
    for n in (0, 1, 17, 500, 998):
        assert abs(t(n + 1) / t(n) - q) <= 1e-13
    # constant within a stage, and the last stage stops one ratio above TN
    assert oracle_lib.temperature(per * 7 + per - 1, n_steps, S, T0, TN, "exp") == t(7)
    assert abs(t(S - 1) - TN / q) <= 1e-13 * TN


def test_cubic_schedule_closed_form(oracle_lib):
    T0, TN, S, n_steps = 1e-2, 1e-5, 1000, 50_000
    per = n_steps // S
    t = lambda n: oracle_lib.temperature(n * per, n_steps, S, T0, TN, "cubic")
    assert t(0) == T0
    assert abs(t(S // 2) - (T0 - (T0 - TN) / 8)) <= 1e-16
    # stage-to-stage drop (T0 - TN) ((n+1)^3 - n^3) / S^3, in exact arithmetic
    for n in (0, 1, 10, 400, 999 - 1):
        drop = Fraction(T0 - TN) * ((n + 1) ** 3 - n ** 3) / S ** 3
        assert abs(Fraction(t(n) - t(n + 1)) - drop) <= Fraction(4e-18)
    # slower than linear early on, ends at the same last-stage value family
    lin = lambda n: oracle_lib.temperature(n * per, n_steps, S, T0, TN, "linear")
    assert all(t(n) > lin(n) for n in range(1, S))
    assert abs(lin(S // 2) - (T0 - (T0 - TN) / 2)) <= 1e-16


def _costs(A, f, b, KU):
    r = A @ f - b
    return math.sqrt(float(r @ r) / KU)


def _draw(key, s, m, support, f, dmax, redraw):
    w = np_philox(key, [s, m, 0, 0])
    p = int(support[(int(w[0]) * len(support)) >> 64])
    fo = f[p]
    fn = fo + dmax * (2.0 * ((int(w[1]) >> 11) * TWO53) - 1.0)
    if redraw:
        j = 0
        while not (0.0 <= fn <= 1.0) and j < 256:
            j += 1
            w = np_philox(key, [s, m, 0, j])
            fn = fo + dmax * (2.0 * ((int(w[1]) >> 11) * TWO53) - 1.0)
        if not (0.0 <= fn <= 1.0):
            fn = fo
    else:
        fn = min(max(fn, 0.0), 1.0)
    return p, fn


def _temperature(schedule, s, n_steps, S, T0, TN):
    n = (s * S) // n_steps
    if schedule == "linear":
        return T0 - n * (T0 - TN) / S
    if schedule == "exp":
        return T0 * (TN / T0) ** (n / S)
    return T0 - n ** 3 * (T0 - TN) / S ** 3


@pytest.mark.parametrize("schedule,proposal", [("exp", "clamp"), ("cubic", "clamp"),
                                               ("linear", "redraw"), ("exp", "redraw")])
def test_chain_replay_schedules_and_redraw(oracle_lib, schedule, proposal):
    N, U, K = 8, 10, 13
    ang = datagen.angles_deg(U)
    ell = datagen.random_ellipses(5, N, 4)
    sino = datagen.radon_ellipses(ell, N, ang, K)
    mask = datagen.circle_mask(N)
    f0 = datagen.uniform_start(sino, mask, N)
    A = brute_clip.dense_system(N, U, K, ang, mask)
    b = sino.reshape(-1)
    KU = float(K * U)
    prm = dict(seed=13, chain_id=2, n_steps=400, n_stages=9, m_cand=3, T0=5e-3, TN=5e-6,
               delta_max=0.4, precision="f64", schedule=schedule, proposal=proposal)
    csr = oracle_lib.pila(N, U, K, ang, mask)
    f_or, st, tr = oracle_lib.sat_run(N, U, K, csr, sino, f0, mask=mask, **prm)
    support = np.flatnonzero(mask.reshape(-1))
    key = [prm["seed"], prm["chain_id"]]
    f = f0.reshape(-1).copy()
    for s in range(prm["n_steps"]):
        T = _temperature(schedule, s, prm["n_steps"], prm["n_stages"], prm["T0"], prm["TN"])
        C0 = _costs(A, f, b, KU)
        cands = [_draw(key, s, m, support, f, prm["delta_max"], proposal == "redraw")
                 for m in range(prm["m_cand"])]
        costs = []
        for p, fn in cands:
            fm = f.copy()
            fm[p] = fn
            costs.append(_costs(A, fm, b, KU))
        ms = int(tr["m_star"][s])
        assert costs[ms] <= min(costs) + 1e-12
        assert abs(tr["dC"][s] - (costs[ms] - C0)) <= 1e-11
        N1 = (int(np_philox(key, [s, 0, 1, 0])[0]) >> 11) * TWO53
        dC = float(tr["dC"][s])
        if not (dC > 0 and abs(N1 - math.exp(-dC / T)) < 1e-9):
            assert bool(tr["accept"][s]) == (dC <= 0.0 or N1 < math.exp(-dC / T))
        if tr["accept"][s]:
            p, fn = cands[ms]
            f[p] = fn
    assert np.array_equal(f.reshape(N, N), f_or)
    if proposal == "redraw":
        # redrawn values never land on the ends of the range
        moved = f_or.reshape(-1)[support] != f0.reshape(-1)[support]
        assert moved.any() and not np.any(np.isin(f_or.reshape(-1)[support][moved], [0.0, 1.0]))


# ---------------------------------------------------------------------------
# pixel-by-pixel SIRT
# ---------------------------------------------------------------------------

def test_sirt_seq_single_pixel_closed_form(oracle_lib):
    """One pixel, K = 1: each angle's ray crosses it with l_u and W_u = l_u^2,
    so one unrelaxed update moves f to the mean of Pm_u / l_u; with
    consistent data that is the true value."""
    U = 7
    ang = datagen.angles_deg(U)
    csr = oracle_lib.pila(1, U, 1, ang, None)
    ln = csr[2]
    assert len(ln) == U
    for u in range(U):
        c, s = abs(math.cos(math.radians(ang[u]))), abs(math.sin(math.radians(ang[u])))
        assert abs(ln[u] - 1.0 / max(c, s)) <= 1e-12
    sino = (0.37 * ln).reshape(U, 1)
    f, cost = oracle_lib.sirt_seq_run(1, U, 1, csr, sino, np.full((1, 1), 0.9), 1, 1, 1.0, seed=3)
    assert abs(f[0, 0] - 0.37) <= 1e-15 and cost[0] <= 1e-15


def test_sirt_seq_weighted_residual_descends(oracle_lib):
    """Each single-pixel update is a coordinate step on (1/2) sum_g r_g^2 / W_g
    whose length lambda/U is inside 2 / curvature (the curvature
    sum_e l_e^2 / W_e is at most the row length <= 2U), so the weighted
    residual never increases, update by update."""
    N, U, K = 8, 10, 13
    ang = datagen.angles_deg(U)
    mask = datagen.circle_mask(N)
    ell = datagen.random_ellipses(4, N, 4)
    sino = datagen.radon_ellipses(ell, N, ang, K)
    f0 = datagen.uniform_start(sino, mask, N)
    A = brute_clip.dense_system(N, U, K, ang, mask)
    W = (A * A).sum(axis=1)
    w = np.where(W > 0, 1.0 / np.where(W > 0, W, 1.0), 0.0)
    csr = oracle_lib.pila(N, U, K, ang, mask)
    for lam in (1.0, 0.3):
        vals = []
        for k in range(0, 120, 3):
            f, _ = oracle_lib.sirt_seq_run(N, U, K, csr, sino, f0, 1, k, lam, seed=8, mask=mask)
            r = A @ f.reshape(-1) - sino.reshape(-1)
            vals.append(float(r @ (w * r)))
        assert all(vals[i + 1] <= vals[i] * (1 + 1e-12) for i in range(len(vals) - 1))
        assert vals[-1] < 0.9 * vals[0]


def test_sirt_seq_fixed_point_and_running_projections(oracle_lib):
    N, U, K = 8, 16, 13
    ang = datagen.angles_deg(U)
    mask = datagen.circle_mask(N)
    A = brute_clip.dense_system(N, U, K, ang, mask)
    sup = np.flatnonzero(mask.reshape(-1))
    rng = np.random.default_rng(2)
    x = np.zeros(N * N)
    x[sup] = rng.random(len(sup))
    b = (A @ x).reshape(U, K)
    csr = oracle_lib.pila(N, U, K, ang, mask)
    # the weighted least-squares solution (here the truth) does not move
    f, cost = oracle_lib.sirt_seq_run(N, U, K, csr, b, x.reshape(N, N), 3, 200, 1.0, seed=1, mask=mask)
    assert np.max(np.abs(f.reshape(-1) - x)) <= 1e-12 and np.all(cost <= 1e-12)
    # from the uniform start it converges to that solution, and its running
    # projections match a dense projection of its image
    f0 = datagen.uniform_start(b, mask, N)
    f, cost = oracle_lib.sirt_seq_run(N, U, K, csr, b, f0, 30000, len(sup), 1.0, seed=4, mask=mask)
    assert np.max(np.abs(f.reshape(-1)[sup] - x[sup])) <= 1e-9
    r = A @ f.reshape(-1) - b.reshape(-1)
    assert abs(cost[-1] - math.sqrt(float(r @ r) / (U * K))) <= 1e-12


# ---------------------------------------------------------------------------
# bilinear DRT and the SAT that uses it
# ---------------------------------------------------------------------------

def _scipy_drt(N, U, K, ang, f):
    T = int(math.ceil(N / math.sqrt(2.0))) + 1
    t = np.arange(-T, T + 1, dtype=np.float64)
    out = np.zeros((U, K))
    img = np.asarray(f, np.float64).reshape(N, N)
    for u in range(U):
        c, s = brute_clip.trig(float(ang[u]))
        for k in range(K):
            sk = k - (K - 1) / 2.0
            x = sk * c - t * s
            y = sk * s + t * c
            cols = x + N / 2.0 - 0.5
            rows = N / 2.0 - 0.5 - y
            out[u, k] = ndimage.map_coordinates(img, [rows, cols], order=1, mode="grid-constant",
                                                cval=0.0).sum()
    return out


@pytest.mark.parametrize("N,U,K", [(8, 7, 13), (11, 12, 17), (16, 5, 24)])
def test_drt_matches_scipy_bilinear(oracle_lib, N, U, K):
    ang = datagen.angles_deg(U)
    f = np.random.default_rng(N).random((N, N))
    assert oracle_lib.drt_half_span(N) == int(math.ceil(N / math.sqrt(2.0))) + 1
    d = oracle_lib.drt(N, U, K, ang, f)
    ref = _scipy_drt(N, U, K, ang, f)
    assert np.max(np.abs(d - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_drt_constant_image_axis_rays(oracle_lib):
    """A constant image c: at 0 and 90 degrees the samples fall on pixel
    centre lines midway between rows (N even), the bilinear image is c inside
    the outermost centres and ramps to 0 over the last half pixel, so a ray
    through the interior sums to N c exactly."""
    N, K = 12, 12
    ang = np.array([0.0, 90.0])
    d = oracle_lib.drt(N, 2, K, ang, np.full((N, N), 0.7))
    # bins whose ray lies between the outermost pixel centres
    inner = [k for k in range(K) if abs(k - (K - 1) / 2.0) <= N / 2.0 - 0.5]
    for u in range(2):
        for k in inner:
            assert abs(d[u, k] - 0.7 * N) <= 1e-13


def test_satdrt_chain_replay(oracle_lib):
    N, U, K = 6, 6, 9
    ang = datagen.angles_deg(U)
    ell = datagen.random_ellipses(2, N, 3)
    sino = datagen.radon_ellipses(ell, N, ang, K)
    f0 = np.full((N, N), float(sino.sum()) / U / (N * N))
    prm = dict(seed=4, chain_id=0, n_steps=60, n_stages=6, m_cand=2, T0=3e-3, TN=3e-6,
               delta_max=0.3)
    f_or, cf, tr = oracle_lib.satdrt_run(N, U, K, ang, sino, f0, **prm)
    support = np.arange(N * N)
    key = [prm["seed"], prm["chain_id"]]
    f = f0.reshape(-1).copy()
    KU = float(U * K)

    def cost(img):
        r = _scipy_drt(N, U, K, ang, img) - sino
        return math.sqrt(float((r * r).sum()) / KU)

    C = cost(f)
    for s in range(prm["n_steps"]):
        cands = [_draw(key, s, m, support, f, prm["delta_max"], False) for m in range(2)]
        cs = []
        for p, fn in cands:
            fm = f.copy()
            fm[p] = fn
            cs.append(cost(fm))
        ms = int(tr["m_star"][s])
        assert cs[ms] <= min(cs) + 1e-12
        assert abs(tr["dC"][s] - (cs[ms] - C)) <= 1e-11
        T = _temperature("linear", s, prm["n_steps"], prm["n_stages"], prm["T0"], prm["TN"])
        N1 = (int(np_philox(key, [s, 0, 1, 0])[0]) >> 11) * TWO53
        dC = float(tr["dC"][s])
        assert bool(tr["accept"][s]) == (dC <= 0.0 or N1 < math.exp(-dC / T))
        if tr["accept"][s]:
            f[cands[ms][0]] = cands[ms][1]
            C = cs[ms]
    assert np.array_equal(f.reshape(N, N), f_or)
    assert abs(cf - C) <= 1e-12
    assert 0 < int(tr["accept"].sum()) < prm["n_steps"]


# ---------------------------------------------------------------------------
# one-byte lengths
# ---------------------------------------------------------------------------

def test_u8_quantiser_bound_and_values(oracle_lib):
    q = np.arange(256, dtype=np.uint8)
    v = oracle_lib.dequantize_u8(q)
    assert np.array_equal(v, (q.astype(np.float32) / np.float32(180.0)).astype(np.float64))
    for k in range(256):
        assert abs(Fraction(float(v[k])) - Fraction(k, 180)) <= Fraction(k, 180) * Fraction(2) ** -24
    for N, U, K in ((16, 30, 23), (24, 45, 35)):
        ang = datagen.angles_deg(U)
        row_ptr, col, ln = oracle_lib.pila(N, U, K, ang, None)
        qq = oracle_lib.quantize_u8(ln)
        assert qq.max() <= 255
        assert np.all(np.abs(ln - qq / 180.0) <= 1.0 / 360.0 + 1e-15)
        # projections with one-byte lengths stay within sum |f| / 360 (+ float rounding)
        f = np.random.default_rng(1).random(N * N)
        lq = oracle_lib.dequantize_u8(qq)
        exact = oracle_lib.forward(N, U, K, (row_ptr, col, ln), f).reshape(-1)
        quant = oracle_lib.forward(N, U, K, (row_ptr, col, lq), f).reshape(-1)
        absf = oracle_lib.forward(N, U, K, (row_ptr, col, np.ones_like(ln)), f).reshape(-1)
        assert np.all(np.abs(quant - exact) <= absf * (1.0 / 360.0 + 2.0 ** -23) + 1e-12)
