"""Pins of the oracle's FP32-residual chain mode (CPU only).

The FP32 mode approximates the FP64 chain by design, so it is pinned by
rounding-error bounds rather than bit equality:

* each FP32 row sum (Eq. 7's inner sum with float operands and float
  accumulation) against the exact rational value of the same sum with the
  unrounded change and lengths, within the bound of its roundings;
* the running residual against a from-scratch dense residual built by
  brute-force clipping (independent of the oracle's PILA): equal to one
  float rounding right after a resync, and within the accumulated rounding
  of the updates applied to each ray when no resync runs.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import brute_clip
import datagen
from test_oracle_geometry import np_philox

U32 = 2.0 ** -24  # unit roundoff of float


def _gamma(n, u=U32):
    return n * u / (1.0 - n * u)


def _problem(N, U, K, seed, noise=1e4):
    ang = datagen.angles_deg(U)
    ell = datagen.random_ellipses(seed, N, 5)
    sino = datagen.radon_ellipses(ell, N, ang, K)
    if noise:
        sino = datagen.poisson_noise(sino, N, noise, seed + 1)
    mask = datagen.circle_mask(N)
    f0 = datagen.uniform_start(sino, mask, N)
    return ang, sino, mask, f0


@pytest.mark.parametrize("N,U,K", [(16, 30, 23), (24, 90, 35)])
def test_fp32_row_sum_within_rounding_bound(oracle_lib, N, U, K):
    ang = datagen.angles_deg(U)
    csr = oracle_lib.pila(N, U, K, ang, None)
    row_ptr, col, ln = csr
    rng = np.random.default_rng(N + U)
    r32 = (rng.standard_normal(U * K) * 3.0).astype(np.float32)
    worst = 0.0
    for trial in range(60):
        p = int(rng.integers(N * N))
        d = float(rng.uniform(-0.05, 0.05))
        S32 = oracle_lib.delta_sse(csr, r32, p, d, fp32=True)
        exact = Fraction(0)
        mag = 0.0
        absterms = 0.0
        n = 0
        for e in range(row_ptr[p], row_ptr[p + 1]):
            t = Fraction(d) * Fraction(float(ln[e]))
            x = 2 * Fraction(float(r32[col[e]])) + t
            exact += t * x
            absterms += abs(float(t * x))
            mag += abs(float(t)) * (2.0 * abs(float(r32[col[e]])) + abs(float(t)))
            n += 1
        # per term: the change, the length, their product, the sum 2r + t and
        # the product with it are rounded to float (10u covers the second-order
        # terms); the running float sum adds gamma_n times the sum of |terms|
        bound = (10.0 * U32 + 1.01 * _gamma(n)) * mag
        err = abs(Fraction(S32) - exact)
        assert float(err) <= bound, (p, d, float(err), bound)
        worst = max(worst, float(err) / bound if bound else 0.0)
        # the FP64 sum of the same operands: gamma_n of the FP64 unit roundoff
        S64, a64 = oracle_lib.delta_sse(csr, r32.astype(np.float64), p, d)
        assert float(abs(Fraction(S64) - exact)) <= 3 * _gamma(n + 3, 2.0 ** -53) * mag + 1e-300
        assert abs(a64 - absterms) <= 1e-12 * absterms + 1e-300
    assert worst > 0.0  # the float path really rounds


def _dense_f32(N, U, K, ang, mask):
    A = brute_clip.dense_system(N, U, K, ang, mask)
    return A.astype(np.float32).astype(np.float64)


def test_fp32_residual_exact_after_every_resync(oracle_lib):
    """resync_every = 1: every accepted nonzero change is followed by an FP64
    recomputation, so the final running residual is the float rounding of
    A f - Pm (lengths as floats) and the running SSE its exact sum of squares."""
    N, U, K = 12, 20, 19
    ang, sino, mask, f0 = _problem(N, U, K, seed=3)
    csr = oracle_lib.pila(N, U, K, ang, mask)
    f, st, tr, r = oracle_lib.sat_run(N, U, K, csr, sino, f0, mask=mask, residual=True, seed=5,
                                      n_steps=3000, n_stages=20, m_cand=4, T0=None, q_auto=40,
                                      delta_max=0.05, precision="f32", resync_every=1)
    assert st["resyncs"] == st["accepts_nonzero"] > 100
    A = _dense_f32(N, U, K, ang, mask)
    terms = np.abs(A) @ np.abs(f.reshape(-1)) + np.abs(sino.reshape(-1))
    r_dense = A @ f.reshape(-1) - sino.reshape(-1)
    err = np.abs(r.reshape(-1) - r_dense)
    assert np.all(err <= U32 * np.abs(r_dense) + 1e-12 * terms + 1e-300)
    sse = float(r_dense @ r_dense)
    assert abs(st["sse_final"] - sse) <= 1e-10 * sse


def test_fp32_residual_drift_within_accumulated_rounding(oracle_lib):
    """No resync: every ray's running FP32 residual differs from the dense
    residual of the final image by at most the roundings of the updates it
    received (u |r| for the sum, gamma_3 |d l| for the float change times the
    float length) plus the first rounding of r0.  A missed, doubled or
    mis-indexed update would be off by a whole |d l| (about 1e-2)."""
    N, U, K = 12, 24, 19
    ang, sino, mask, f0 = _problem(N, U, K, seed=7)
    csr = oracle_lib.pila(N, U, K, ang, mask)
    prm = dict(seed=9, chain_id=1, n_steps=4000, n_stages=20, m_cand=3, T0=None, q_auto=40,
               delta_max=0.05, precision="f32", resync_every=0)
    f, st, tr, r = oracle_lib.sat_run(N, U, K, csr, sino, f0, mask=mask, residual=True, **prm)
    assert st["resyncs"] == 0 and st["accepts_nonzero"] > 200
    A = _dense_f32(N, U, K, ang, mask)
    r_dense = A @ f.reshape(-1) - sino.reshape(-1)
    # replay which pixels changed (independent generator) to count each ray's updates
    support = np.flatnonzero(mask.reshape(-1))
    fr = f0.reshape(-1).copy()
    n_upd = np.zeros(U * K)
    for s in range(prm["n_steps"]):
        if not tr["accept"][s]:
            continue
        w = np_philox([prm["seed"], prm["chain_id"]], [s, int(tr["m_star"][s]), 0, 0])
        p = int(support[(int(w[0]) * len(support)) >> 64])
        delta = prm["delta_max"] * (2.0 * ((int(w[1]) >> 11) * 2.0 ** -53) - 1.0)
        fn = min(max(fr[p] + delta, 0.0), 1.0)
        if fn != fr[p]:
            n_upd += A[:, p] != 0
            fr[p] = fn
    assert np.array_equal(fr, f.reshape(-1))
    R = float(np.max(np.abs(r_dense))) + 1.0
    dl = prm["delta_max"] * math.sqrt(2.0) * 1.01
    bound = U32 * (np.abs(sino.reshape(-1)) + R) + n_upd * (U32 * R + _gamma(3) * dl) + 1e-12
    err = np.abs(r.reshape(-1) - r_dense)
    assert np.all(err <= bound), float(np.max(err / bound))
    assert np.max(err) > 0.0
