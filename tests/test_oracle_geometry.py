"""Pins of the oracle's generator, PILA and projection (CPU only).

The PILA (section II-B, Eq. 5) is pinned three ways: hand-derived lengths on
a 2 x 2 grid, brute-force Liang-Barsky clipping of every ray against every
pixel, and the exact chord of the whole square.  Eq. 1 projection is pinned
by the chord of an off-centre disk (orientation and angle sense).
"""
import math
import os

import numpy as np
import pytest

import brute_clip
import datagen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def np_philox(key, ctr):
    """numpy's Philox4x64-10 block at counter ctr (numpy pre-increments)."""
    c = sum(int(x) << (64 * i) for i, x in enumerate(ctr))
    c = (c - 1) % (1 << 256)
    words = [(c >> (64 * i)) & ((1 << 64) - 1) for i in range(4)]
    bg = np.random.Philox(key=np.array([int(key[0]), int(key[1])], dtype=np.uint64),
                          counter=np.array(words, dtype=np.uint64))
    return bg.random_raw(4)


def test_philox_matches_numpy(oracle_lib):
    rng = np.random.default_rng(7)
    for _ in range(200):
        key = rng.integers(0, 2**63, size=2, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, size=2, dtype=np.uint64)
        ctr = rng.integers(0, 2**63, size=4, dtype=np.uint64)
        ctr[0] += np.uint64(1)
        assert np.array_equal(oracle_lib.philox(key, ctr), np_philox(key, ctr))
    # small counters as the chain uses them: (step, slot, purpose, 0)
    for s in (0, 1, 2, 4095, 10**7):
        for m in (0, 1, 63):
            for purpose in (0, 1, 2):
                assert np.array_equal(oracle_lib.philox([1001, 0], [s, m, purpose, 0]),
                                      np_philox([1001, 0], [s, m, purpose, 0]))


def _csr_to_dense(N, U, K, csr):
    row_ptr, col, ln = csr
    A = np.zeros((U * K, N * N))
    for p in range(N * N):
        for e in range(row_ptr[p], row_ptr[p + 1]):
            assert A[col[e], p] == 0.0, "duplicate (pixel, ray) entry"
            A[col[e], p] = ln[e]
    return A


def test_pila_golden_2x2(oracle_lib):
    N, U, K = 2, 4, 3
    rows = np.loadtxt(os.path.join(GOLDEN, "pila_2x2_u4_k3.txt"), comments="#")
    row_ptr, col, ln = oracle_lib.pila(N, U, K, datagen.angles_deg(U))
    got = sorted((p, int(col[e]) // K, int(col[e]) % K, float(ln[e]))
                 for p in range(N * N) for e in range(row_ptr[p], row_ptr[p + 1]))
    want = sorted((int(a), int(b), int(c), float(d)) for a, b, c, d in rows)
    assert [g[:3] for g in got] == [w[:3] for w in want]
    for g, w in zip(got, want):
        assert abs(g[3] - w[3]) <= 1e-14


@pytest.mark.parametrize("N,U,K", [(8, 4, 8), (8, 8, 11), (8, 90, 12), (16, 180, 23),
                                   (16, 8, 16), (7, 90, 10), (9, 180, 13), (16, 12, 17),
                                   (5, 36, 7)])
def test_pila_matches_bruteforce(oracle_lib, N, U, K):
    ang = datagen.angles_deg(U)
    A_bf = brute_clip.dense_system(N, U, K, ang)
    csr = oracle_lib.pila(N, U, K, ang)
    A_or = _csr_to_dense(N, U, K, csr)
    assert np.array_equal(A_bf > 0, A_or > 0), "index sets differ"
    assert np.max(np.abs(A_bf - A_or)) <= 1e-12
    # rows ordered by ray index
    row_ptr, col, _ = csr
    for p in range(N * N):
        seg = col[row_ptr[p]:row_ptr[p + 1]]
        assert np.all(np.diff(seg) > 0)


def test_pila_matches_bruteforce_masked(oracle_lib):
    N, U, K = 12, 30, 17
    ang = datagen.angles_deg(U)
    mask = datagen.circle_mask(N)
    A_bf = brute_clip.dense_system(N, U, K, ang, mask)
    A_or = _csr_to_dense(N, U, K, oracle_lib.pila(N, U, K, ang, mask))
    assert np.array_equal(A_bf > 0, A_or > 0)
    assert np.max(np.abs(A_bf - A_or)) <= 1e-12


def test_pila_bruteforce_odd_angles(oracle_lib):
    # angles that are not of the form u*180/U, including negative and > 180
    ang = np.array([-30.0, 0.0, 12.5, 45.0, 90.0, 135.0, 180.0, 200.0, 270.0, 333.3])
    N, K = 10, 15
    A_bf = brute_clip.dense_system(N, len(ang), K, ang)
    A_or = _csr_to_dense(N, len(ang), K, oracle_lib.pila(N, len(ang), K, ang))
    assert np.array_equal(A_bf > 0, A_or > 0)
    assert np.max(np.abs(A_bf - A_or)) <= 1e-12


@pytest.mark.parametrize("N,U,K", [(64, 90, 64), (256, 180, 367), (63, 45, 91)])
def test_square_chord_exact(oracle_lib, N, U, K):
    """All-ones image: each ray's projection is its chord through the square."""
    ang = datagen.angles_deg(U)
    csr = oracle_lib.pila(N, U, K, ang)
    P = oracle_lib.forward(N, U, K, csr, np.ones((N, N)))
    cs = oracle_lib.trig(ang)
    sk = datagen.bin_centres(K)
    want = np.array([[brute_clip.slab_length(N, cs[u, 0], cs[u, 1], sk[k]) for k in range(K)]
                     for u in range(U)])
    assert np.max(np.abs(P - want)) <= 1e-12 * N


def test_square_chord_large_grid_subset(oracle_lib):
    """The 1024 x 1024, 1449-bin geometry on a few of its angles."""
    N, K = 1024, 1449
    ang = np.array([0.0, 0.25, 44.75, 45.0, 89.75, 90.0, 137.5])
    U = len(ang)
    csr = oracle_lib.pila(N, U, K, ang)
    P = oracle_lib.forward(N, U, K, csr, np.ones((N, N)))
    cs = oracle_lib.trig(ang)
    sk = datagen.bin_centres(K)
    want = np.array([[brute_clip.slab_length(N, cs[u, 0], cs[u, 1], sk[k]) for k in range(K)]
                     for u in range(U)])
    assert np.max(np.abs(P - want)) <= 1e-12 * N


@pytest.mark.parametrize("N,U,K", [(64, 90, 64), (32, 180, 46), (33, 60, 47)])
def test_pila_invariants(oracle_lib, N, U, K):
    ang = datagen.angles_deg(U)
    row_ptr, col, ln = oracle_lib.pila(N, U, K, ang)
    cs = oracle_lib.trig(ang)
    u_of = col // K
    bound = 1.0 / np.maximum(np.abs(cs[:, 0]), np.abs(cs[:, 1]))
    assert np.all(ln > 1e-9)
    assert np.all(ln <= bound[u_of] + 1e-12)
    assert np.all(ln <= math.sqrt(2.0) + 1e-12)
    axis = (np.fmod(ang, 90.0) == 0.0)[u_of]
    assert np.all(ln[axis] == 1.0)
    # at most two rays per (pixel, angle)
    pix = np.repeat(np.arange(N * N), np.diff(row_ptr))
    key = pix.astype(np.int64) * U + u_of
    _, counts = np.unique(key, return_counts=True)
    assert counts.max() <= 2


def _disk_fractions(N, x0, y0, R, ss=64):
    """Area fraction of each pixel covered by the disk (supersampled)."""
    h = N / 2.0
    v = np.zeros((N, N))
    off = (np.arange(ss) + 0.5) / ss
    for i in range(N):
        yb = h - 1 - i
        for j in range(N):
            xl = j - h
            # corners: fully inside / outside decided exactly
            cx = np.array([xl, xl + 1.0])
            cy = np.array([yb, yb + 1.0])
            dmin = math.hypot(max(cx[0] - x0, 0, x0 - cx[1]), max(cy[0] - y0, 0, y0 - cy[1]))
            dmax = math.hypot(max(abs(cx[0] - x0), abs(cx[1] - x0)), max(abs(cy[0] - y0), abs(cy[1] - y0)))
            if dmax <= R:
                v[i, j] = 1.0
            elif dmin >= R:
                v[i, j] = 0.0
            else:
                X = xl + off[None, :]
                Y = yb + off[:, None]
                v[i, j] = np.mean((X - x0) ** 2 + (Y - y0) ** 2 <= R * R)
    return v


@pytest.mark.parametrize("R", [6.0, 12.0, 20.0])
def test_disk_chord(oracle_lib, R):
    """Projection of an off-centre disk against the chord 2 sqrt(R^2 - d^2).

    Uncut pixels contribute their exact chord piece; a cut pixel contributes
    l * v instead of a true piece in [0, l], so |P - chord| is bounded by the
    sum of l * max(v, 1 - v) over cut pixels plus the sampling error.
    """
    N, U, K = 64, 36, 64
    x0, y0 = 7.3, -4.1
    ang = datagen.angles_deg(U)
    csr = oracle_lib.pila(N, U, K, ang)
    v = _disk_fractions(N, x0, y0, R)
    P = oracle_lib.forward(N, U, K, csr, v)
    cut = ((v > 0) & (v < 1)).astype(float)
    wcut = cut * np.maximum(v, 1 - v) + cut * (2.0 * 64 + 4) / 64 ** 2
    bound = oracle_lib.forward(N, U, K, csr, wcut)
    cs = oracle_lib.trig(ang)
    sk = datagen.bin_centres(K)
    d = sk[None, :] - (x0 * cs[:, 0][:, None] + y0 * cs[:, 1][:, None])
    chord = 2.0 * np.sqrt(np.maximum(R * R - d * d, 0.0))
    err = np.abs(P - chord)
    assert np.all(err <= bound + 1e-9)
    # each projection is centred where the disk centre projects (orientation
    # and angle-sense pin): first moment over the bins
    centroid = (P * sk[None, :]).sum(axis=1) / P.sum(axis=1)
    assert np.max(np.abs(centroid - (x0 * cs[:, 0] + y0 * cs[:, 1]))) <= 0.05


def test_backward_is_transpose(oracle_lib):
    N, U, K = 12, 20, 17
    ang = datagen.angles_deg(U)
    csr = oracle_lib.pila(N, U, K, ang)
    rng = np.random.default_rng(3)
    f = rng.random((N, N))
    y = rng.random((U, K))
    lhs = float(np.sum(oracle_lib.forward(N, U, K, csr, f) * y))
    rhs = float(np.sum(f * oracle_lib.backward(N, csr, y)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    A = brute_clip.dense_system(N, U, K, ang)
    assert np.max(np.abs(oracle_lib.forward(N, U, K, csr, f).reshape(-1) - A @ f.reshape(-1))) <= 1e-11


def test_ray_listing_matches_pila(oracle_lib):
    N, U, K = 16, 12, 23
    ang = datagen.angles_deg(U)
    (row_ptr, col, ln), (off, pix, rl) = oracle_lib.pila(N, U, K, ang, with_rays=True)
    assert off[-1] == row_ptr[-1]
    A1 = np.zeros((U * K, N * N))
    for g in range(U * K):
        A1[g, pix[off[g]:off[g + 1]]] = rl[off[g]:off[g + 1]]
    assert np.array_equal(A1, _csr_to_dense(N, U, K, (row_ptr, col, ln)))


def _exact_chord(N, c, s, sk, i, j):
    """Chord of the line x c + y s = sk through pixel (i, j), exact rationals.

    c, s are the double values used by the implementations (so c^2 + s^2 is
    1 only up to rounding); the foot point sk (c, s) / (c^2 + s^2) lies
    exactly on the line, the parametric interval is exact, and it is scaled
    by |(c, s)| at the end.
    """
    from fractions import Fraction as F
    h = F(N, 2)
    x0, y0 = F(j) - h, h - 1 - F(i)
    c, s, sk = F(c), F(s), F(sk)
    rho2 = c * c + s * s
    px, py, dx, dy = sk * c / rho2, sk * s / rho2, -s, c
    ta, tb = (x0 - px) / dx, (x0 + 1 - px) / dx
    tc, td = (y0 - py) / dy, (y0 + 1 - py) / dy
    lo = max(min(ta, tb), min(tc, td))
    hi = min(max(ta, tb), max(tc, td))
    if hi <= lo:
        return 0.0
    return float(hi - lo) * math.sqrt(float(rho2))


@pytest.mark.parametrize("N,K,deg", [(1024, 1449, 0.25), (1024, 1449, 89.75), (1024, 1449, 44.75),
                                     (1024, 1449, 92.25), (1024, 1449, 1.0), (512, 725, 0.5),
                                     (256, 367, 1.0), (10, 15, 1e-3)])
def test_lengths_exact_rational_large_grid(oracle_lib, N, K, deg):
    """Near-axis rays on large grids: lengths within 1e-13 of exact arithmetic."""
    cs = oracle_lib.trig([deg])[0]
    rng = np.random.default_rng(int(deg * 100) + N)
    worst = 0.0
    for k in rng.choice(K, size=6, replace=False):
        pix, ln = oracle_lib.trace_ray(N, K, deg, int(k))
        for q in rng.choice(len(pix), size=min(40, len(pix)), replace=False) if len(pix) else []:
            p = int(pix[q])
            ex = _exact_chord(N, cs[0], cs[1], k - (K - 1) / 2.0, p // N, p % N)
            worst = max(worst, abs(ex - ln[q]))
    assert worst <= 1e-13


def test_pixel_row_matches_full_pila(oracle_lib):
    N, U, K = 24, 30, 35
    ang = datagen.angles_deg(U)
    mask = datagen.circle_mask(N)
    row_ptr, col, ln = oracle_lib.pila(N, U, K, ang, mask)
    for p in range(0, N * N, 7):
        g, l = oracle_lib.pixel_row(N, U, K, ang, p, mask)
        assert np.array_equal(g, col[row_ptr[p]:row_ptr[p + 1]])
        assert np.array_equal(l, ln[row_ptr[p]:row_ptr[p + 1]])
