"""Checks of the seeded input generators (CPU only)."""
import math

import numpy as np

import datagen


def _ellipse_projection(cx, cy, a, b, th, g, alpha, s):
    """Closed-form Radon transform of a uniform ellipse."""
    p = s - (cx * math.cos(alpha) + cy * math.sin(alpha))
    a2 = (a * math.cos(alpha - th)) ** 2 + (b * math.sin(alpha - th)) ** 2
    if p * p >= a2:
        return 0.0
    return g * 2.0 * a * b * math.sqrt(a2 - p * p) / a2


def test_single_ellipse_closed_form():
    ell = np.array([[3.5, -2.0, 9.0, 4.0, 0.7, 0.8]])
    N, U, K = 32, 17, 45
    ang = datagen.angles_deg(U)
    P = datagen.radon_ellipses(ell, N, ang, K)
    sk = datagen.bin_centres(K)
    want = np.array([[_ellipse_projection(*ell[0], math.radians(ang[u]), sk[k]) for k in range(K)]
                     for u in range(U)])
    assert np.max(np.abs(P - want)) <= 1e-11


def test_overwrite_painting():
    # inner ellipse painted after (on top of) the outer one
    outer = [0.0, 0.0, 10.0, 8.0, 0.3, 0.4]
    inner = [1.0, 0.5, 4.0, 3.0, 1.1, 0.9]
    ell = np.array([outer, inner])
    N, U, K = 32, 9, 45
    ang = datagen.angles_deg(U)
    P = datagen.radon_ellipses(ell, N, ang, K)
    sk = datagen.bin_centres(K)
    for u in range(U):
        al = math.radians(ang[u])
        for k in range(K):
            want = (_ellipse_projection(*outer, al, sk[k])
                    + _ellipse_projection(*inner[:5], inner[5] - outer[5], al, sk[k]))
            assert abs(P[u, k] - want) <= 1e-10


def test_phantom_reproducible_and_in_range():
    a = datagen.random_ellipses(101, 64, 10)
    b = datagen.random_ellipses(101, 64, 10)
    assert np.array_equal(a, b)
    img = datagen.rasterize(a, 64)
    assert img.min() >= 0.0 and img.max() <= 1.0
    # every ellipse lies inside the inscribed circle
    for cx, cy, ea, eb, th, g in a:
        assert math.hypot(cx, cy) + max(ea, eb) < 32.0
    mask = datagen.circle_mask(64)
    assert np.all(img[mask == 0] == 0.0)


def test_mask_sizes():
    for N in (64, 128, 256, 512, 1024):
        P = int(datagen.circle_mask(N).sum())
        assert abs(P - math.pi * N * N / 4) <= 2.5 * N


def test_noise_reproducible():
    ell = datagen.random_ellipses(102, 32, 5)
    P = datagen.radon_ellipses(ell, 32, datagen.angles_deg(12), 46)
    n1 = datagen.poisson_noise(P, 32, 1e4, 202)
    n2 = datagen.poisson_noise(P, 32, 1e4, 202)
    assert np.array_equal(n1, n2)
    # noise is small relative to the signal at I0 = 1e4
    assert np.sqrt(np.mean((n1 - P) ** 2)) < 0.05 * np.max(P) + 1.0


def test_uniform_start_mass():
    ell = datagen.random_ellipses(7, 48, 6)
    N, U, K = 48, 30, 68
    P = datagen.radon_ellipses(ell, N, datagen.angles_deg(U), K)
    mask = datagen.circle_mask(N)
    f0 = datagen.uniform_start(P, mask, N)
    truth = datagen.rasterize(ell, N, ss=8)
    c = f0[mask != 0][0]
    assert np.all(f0[mask == 0] == 0.0)
    assert abs(c - truth.sum() / mask.sum()) <= 0.01 * c + 1e-6


def test_volume_slices():
    sl = datagen.batch_slices(3, 6, (32, 48), (12, 18), 1e4)
    assert len(sl) == 6
    for s in sl:
        assert s.sino.shape == (s.U, s.K)
        assert s.K == datagen.n_bins_for(s.N)
        assert s.truth.min() >= 0 and s.truth.max() <= 1
