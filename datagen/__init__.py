"""Seeded synthetic inputs for parallel-beam simulated annealing tomography.

This module is the only code shared by the CPU oracle and the HIP path, and
it holds none of the method's arithmetic: no intersection lengths, no
projection through a pixel grid, no cost, no annealing.  It draws phantoms
(random ellipses, or slices of random ellipsoids), computes their *analytic*
line integrals (the continuous Radon transform of a piecewise-constant
object, which is how a physical scanner sees it, not the discrete pixel sum
of Eq. 1), adds photon noise, and builds masks and starting images.

Geometry conventions used for the rays (the paper leaves them open; they are
shared with both implementations as part of the problem statement):

* The image is N x N unit pixels centred on the rotation axis; x points right,
  y points up, pixel (i, j) (row i from the top) covers
  x in [j - N/2, j - N/2 + 1), y in [N/2 - 1 - i, N/2 - i).
* Angle u is alpha_u = u * 180 / U degrees (U angles uniform in [0, 180)).
* Detector bin k (K bins at unit spacing) carries the ray
  x cos(alpha) + y sin(alpha) = s_k with s_k = k - (K - 1) / 2.

Phantom values lie in [0, 1] (the gray range used by the paper's examples,
section III).  The paper's own phantoms are figures that are not available,
so these seeded phantoms stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

__all__ = [
    "angles_deg", "n_bins_for", "bin_centres", "circle_mask", "random_ellipses",
    "rasterize", "radon_ellipses", "poisson_noise", "uniform_start",
    "random_ellipsoids", "volume_slice", "Slice", "make_slice", "CONFIGS",
    "nrmse", "rmse",
]


# ---------------------------------------------------------------------------
# geometry of the measurement (problem statement, not method)
# ---------------------------------------------------------------------------

def angles_deg(U: int) -> np.ndarray:
    """U projection angles uniform in [0, 180) degrees: u * 180 / U."""
    return np.array([u * 180.0 / U for u in range(U)], dtype=np.float64)


def n_bins_for(N: int) -> int:
    """Detector bins that cover the image diagonal: ceil(sqrt(2) N)."""
    return int(math.ceil(math.sqrt(2.0) * N))


def bin_centres(K: int) -> np.ndarray:
    """Signed detector coordinate of each bin centre, s_k = k - (K-1)/2."""
    return np.arange(K, dtype=np.float64) - (K - 1) / 2.0


def circle_mask(N: int) -> np.ndarray:
    """Support mask: pixels whose centre lies inside the inscribed circle."""
    h = N / 2.0
    c = np.arange(N, dtype=np.float64) - h + 0.5
    x = c[None, :]
    y = -c[:, None]
    return ((x * x + y * y) <= h * h).astype(np.uint8)


# ---------------------------------------------------------------------------
# phantoms
# ---------------------------------------------------------------------------

def random_ellipses(seed: int, N: int, n_ell: int) -> np.ndarray:
    """n_ell random ellipses in pixel units, painted in order (later on top).

    Rows are (cx, cy, a, b, theta, gray).  Centres are uniform in the disk of
    radius 0.6 N/2, semi-axes uniform in [0.05, 0.35] N/2, so every ellipse
    lies inside the inscribed circle; theta uniform in [0, pi); gray uniform
    in [0, 1].
    """
    rng = np.random.default_rng(seed)
    h = N / 2.0
    out = np.empty((n_ell, 6), dtype=np.float64)
    for e in range(n_ell):
        rad = 0.6 * h * math.sqrt(rng.random())
        phi = 2.0 * math.pi * rng.random()
        out[e, 0] = rad * math.cos(phi)
        out[e, 1] = rad * math.sin(phi)
        out[e, 2] = (0.05 + 0.30 * rng.random()) * h
        out[e, 3] = (0.05 + 0.30 * rng.random()) * h
        out[e, 4] = math.pi * rng.random()
        out[e, 5] = rng.random()
    return out


def rasterize(ell: np.ndarray, N: int, ss: int = 4) -> np.ndarray:
    """Pixel phantom: mean of the painted object over ss x ss sub-samples."""
    h = N / 2.0
    off = (np.arange(ss, dtype=np.float64) + 0.5) / ss
    xs = (np.arange(N, dtype=np.float64)[:, None] - h + off[None, :]).reshape(-1)
    ys = (h - np.arange(N, dtype=np.float64)[:, None] - off[None, :]).reshape(-1)
    img = np.zeros((N * ss, N * ss), dtype=np.float64)
    X = xs[None, :]
    Y = ys[:, None]
    for cx, cy, a, b, th, g in ell:
        ct, st = math.cos(th), math.sin(th)
        dx = X - cx
        dy = Y - cy
        u = (dx * ct + dy * st) / a
        v = (-dx * st + dy * ct) / b
        img[(u * u + v * v) <= 1.0] = g
    return img.reshape(N, ss, N, ss).mean(axis=(1, 3))


def _ellipse_intervals(ell: np.ndarray, cth: np.ndarray, sth: np.ndarray,
                       s: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Parameter interval [t0, t1] of each ray inside each ellipse.

    A ray is the point set (s cos - t sin, s sin + t cos), t real.  Returns
    arrays (R, E); rays that miss an ellipse get t0 = t1 = 0.
    """
    R = s.shape[0]
    E = ell.shape[0]
    t0 = np.zeros((R, E))
    t1 = np.zeros((R, E))
    px = (s * cth)[:, None] - ell[None, :, 0]
    py = (s * sth)[:, None] - ell[None, :, 1]
    dx = -sth[:, None]
    dy = cth[:, None]
    ce = np.cos(ell[:, 4])[None, :]
    se = np.sin(ell[:, 4])[None, :]
    a = ell[:, 2][None, :]
    b = ell[:, 3][None, :]
    qx = (px * ce + py * se) / a
    qy = (-px * se + py * ce) / b
    ex = (dx * ce + dy * se) / a
    ey = (-dx * se + dy * ce) / b
    A = ex * ex + ey * ey
    B = 2.0 * (qx * ex + qy * ey)
    C = qx * qx + qy * qy - 1.0
    disc = B * B - 4.0 * A * C
    hit = disc > 0.0
    sq = np.sqrt(np.where(hit, disc, 0.0))
    t0 = np.where(hit, (-B - sq) / (2.0 * A), 0.0)
    t1 = np.where(hit, (-B + sq) / (2.0 * A), 0.0)
    return t0, t1


def radon_ellipses(ell: np.ndarray, N: int, angles: np.ndarray, K: int,
                   chunk: int = 8192) -> np.ndarray:
    """Exact line integrals of the painted (overwrite) ellipse object.

    Along each ray the object is piecewise constant: at parameter t its value
    is the gray of the last-painted ellipse that contains the point.  Sorting
    all interval end points and taking the top-most covering ellipse on each
    elementary piece gives the integral exactly (up to rounding).
    Returns the U x K sinogram in float64 (row-major, angle-major).
    """
    U = len(angles)
    rad = np.deg2rad(np.asarray(angles, dtype=np.float64))
    cu = np.cos(rad)
    su = np.sin(rad)
    sk = bin_centres(K)
    cth = np.repeat(cu, K)
    sth = np.repeat(su, K)
    ss = np.tile(sk, U)
    out = np.zeros(U * K, dtype=np.float64)
    E = ell.shape[0]
    gray = ell[:, 5]
    for r0 in range(0, U * K, chunk):
        r1 = min(U * K, r0 + chunk)
        t0, t1 = _ellipse_intervals(ell, cth[r0:r1], sth[r0:r1], ss[r0:r1])
        pts = np.sort(np.concatenate([t0, t1], axis=1), axis=1)
        mid = 0.5 * (pts[:, 1:] + pts[:, :-1])
        seg = pts[:, 1:] - pts[:, :-1]
        inside = (mid[:, :, None] > t0[:, None, :]) & (mid[:, :, None] < t1[:, None, :])
        idx = np.arange(E)[None, None, :]
        top = np.where(inside, idx, -1).max(axis=2)
        val = np.where(top >= 0, gray[np.maximum(top, 0)], 0.0)
        out[r0:r1] = (val * seg).sum(axis=1)
    return out.reshape(U, K)


# attenuation per pixel unit of a gray value of 1, in units of 1 / N: a ray
# through the middle of an object of mean gray 0.1 keeps about e^-1.6 = 20%
# of its photons, the transmission a CT scan is set up for
ATTENUATION = 16.0


def poisson_noise(sino: np.ndarray, N: int, I0: float, seed: int) -> np.ndarray:
    """Photon-counting noise on a transmission measurement.

    The object's attenuation is its gray value times mu = ATTENUATION / N per
    pixel unit, so the expected count on a ray is I0 exp(-mu P); the noisy
    line integral is -ln(max(n, 1) / I0) / mu.
    """
    rng = np.random.default_rng(seed)
    mu = ATTENUATION / N
    lam = I0 * np.exp(-mu * np.asarray(sino, dtype=np.float64))
    n = rng.poisson(lam).astype(np.float64)
    return -np.log(np.maximum(n, 1.0) / I0) / mu


def uniform_start(sino: np.ndarray, mask: Optional[np.ndarray], N: int,
                  f_min: float = 0.0, f_max: float = 1.0) -> np.ndarray:
    """Uniform solid starting image on the support (section III set-up).

    The level matches the measured mass: every projection integrates the
    whole object, so the mean over angles of the bin sums, divided by the
    number of support pixels, is the object's mean gray on the support.
    """
    sino = np.asarray(sino, dtype=np.float64)
    U = sino.shape[0]
    m = np.ones((N, N), np.uint8) if mask is None else np.asarray(mask, np.uint8)
    P = int(m.sum())
    c = float(sino.sum()) / U / max(P, 1)
    c = min(max(c, f_min), f_max)
    return np.where(m.reshape(N, N) != 0, c, 0.0).astype(np.float64)


def rmse(f: np.ndarray, f_true: np.ndarray) -> float:
    d = np.asarray(f, np.float64) - np.asarray(f_true, np.float64)
    return float(np.sqrt(np.mean(d * d)))


def nrmse(f: np.ndarray, f_true: np.ndarray) -> float:
    """RMS error normalised by the mean of the true image (section III-B)."""
    return rmse(f, f_true) / float(np.mean(f_true))


# ---------------------------------------------------------------------------
# 3-D volume for batches of slices
# ---------------------------------------------------------------------------

def random_ellipsoids(seed: int, n: int = 32) -> np.ndarray:
    """Random ellipsoids in the unit cube [-1,1]^3 (z-axis aligned extent).

    Rows are (cx, cy, cz, a, b, c, theta, gray) with (cx, cy) uniform in the
    disk of radius 0.6, semi-axes in [0.05, 0.35], rotation theta about z.
    """
    rng = np.random.default_rng(seed)
    out = np.empty((n, 8), dtype=np.float64)
    for e in range(n):
        rad = 0.6 * math.sqrt(rng.random())
        phi = 2.0 * math.pi * rng.random()
        out[e, 0] = rad * math.cos(phi)
        out[e, 1] = rad * math.sin(phi)
        out[e, 2] = -0.9 + 1.8 * rng.random()
        out[e, 3] = 0.05 + 0.30 * rng.random()
        out[e, 4] = 0.05 + 0.30 * rng.random()
        out[e, 5] = 0.10 + 0.60 * rng.random()
        out[e, 6] = math.pi * rng.random()
        out[e, 7] = rng.random()
    return out


def volume_slice(vol: np.ndarray, z: float, N: int) -> np.ndarray:
    """The 2-D ellipses (pixel units, paint order kept) cut by plane z."""
    h = N / 2.0
    rows = []
    for cx, cy, cz, a, b, c, th, g in vol:
        q = (z - cz) / c
        if abs(q) >= 1.0:
            continue
        sc = math.sqrt(1.0 - q * q)
        rows.append((cx * h, cy * h, a * sc * h, b * sc * h, th, g))
    if not rows:
        return np.zeros((0, 6), dtype=np.float64)
    return np.array(rows, dtype=np.float64)


@dataclass
class Slice:
    """One reconstruction problem: geometry, measured sinogram, truth, start."""
    N: int
    U: int
    K: int
    angles: np.ndarray
    mask: Optional[np.ndarray]
    sino: np.ndarray          # U x K measured (possibly noisy) line integrals
    truth: np.ndarray         # N x N area-averaged phantom
    f0: np.ndarray            # N x N uniform start on the support
    meta: dict = field(default_factory=dict)


def make_slice(N: int, U: int, K: int, ell: np.ndarray, *, masked: bool,
               I0: Optional[float] = None, noise_seed: int = 0,
               f_min: float = 0.0, f_max: float = 1.0) -> Slice:
    ang = angles_deg(U)
    sino = radon_ellipses(ell, N, ang, K)
    if I0 is not None:
        sino = poisson_noise(sino, N, I0, noise_seed)
    mask = circle_mask(N) if masked else None
    truth = rasterize(ell, N)
    f0 = uniform_start(sino, mask, N, f_min, f_max)
    return Slice(N, U, K, ang, mask, sino, truth, f0,
                 {"n_ell": int(ell.shape[0]), "I0": I0, "noise_seed": noise_seed})


# ---------------------------------------------------------------------------
# the five workloads (sizes and seeds)
# ---------------------------------------------------------------------------

CONFIGS = {
    # plain single chain in FP64: the parity workload
    "c1": dict(N=64, U=90, K=64, n_ell=10, phantom_seed=101, I0=None, masked=False,
               M=1, n_steps=200_000, delta_max=0.05, f_min=0.0, f_max=1.0,
               T0=1e-2, TN=1e-6, n_stages=1000, chain_seed=1001, precision="f64",
               resync_every=0),
    # single chain, FP32 residual with FP64 resync, BoME M=16
    "c2": dict(N=256, U=180, K=367, n_ell=10, phantom_seed=102, I0=1e4, noise_seed=202,
               masked=True, M=16, n_steps=5_000_000, delta_max=0.05, f_min=0.0,
               f_max=1.0, T0=None, TN=None, q_auto=200, tn_ratio=1e3, n_stages=1000,
               chain_seed=1002, precision="f32", resync_every=4096),
    # batch of slices from a 3-D volume, mixed sizes
    "c3": dict(volume_seed=103, n_slices=512, sizes=(128, 256, 512), n_angles=(90, 180, 360),
               I0=1e4, masked=True, M=8, sweeps=16, delta_max=0.05, f_min=0.0, f_max=1.0,
               q_auto=200, tn_ratio=1e3, n_stages=1000, chain_seed0=2000, precision="f32",
               resync_every=4096),
    # one large slice: SAT at M=32 plus 200 SIRT iterations
    "c4": dict(N=1024, U=720, K=1449, n_ell=30, phantom_seed=104, I0=1e4, noise_seed=204,
               masked=True, M=32, n_steps=1_000_000, delta_max=0.05, f_min=0.0, f_max=1.0,
               q_auto=200, tn_ratio=1e3, n_stages=1000, chain_seed=1004, precision="f32",
               resync_every=4096, sirt_iters=200, sirt_lambda=0.1),
    # serving stream
    "c5": dict(seed=105, n_requests=10_000, rate=200.0, sizes=(128, 256, 384, 512, 768, 1024),
               n_angles=(90, 180, 360, 720), I0_range=(1e3, 1e5), masked=True, M=8,
               sweeps=2, delta_max=0.05, f_min=0.0, f_max=1.0, q_auto=200, tn_ratio=1e3,
               n_stages=1000, precision="f32", resync_every=4096),
}


def config_slice(name: str) -> Slice:
    """The single-slice workloads c1, c2 and c4 as Slice objects."""
    c = CONFIGS[name]
    N, U, K = c["N"], c["U"], c["K"]
    ell = random_ellipses(c["phantom_seed"], N, c["n_ell"])
    return make_slice(N, U, K, ell, masked=c["masked"], I0=c["I0"],
                      noise_seed=c.get("noise_seed", 0), f_min=c["f_min"], f_max=c["f_max"])


def batch_slice_specs(seed: int, n: int, sizes, n_angles, I0: float, masked: bool = True,
                      volume_seed: Optional[int] = None) -> List[dict]:
    """Arguments of make_slice for n slices cut from one random ellipsoid volume
    (sizes and angle counts drawn per slice), so that callers may build the
    slices in parallel; batch_slices builds them in order."""
    rng = np.random.default_rng(seed)
    vol = random_ellipsoids(seed if volume_seed is None else volume_seed)
    out = []
    for s in range(n):
        z = -0.9 + 1.8 * s / max(n - 1, 1)
        N = int(rng.choice(sizes))
        U = int(rng.choice(n_angles))
        out.append(dict(N=N, U=U, K=n_bins_for(N), ell=volume_slice(vol, z, N), masked=masked,
                        I0=I0, noise_seed=seed * 1000 + s))
    return out


def slice_from_spec(spec: dict) -> Slice:
    return make_slice(spec["N"], spec["U"], spec["K"], spec["ell"], masked=spec["masked"],
                      I0=spec["I0"], noise_seed=spec["noise_seed"])


def batch_slices(seed: int, n: int, sizes, n_angles, I0: float, masked: bool = True,
                 volume_seed: Optional[int] = None) -> List[Slice]:
    """n slices cut from one random ellipsoid volume, sizes drawn per slice."""
    return [slice_from_spec(sp) for sp in batch_slice_specs(seed, n, sizes, n_angles, I0, masked,
                                                            volume_seed)]
