"""Brute-force ray/pixel clipping (test-only, independent of both paths).

Every ray is clipped against every pixel square with the Liang-Barsky
parametric test, giving the exact chord length of the line inside the
closed square.  Rays lying exactly on a pixel edge (axis-parallel rays at
0 / 90 degrees) are given to the pixel whose half-open interval contains
them.  Chords at or below 1e-9 (corner touches) are dropped.  Cost is
O(rays x pixels): small grids only.
"""
from __future__ import annotations

import math

import numpy as np

TAU = 1e-9


def trig(deg: float):
    if math.fmod(deg, 90.0) == 0.0:
        q = int(deg // 90.0) % 4
        return [(1.0, 0.0), (0.0, 1.0), (-1.0, 0.0), (0.0, -1.0)][q]
    a = math.radians(deg)
    return math.cos(a), math.sin(a)


def dense_system(N: int, U: int, K: int, angles, mask=None) -> np.ndarray:
    """Dense G x N^2 matrix of intersection lengths, G = U*K rays."""
    h = N / 2.0
    ii, jj = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    x0 = (jj - h).reshape(-1).astype(np.float64)       # left edge of pixel p = i*N + j
    y0 = (h - 1 - ii).reshape(-1).astype(np.float64)   # bottom edge
    A = np.zeros((U * K, N * N), dtype=np.float64)
    sk = np.arange(K, dtype=np.float64) - (K - 1) / 2.0
    for u, deg in enumerate(angles):
        c, s = trig(float(deg))
        for k in range(K):
            g = u * K + k
            rho2 = c * c + s * s               # 1 up to rounding
            px, py = sk[k] * c / rho2, sk[k] * s / rho2   # foot point on x c + y s = sk
            dx, dy = -s, c                     # direction, length sqrt(rho2)
            if dx == 0.0:                      # vertical ray, half-open columns
                A[g] = ((px >= x0) & (px < x0 + 1.0)).astype(np.float64)
            elif dy == 0.0:                    # horizontal ray, half-open rows
                A[g] = ((py >= y0) & (py < y0 + 1.0)).astype(np.float64)
            else:
                ta = (x0 - px) / dx
                tb = (x0 + 1.0 - px) / dx
                tc = (y0 - py) / dy
                td = (y0 + 1.0 - py) / dy
                tlo = np.maximum(np.minimum(ta, tb), np.minimum(tc, td))
                thi = np.minimum(np.maximum(ta, tb), np.maximum(tc, td))
                A[g] = np.maximum(thi - tlo, 0.0) * math.sqrt(rho2)
    A[A <= TAU] = 0.0
    if mask is not None:
        A[:, np.asarray(mask).reshape(-1) == 0] = 0.0
    return A


def slab_length(N: int, c: float, s: float, sk: float) -> float:
    """Length of the ray x c + y s = sk inside the square [-N/2, N/2]^2.

    An axis-parallel ray on the square's boundary counts only on the closed
    (left / bottom) side, as the half-open pixel rule gives it.
    """
    h = N / 2.0
    rho2 = c * c + s * s
    px, py, dx, dy = sk * c / rho2, sk * s / rho2, -s, c
    lo, hi = -math.inf, math.inf
    for p, d in ((px, dx), (py, dy)):
        if d == 0.0:
            if p < -h or p >= h:
                return 0.0
            continue
        t1, t2 = (-h - p) / d, (h - p) / d
        lo = max(lo, min(t1, t2))
        hi = min(hi, max(t1, t2))
    return max(hi - lo, 0.0) * math.sqrt(rho2)
