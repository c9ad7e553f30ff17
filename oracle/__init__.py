"""Plain FP64 CPU oracle (ctypes wrapper around oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package; the product path
(paper_1411_4622_amd) never does, and this package never imports it.

Each function states the passage of the paper it follows; the C source
holds the arithmetic.  Parity of the FP32-residual chain mode is an
approximation by design and has no exact pin (only drift bounds).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (scalar, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class SatParams(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("chain_id", C.c_uint64), ("n_steps", C.c_int64),
                ("n_stages", C.c_int32), ("m_cand", C.c_int32), ("T0", C.c_double),
                ("TN", C.c_double), ("q_auto", C.c_int32), ("precision", C.c_int32),
                ("tn_ratio", C.c_double), ("delta_max", C.c_double), ("f_min", C.c_double),
                ("f_max", C.c_double), ("resync_every", C.c_int64)]


class SatStats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("accepts", C.c_int64), ("accepts_nonzero", C.c_int64),
                ("resyncs", C.c_int32), ("pad", C.c_int32), ("T0_used", C.c_double),
                ("TN_used", C.c_double), ("sse_final", C.c_double), ("cost_final", C.c_double),
                ("max_drift_r", C.c_double), ("max_drift_sse", C.c_double)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = build(force=False)
    lib = C.CDLL(path)
    P = C.c_void_p
    lib.or_philox.argtypes = [P, P, P]
    lib.or_trig.argtypes = [C.c_int32, P, P]
    lib.or_rays.argtypes = [C.c_int32, C.c_int32, C.c_int32, P, P, P, P, P, P]
    lib.or_rays.restype = C.c_int64
    lib.or_pila_from_rays.argtypes = [C.c_int32, C.c_int32, C.c_int32, P, P, P, P, P, P]
    lib.or_trace_ray.argtypes = [C.c_int32, C.c_int32, C.c_double, C.c_int32, P, P, P]
    lib.or_trace_ray.restype = C.c_int32
    lib.or_pixel_row.argtypes = [C.c_int32, C.c_int32, C.c_int32, P, P, C.c_int32, P, P]
    lib.or_pixel_row.restype = C.c_int32
    lib.or_forward.argtypes = [C.c_int32, C.c_int32, C.c_int32, P, P, P, P, P]
    lib.or_backward.argtypes = [C.c_int32, P, P, P, P, P]
    lib.or_temperature.argtypes = [C.c_int64, C.c_int64, C.c_int32, C.c_double, C.c_double]
    lib.or_temperature.restype = C.c_double
    lib.or_sat_run.argtypes = [C.c_int32, C.c_int32, C.c_int32, P, P, P, P, P, P, P, P, P, P, P, P]
    lib.or_sat_run.restype = C.c_int
    lib.or_sirt_run.argtypes = [C.c_int32, C.c_int32, C.c_int32, P, P, P, P, C.c_int32,
                                C.c_double, P, P]
    lib.or_sirt_run.restype = C.c_int
    _lib = lib
    return lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def philox(key, ctr) -> np.ndarray:
    """Philox4x64-10 block for (key[2], counter[4]) -> 4 uint64 words."""
    k = np.ascontiguousarray(key, dtype=np.uint64)
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    _load().or_philox(_p(k), _p(c), _p(out))
    return out


def trig(angles) -> np.ndarray:
    a = np.ascontiguousarray(angles, dtype=np.float64)
    cs = np.zeros(2 * len(a), dtype=np.float64)
    _load().or_trig(len(a), _p(a), _p(cs))
    return cs.reshape(-1, 2)


def rays(N: int, U: int, K: int, angles, mask=None):
    """Siddon ray-major listing (section II-B): (off[G+1], pix[nnz], len[nnz])."""
    lib = _load()
    a = np.ascontiguousarray(angles, dtype=np.float64)
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
    G = U * K
    cnt = np.zeros(G, dtype=np.int32)
    lib.or_rays(N, U, K, _p(a), _p(m), _p(cnt), None, None, None)
    off = np.zeros(G + 1, dtype=np.int64)
    np.cumsum(cnt, out=off[1:])
    pix = np.zeros(int(off[-1]), dtype=np.int32)
    ln = np.zeros(int(off[-1]), dtype=np.float64)
    lib.or_rays(N, U, K, _p(a), _p(m), None, _p(off), _p(pix), _p(ln))
    return off, pix, ln


def pila(N: int, U: int, K: int, angles, mask=None, with_rays: bool = False):
    """PILA of Eq. 5 as pixel-major CSR (row_ptr[N*N+1], col=g ascending, len)."""
    off, pix, ln = rays(N, U, K, angles, mask)
    row_ptr = np.zeros(N * N + 1, dtype=np.int64)
    col = np.zeros(len(pix), dtype=np.int32)
    plen = np.zeros(len(pix), dtype=np.float64)
    _load().or_pila_from_rays(N, U, K, _p(off), _p(pix), _p(ln), _p(row_ptr), _p(col), _p(plen))
    if with_rays:
        return (row_ptr, col, plen), (off, pix, ln)
    return row_ptr, col, plen


def trace_ray(N: int, K: int, deg: float, k: int, mask=None):
    """One ray traced on its own (Siddon): (pixels in trace order, lengths)."""
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
    pix = np.zeros(2 * N + 8, dtype=np.int32)
    ln = np.zeros(2 * N + 8, dtype=np.float64)
    n = _load().or_trace_ray(N, K, float(deg), int(k), _p(m), _p(pix), _p(ln))
    return pix[:n].copy(), ln[:n].copy()


def pixel_row(N: int, U: int, K: int, angles, p: int, mask=None):
    """PILA row of one pixel (Eq. 5), traced ray by ray: (g ascending, lengths)."""
    a = np.ascontiguousarray(angles, dtype=np.float64)
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
    g = np.zeros(4 * U + 8, dtype=np.int32)
    ln = np.zeros(4 * U + 8, dtype=np.float64)
    n = _load().or_pixel_row(N, U, K, _p(a), _p(m), int(p), _p(g), _p(ln))
    return g[:n].copy(), ln[:n].copy()


def forward(N: int, U: int, K: int, csr, f) -> np.ndarray:
    """Eq. 1 for all rays through the PILA: U x K sinogram of image f."""
    row_ptr, col, ln = csr
    fv = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
    out = np.zeros(U * K, dtype=np.float64)
    _load().or_forward(N, U, K, _p(row_ptr), _p(col), _p(ln), _p(fv), _p(out))
    return out.reshape(U, K)


def backward(N: int, csr, y) -> np.ndarray:
    """Transpose of Eq. 1: N x N image of sum_g l(p, g) y_g."""
    row_ptr, col, ln = csr
    yv = np.ascontiguousarray(y, dtype=np.float64).reshape(-1)
    out = np.zeros(N * N, dtype=np.float64)
    _load().or_backward(N, _p(row_ptr), _p(col), _p(ln), _p(yv), _p(out))
    return out.reshape(N, N)


def temperature(s: int, n_steps: int, n_stages: int, T0: float, TN: float) -> float:
    """Eq. 2 evaluated at the stage of step s."""
    return float(_load().or_temperature(s, n_steps, n_stages, T0, TN))


def make_params(**kw) -> SatParams:
    p = SatParams()
    p.seed = kw.get("seed", 0)
    p.chain_id = kw.get("chain_id", 0)
    p.n_steps = kw["n_steps"]
    p.n_stages = kw.get("n_stages", 1000)
    p.m_cand = kw.get("m_cand", 1)
    p.T0 = kw.get("T0") or 0.0
    p.TN = kw.get("TN") or 0.0
    p.q_auto = kw.get("q_auto", 200)
    p.precision = 1 if kw.get("precision", "f64") in ("f32", 1) else 0
    p.tn_ratio = kw.get("tn_ratio", 1e3)
    p.delta_max = kw.get("delta_max", 0.05)
    p.f_min = kw.get("f_min", 0.0)
    p.f_max = kw.get("f_max", 1.0)
    p.resync_every = kw.get("resync_every", 0)
    return p


def sat_run(N: int, U: int, K: int, csr, sino, f0, mask=None, trace: bool = True, **kw):
    """One SAT chain (section II-A/B, BoME of III-B).  Returns (f, stats, trace)."""
    row_ptr, col, ln = csr
    prm = make_params(**kw)
    f = np.ascontiguousarray(f0, dtype=np.float64).reshape(-1).copy()
    s = np.ascontiguousarray(sino, dtype=np.float64).reshape(-1)
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
    st = SatStats()
    n = prm.n_steps
    tr = None
    if trace:
        tr = dict(m_star=np.zeros(n, np.int32), accept=np.zeros(n, np.uint8),
                  dC=np.zeros(n, np.float64), scale=np.zeros(n, np.float64))
    rc = _load().or_sat_run(N, U, K, _p(m), _p(row_ptr), _p(col), _p(ln), _p(s), C.byref(prm),
                            _p(f), C.byref(st), _p(tr["m_star"]) if tr else None,
                            _p(tr["accept"]) if tr else None, _p(tr["dC"]) if tr else None,
                            _p(tr["scale"]) if tr else None)
    if rc != 0:
        raise RuntimeError("oracle sat_run failed with %d" % rc)
    stats = {k: getattr(st, k) for k, _ in SatStats._fields_ if k != "pad"}
    return f.reshape(N, N), stats, tr


def sirt_run(N: int, U: int, K: int, csr, sino, f0, n_iter: int, lam: float):
    """SIRT with exact lengths (section III-D, Eq. 10-11), simultaneous form."""
    row_ptr, col, ln = csr
    f = np.ascontiguousarray(f0, dtype=np.float64).reshape(-1).copy()
    s = np.ascontiguousarray(sino, dtype=np.float64).reshape(-1)
    cost = np.zeros(n_iter, dtype=np.float64)
    _load().or_sirt_run(N, U, K, _p(row_ptr), _p(col), _p(ln), _p(s), n_iter, lam, _p(f), _p(cost))
    return f.reshape(N, N), cost
