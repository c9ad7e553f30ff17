"""Plain FP64 CPU oracle (ctypes wrapper around oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package; the product path
(paper_1411_4622_amd) never does, and this package never imports it.

Each function states the passage of the paper it follows; the C source
holds the arithmetic.  The FP32-residual chain mode is an approximation by
design; it is pinned by rounding-error bounds (see oracle.c).
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
                ("f_max", C.c_double), ("resync_every", C.c_int64), ("schedule", C.c_int32),
                ("proposal", C.c_int32)]


SCHEDULES = {"linear": 0, "exp": 1, "cubic": 2}
PROPOSALS = {"clamp": 0, "redraw": 1}


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
    lib.or_temperature.argtypes = [C.c_int64, C.c_int64, C.c_int32, C.c_double, C.c_double,
                                   C.c_int32]
    lib.or_temperature.restype = C.c_double
    lib.or_sat_run.argtypes = [C.c_int32, C.c_int32, C.c_int32, P, P, P, P, P, P, P, P, P, P, P, P, P]
    lib.or_sat_run.restype = C.c_int
    lib.or_delta_sse64.argtypes = [P, P, P, P, C.c_int32, C.c_double, P]
    lib.or_delta_sse64.restype = C.c_double
    lib.or_delta_sse32.argtypes = [P, P, P, P, C.c_int32, C.c_double]
    lib.or_delta_sse32.restype = C.c_float
    lib.or_sirt_seq_run.argtypes = [C.c_int32, C.c_int32, C.c_int32, P, P, P, P, C.c_int64, P,
                                    C.c_int32, C.c_int64, C.c_double, C.c_uint64, P, P]
    lib.or_sirt_seq_run.restype = C.c_int
    lib.or_drt_half_span.argtypes = [C.c_int32]
    lib.or_drt_half_span.restype = C.c_int32
    lib.or_drt.argtypes = [C.c_int32, C.c_int32, C.c_int32, P, P, P]
    lib.or_satdrt_run.argtypes = [C.c_int32, C.c_int32, C.c_int32, P, P, P, P, P, P, P, P, P]
    lib.or_satdrt_run.restype = C.c_int
    lib.or_quantize_u8.argtypes = [C.c_int64, P, P]
    lib.or_dequantize_u8.argtypes = [C.c_int64, P, P]
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


def temperature(s: int, n_steps: int, n_stages: int, T0: float, TN: float,
                schedule: str = "linear") -> float:
    """Temperature at the stage of step s: Eq. 2 (linear), the exponential
    schedule of section III-C (its second Eq. 8) or the cubic one (Eq. 9)."""
    return float(_load().or_temperature(s, n_steps, n_stages, T0, TN, SCHEDULES[schedule]))


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
    p.schedule = SCHEDULES[kw.get("schedule", "linear")]
    p.proposal = PROPOSALS[kw.get("proposal", "clamp")]
    return p


def sat_run(N: int, U: int, K: int, csr, sino, f0, mask=None, trace: bool = True,
            residual: bool = False, **kw):
    """One SAT chain (section II-A/B, BoME of III-B).  Returns (f, stats, trace),
    and the final running residual (U x K) as a fourth item when residual=True."""
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
    r_out = np.zeros(U * K, dtype=np.float64) if residual else None
    rc = _load().or_sat_run(N, U, K, _p(m), _p(row_ptr), _p(col), _p(ln), _p(s), C.byref(prm),
                            _p(f), C.byref(st), _p(tr["m_star"]) if tr else None,
                            _p(tr["accept"]) if tr else None, _p(tr["dC"]) if tr else None,
                            _p(tr["scale"]) if tr else None, _p(r_out))
    if rc != 0:
        raise RuntimeError("oracle sat_run failed with %d" % rc)
    stats = {k: getattr(st, k) for k, _ in SatStats._fields_ if k != "pad"}
    if residual:
        return f.reshape(N, N), stats, tr, r_out.reshape(U, K)
    return f.reshape(N, N), stats, tr


def sirt_run(N: int, U: int, K: int, csr, sino, f0, n_iter: int, lam: float):
    """SIRT with exact lengths (section III-D, Eq. 10-11), simultaneous form."""
    row_ptr, col, ln = csr
    f = np.ascontiguousarray(f0, dtype=np.float64).reshape(-1).copy()
    s = np.ascontiguousarray(sino, dtype=np.float64).reshape(-1)
    cost = np.zeros(n_iter, dtype=np.float64)
    _load().or_sirt_run(N, U, K, _p(row_ptr), _p(col), _p(ln), _p(s), n_iter, lam, _p(f), _p(cost))
    return f.reshape(N, N), cost


def delta_sse(csr, r, p: int, d: float, fp32: bool = False):
    """Eq. 7's inner sum for pixel p changed by d against residual r: FP64
    (returns (S, sum of |terms|)) or with the FP32 operands and accumulation
    of an FP32 chain (returns S as a float)."""
    row_ptr, col, ln = csr
    lib = _load()
    if fp32:
        r32 = np.ascontiguousarray(r, dtype=np.float32).reshape(-1)
        return float(lib.or_delta_sse32(_p(row_ptr), _p(col), _p(ln), _p(r32), int(p), float(d)))
    r64 = np.ascontiguousarray(r, dtype=np.float64).reshape(-1)
    a = C.c_double(0.0)
    S = lib.or_delta_sse64(_p(row_ptr), _p(col), _p(ln), _p(r64), int(p), float(d), C.byref(a))
    return float(S), float(a.value)


def support_of(N: int, mask=None) -> np.ndarray:
    m = np.ones(N * N, np.uint8) if mask is None else np.asarray(mask, np.uint8).reshape(-1)
    return np.flatnonzero(m).astype(np.int32)


def sirt_seq_run(N: int, U: int, K: int, csr, sino, f0, n_iter: int, m_per: int, lam: float,
                 seed: int, mask=None):
    """SIRT pixel by pixel (section III-D as described, Eq. 10-11): n_iter
    iterations of m_per pixel updates, pixels drawn at random over the
    support.  Returns (f, cost after each iteration)."""
    row_ptr, col, ln = csr
    sup = support_of(N, mask)
    f = np.ascontiguousarray(f0, dtype=np.float64).reshape(-1).copy()
    s = np.ascontiguousarray(sino, dtype=np.float64).reshape(-1)
    cost = np.zeros(max(n_iter, 1), dtype=np.float64)
    rc = _load().or_sirt_seq_run(N, U, K, _p(row_ptr), _p(col), _p(ln), _p(s), len(sup), _p(sup),
                                 int(n_iter), int(m_per), float(lam), int(seed), _p(f), _p(cost))
    if rc != 0:
        raise RuntimeError("oracle sirt_seq_run failed with %d" % rc)
    return f.reshape(N, N), cost[:n_iter]


def drt_half_span(N: int) -> int:
    """Samples of the bilinear DRT run at t = -T .. T along each ray."""
    return int(_load().or_drt_half_span(N))


def drt(N: int, U: int, K: int, angles, f) -> np.ndarray:
    """Eq. 1 the conventional way (section III-A's comparison): U x K
    sinogram of image f by bilinear interpolation at unit steps."""
    a = np.ascontiguousarray(angles, dtype=np.float64)
    fv = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
    out = np.zeros(U * K, dtype=np.float64)
    _load().or_drt(N, U, K, _p(a), _p(fv), _p(out))
    return out.reshape(U, K)


def satdrt_run(N: int, U: int, K: int, angles, sino, f0, mask=None, **kw):
    """SAT whose evaluation step projects each estimate's whole image with the
    bilinear DRT (section III-A's comparison method).  T0/TN must be given.
    Returns (f, final cost, trace)."""
    prm = make_params(**kw)
    a = np.ascontiguousarray(angles, dtype=np.float64)
    f = np.ascontiguousarray(f0, dtype=np.float64).reshape(-1).copy()
    s = np.ascontiguousarray(sino, dtype=np.float64).reshape(-1)
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
    n = prm.n_steps
    tr = dict(m_star=np.zeros(max(n, 1), np.int32), accept=np.zeros(max(n, 1), np.uint8),
              dC=np.zeros(max(n, 1), np.float64))
    cf = C.c_double(0.0)
    rc = _load().or_satdrt_run(N, U, K, _p(a), _p(m), _p(s), C.byref(prm), _p(f),
                               _p(tr["m_star"]), _p(tr["accept"]), _p(tr["dC"]), C.byref(cf))
    if rc != 0:
        raise RuntimeError("oracle satdrt_run failed with %d" % rc)
    return f.reshape(N, N), float(cf.value), {k: v[:n] for k, v in tr.items()}


def quantize_u8(lengths) -> np.ndarray:
    """One-byte lengths of section II-B: round(180 l)."""
    ln = np.ascontiguousarray(lengths, dtype=np.float64).reshape(-1)
    q = np.zeros(len(ln), dtype=np.uint8)
    _load().or_quantize_u8(len(ln), _p(ln), _p(q))
    return q


def dequantize_u8(q) -> np.ndarray:
    """The length each byte stands for, q / 180 in float, widened to double."""
    qq = np.ascontiguousarray(q, dtype=np.uint8).reshape(-1)
    out = np.zeros(len(qq), dtype=np.float64)
    _load().or_dequantize_u8(len(qq), _p(qq), _p(out))
    return out
