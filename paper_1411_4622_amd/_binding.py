"""ctypes binding of libpila.so (argument marshalling only).

Device memory comes from torch tensors on the current HIP device and work is
enqueued on torch's current stream; every step of the computation runs in
the library's HIP kernels.  If the library has not been built the first
call raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpila.so")

PILA_OK, PILA_EINVAL, PILA_ENOMEM, PILA_EHIP, PILA_ESIZE = 0, -1, -2, -3, -4
PILA_ECANCELED, PILA_EBUSY, PILA_ENOTFOUND, PILA_ETIMEDOUT = -5, -6, -7, -8
PILA_F64, PILA_F32, PILA_U8 = 0, 1, 2
PILA_SIRT_REUSE_LAYOUT = 1
SCHEDULES = {"linear": 0, "exp": 1, "cubic": 2}      # PILA_SCHED_*
PROPOSALS = {"clamp": 0, "redraw": 1}                # PILA_PROP_*
BODY_PIPED, BODY_LONG, BODY_GENERAL, BODY_SPLIT = 1, 2, 3, 4  # PILA_BODY_* kinds
BODY_GLOBAL_R, BODY_SEGMENTED = 16, 32                # PILA_BODY_* flags

EXPORTED = ["pila_build_scratch_size", "pila_build", "pila_forward", "pila_backproject", "sat_workspace_size",
            "sat_workspace_min", "sat_run", "sat_run_static",
            "sat_batch_workspace_size", "sat_run_batch", "sat_graph_create", "sat_batch_graph_create",
            "sat_graph_launch", "sat_graph_stats", "sat_graph_destroy", "sirt_workspace_size", "sirt_run",
            "sirt_seq_workspace_size", "sirt_seq_run", "sat_drt_workspace_size", "sat_drt_run",
            "srv_create", "srv_prepare", "srv_submit", "srv_poll", "srv_cancel", "srv_get_status",
            "srv_destroy", "pila_get_device_info", "pila_last_error"]


class PilaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("libpila error %d: %s" % (code, msg))
        self.code = code


class CGeom(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_angles", C.c_int32), ("n_bins", C.c_int32),
                ("len_dtype", C.c_int32), ("angles_deg", C.c_void_p), ("mask", C.c_void_p)]


class CCsr(C.Structure):
    _fields_ = [("nnz", C.c_int64), ("n_support", C.c_int32), ("max_row", C.c_int32),
                ("k_lo", C.c_int32), ("k_hi", C.c_int32), ("row_ptr", C.c_void_p), ("col", C.c_void_p), ("len", C.c_void_p),
                ("support", C.c_void_p), ("trig", C.c_void_p), ("t_row_ptr", C.c_void_p),
                ("t_col", C.c_void_p), ("t_len", C.c_void_p)]


class CSatParams(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("chain_id", C.c_uint64), ("n_steps", C.c_int64),
                ("n_stages", C.c_int32), ("m_cand", C.c_int32), ("T0", C.c_double),
                ("TN", C.c_double), ("q_auto", C.c_int32), ("precision", C.c_int32),
                ("tn_ratio", C.c_double), ("delta_max", C.c_double), ("f_min", C.c_double),
                ("f_max", C.c_double), ("resync_every", C.c_int64), ("schedule", C.c_int32),
                ("proposal", C.c_int32)]


class CSatStats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("accepts", C.c_int64), ("accepts_nonzero", C.c_int64),
                ("resyncs", C.c_int32), ("status", C.c_int32), ("T0_used", C.c_double),
                ("TN_used", C.c_double), ("sse_final", C.c_double), ("cost_final", C.c_double),
                ("max_drift_r", C.c_double), ("max_drift_sse", C.c_double),
                ("chain_launches", C.c_int32), ("body", C.c_int32), ("chain_kernel_ms", C.c_double),
                ("t_begin", C.c_int64), ("t_end", C.c_int64)]


class CSatTrace(C.Structure):
    _fields_ = [("m_star", C.c_void_p), ("accept", C.c_void_p), ("dC", C.c_void_p)]


class CSatJob(C.Structure):
    _fields_ = [("geom", C.POINTER(CGeom)), ("csr", C.POINTER(CCsr)), ("d_sino", C.c_void_p),
                ("d_image", C.c_void_p), ("params", CSatParams), ("waves_per_chain", C.c_int32),
                ("reserved", C.c_int32)]


class CSatLaunch(C.Structure):
    _fields_ = [("waves_per_chain", C.c_int32), ("chains_per_cu", C.c_int32),
                ("lds_residual", C.c_int32), ("max_groups", C.c_int32),
                ("h_group_ms", C.POINTER(C.c_float)), ("h_group_desc", C.POINTER(C.c_int32)),
                ("h_group_chains", C.POINTER(C.c_int32))]


class CSirtParams(C.Structure):
    _fields_ = [("n_iter", C.c_int32), ("flags", C.c_int32), ("lam", C.c_double)]


class CSirtSeqParams(C.Structure):
    _fields_ = [("n_iter", C.c_int32), ("reserved", C.c_int32), ("m_per", C.c_int64), ("lam", C.c_double),
                ("seed", C.c_uint64)]


class CSrvConfig(C.Structure):
    _fields_ = [("mem_budget", C.c_size_t), ("max_slots", C.c_int32), ("waves_per_chain", C.c_int32),
                ("ring_size", C.c_int32), ("idle_us", C.c_int32), ("general_slots", C.c_int32),
                ("long_slots", C.c_int32)]


class CSrvRequest(C.Structure):
    _fields_ = [("geom", C.POINTER(CGeom)), ("d_sino", C.c_void_p), ("d_image", C.c_void_p),
                ("params", CSatParams)]


class CSrvStatus(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("reaped", C.c_int64), ("in_flight", C.c_int64),
                ("launches", C.c_int64), ("bytes_used", C.c_size_t), ("bytes_budget", C.c_size_t),
                ("pila_cached", C.c_int32), ("kernel_running", C.c_int32)]


class CDeviceInfo(C.Structure):
    _fields_ = [("cu_count", C.c_int32), ("lds_per_block", C.c_int32), ("clock_khz", C.c_int32),
                ("warp_size", C.c_int32), ("hbm_bytes", C.c_size_t), ("name", C.c_char * 64),
                ("wallclock_khz", C.c_int32), ("pad", C.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libpila.so and declare its signatures (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libpila.so is not built (expected at %s); run "
                           "python paper_1411_4622_amd/build.py" % path)
    lib = C.CDLL(path)
    V, I32 = C.c_void_p, C.c_int32
    G, CS = C.POINTER(CGeom), C.POINTER(CCsr)
    lib.pila_build_scratch_size.argtypes = [G, C.POINTER(C.c_size_t)]
    lib.pila_build.argtypes = [G, CS, V, C.c_size_t, V]
    lib.pila_forward.argtypes = [G, CS, V, V, V]
    lib.pila_backproject.argtypes = [G, CS, V, V, V]
    lib.sat_workspace_size.argtypes = [G, C.POINTER(CSatParams), C.POINTER(C.c_size_t)]
    lib.sat_workspace_min.argtypes = [G, C.POINTER(CSatParams), C.POINTER(C.c_size_t)]
    lib.sat_run.argtypes = [G, CS, V, C.POINTER(CSatParams), V, V, C.c_size_t,
                            C.POINTER(CSatStats), C.POINTER(CSatTrace), V]
    lib.sat_run_static.argtypes = [G, CS, V, C.POINTER(CSatParams), V, C.POINTER(CSatStats),
                                   C.POINTER(CSatTrace), V]
    lib.sat_batch_workspace_size.argtypes = [I32, C.POINTER(CSatJob), C.POINTER(C.c_size_t)]
    lib.sat_run_batch.argtypes = [I32, C.POINTER(CSatJob), C.POINTER(CSatLaunch), V, C.c_size_t,
                                  C.POINTER(CSatStats), V]
    lib.sat_graph_create.argtypes = [G, CS, V, C.POINTER(CSatParams), V, V, C.c_size_t,
                                     C.POINTER(CSatTrace), C.POINTER(V)]
    lib.sat_batch_graph_create.argtypes = [I32, C.POINTER(CSatJob), C.POINTER(CSatLaunch), V, C.c_size_t,
                                           C.POINTER(V)]
    lib.sat_graph_launch.argtypes = [V, V]
    lib.sat_graph_stats.argtypes = [V, C.POINTER(CSatStats), V]
    lib.sat_graph_destroy.argtypes = [V]
    lib.sirt_workspace_size.argtypes = [G, C.POINTER(CSirtParams), C.POINTER(C.c_size_t)]
    lib.sirt_run.argtypes = [G, CS, V, C.POINTER(CSirtParams), V, V, C.c_size_t, V, V]
    lib.sat_drt_workspace_size.argtypes = [G, C.POINTER(CSatParams), C.POINTER(C.c_size_t)]
    lib.sat_drt_run.argtypes = [G, V, C.POINTER(CSatParams), V, V, C.c_size_t, V, C.POINTER(CSatTrace), V]
    lib.sirt_seq_workspace_size.argtypes = [G, C.POINTER(CSirtSeqParams), C.POINTER(C.c_size_t)]
    lib.sirt_seq_run.argtypes = [G, CS, V, C.POINTER(CSirtSeqParams), V, V, C.c_size_t, V, V]
    lib.srv_create.argtypes = [C.POINTER(CSrvConfig), C.POINTER(V)]
    lib.srv_prepare.argtypes = [V, G]
    lib.srv_submit.argtypes = [V, C.POINTER(CSrvRequest), C.POINTER(C.c_uint64)]
    lib.srv_poll.argtypes = [V, C.c_uint64, C.POINTER(I32), C.POINTER(CSatStats)]
    lib.srv_cancel.argtypes = [V, C.c_uint64]
    lib.srv_get_status.argtypes = [V, C.POINTER(CSrvStatus)]
    lib.srv_destroy.argtypes = [V]
    lib.pila_get_device_info.argtypes = [C.POINTER(CDeviceInfo)]
    lib.pila_last_error.restype = C.c_char_p
    for name in EXPORTED:
        if name != "pila_last_error":
            getattr(lib, name).restype = I32
    _lib = lib
    return lib


def last_error() -> str:
    return load().pila_last_error().decode()


def _check(rc: int):
    if rc != PILA_OK:
        raise PilaError(rc, last_error())


def _torch():
    import torch
    return torch


def _stream():
    return C.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


# ---------------------------------------------------------------------------
# geometry and PILA
# ---------------------------------------------------------------------------

class Geometry:
    """Problem statement: image size, angles (degrees), bins, support mask."""

    def __init__(self, n: int, angles_deg: Sequence[float], n_bins: int, mask=None,
                 len_dtype: str = "f64"):
        self.n = int(n)
        self.angles = np.ascontiguousarray(angles_deg, dtype=np.float64)
        self.n_angles = len(self.angles)
        self.n_bins = int(n_bins)
        self.mask = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
        self.len_dtype = {"f64": PILA_F64, "f32": PILA_F32, "u8": PILA_U8}.get(len_dtype, len_dtype)
        if self.len_dtype not in (PILA_F64, PILA_F32, PILA_U8):
            raise ValueError("len_dtype must be 'f64', 'f32' or 'u8'")
        self._c = CGeom(self.n, self.n_angles, self.n_bins, self.len_dtype,
                        self.angles.ctypes.data, None if self.mask is None else self.mask.ctypes.data)

    @property
    def c(self) -> CGeom:
        return self._c

    @property
    def n_rays(self) -> int:
        return self.n_angles * self.n_bins


class Pila:
    """A built PILA: device tensors plus the C descriptor pointing at them."""

    def __init__(self, geom: Geometry, tensors: dict, nnz: int, n_support: int, max_row: int,
                 k_lo: int = 0, k_hi: int = -1):
        self.geom = geom
        self.t = tensors
        self.nnz = nnz
        self.n_support = n_support
        self.max_row = max_row
        self.k_lo, self.k_hi = k_lo, k_hi
        t = tensors
        self._c = CCsr(nnz, n_support, max_row, k_lo, k_hi, _ptr(t["row_ptr"]), _ptr(t["col"]), _ptr(t["len"]),
                       _ptr(t["support"]), _ptr(t["trig"]), _ptr(t["t_row_ptr"]), _ptr(t["t_col"]),
                       _ptr(t["t_len"]))

    @property
    def c(self) -> CCsr:
        return self._c

    def __getattr__(self, k):
        t = self.__dict__.get("t")
        if t is not None and k in t:
            return t[k]
        raise AttributeError(k)


def pila_build(geom: Geometry, device=None) -> Pila:
    """Build the PILA of a geometry on the current device (two-phase call)."""
    torch = _torch()
    lib = load()
    dev = device or torch.device("cuda", torch.cuda.current_device())
    NP, G, U = geom.n * geom.n, geom.n_rays, geom.n_angles
    row_ptr = torch.empty(NP + 1, dtype=torch.int64, device=dev)
    t_row_ptr = torch.empty(G + 1, dtype=torch.int64, device=dev)
    trig = torch.empty(2 * U, dtype=torch.float64, device=dev)
    csr = CCsr(0, 0, 0, 0, -1, row_ptr.data_ptr(), None, None, None, trig.data_ptr(),
               t_row_ptr.data_ptr(), None, None)
    nb = C.c_size_t(0)
    _check(lib.pila_build_scratch_size(C.byref(geom.c), C.byref(nb)))
    scratch = torch.empty(int(nb.value), dtype=torch.uint8, device=dev)
    _check(lib.pila_build(C.byref(geom.c), C.byref(csr), scratch.data_ptr(), scratch.numel(),
                          _stream()))
    nnz, P, max_row = int(csr.nnz), int(csr.n_support), int(csr.max_row)
    k_lo, k_hi = int(csr.k_lo), int(csr.k_hi)
    ldt = {PILA_F64: torch.float64, PILA_F32: torch.float32, PILA_U8: torch.uint8}[geom.len_dtype]
    col = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
    ln = torch.empty(max(nnz, 1), dtype=ldt, device=dev)
    t_col = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
    t_ln = torch.empty(max(nnz, 1), dtype=ldt, device=dev)
    support = torch.empty(max(P, 1), dtype=torch.int32, device=dev)
    csr.col, csr.len, csr.t_col, csr.t_len, csr.support = (col.data_ptr(), ln.data_ptr(),
                                                           t_col.data_ptr(), t_ln.data_ptr(),
                                                           support.data_ptr())
    _check(lib.pila_build(C.byref(geom.c), C.byref(csr), scratch.data_ptr(), scratch.numel(),
                          _stream()))
    return Pila(geom, dict(row_ptr=row_ptr, col=col[:nnz], len=ln[:nnz], support=support[:P],
                           trig=trig, t_row_ptr=t_row_ptr, t_col=t_col[:nnz], t_len=t_ln[:nnz]),
                nnz, P, max_row, k_lo, k_hi)


def pila_forward(pila: Pila, image, out=None):
    """Eq. 1 for all rays: U x K float64 sinogram of an N x N float64 image."""
    torch = _torch()
    g = pila.geom
    assert image.dtype == torch.float64 and image.is_cuda and image.numel() == g.n * g.n
    image = image.contiguous()
    if out is None:
        out = torch.empty(g.n_angles, g.n_bins, dtype=torch.float64, device=image.device)
    _check(load().pila_forward(C.byref(g.c), C.byref(pila.c), image.data_ptr(), out.data_ptr(),
                               _stream()))
    return out


def pila_backproject(pila: Pila, sino, out=None):
    """Transpose of Eq. 1: N x N float64 image from a U x K float64 sinogram."""
    torch = _torch()
    g = pila.geom
    assert sino.dtype == torch.float64 and sino.is_cuda and sino.numel() == g.n_rays
    sino = sino.contiguous()
    if out is None:
        out = torch.empty(g.n, g.n, dtype=torch.float64, device=sino.device)
    _check(load().pila_backproject(C.byref(g.c), C.byref(pila.c), sino.data_ptr(), out.data_ptr(),
                                   _stream()))
    return out


# ---------------------------------------------------------------------------
# annealing
# ---------------------------------------------------------------------------

@dataclass
class SatParams:
    n_steps: int
    seed: int = 0
    chain_id: int = 0
    n_stages: int = 1000
    m_cand: int = 1
    T0: Optional[float] = None      # None: Eq. 8
    TN: Optional[float] = None
    q_auto: int = 200
    precision: str = "f64"
    tn_ratio: float = 1e3
    delta_max: float = 0.05
    f_min: float = 0.0
    f_max: float = 1.0
    resync_every: int = 0
    schedule: str = "linear"        # "linear" (Eq. 2), "exp" (section III-C), "cubic" (Eq. 9)
    proposal: str = "clamp"         # "clamp", or "redraw" (Eq. 3 as printed)

    def c(self) -> CSatParams:
        return CSatParams(self.seed, self.chain_id, self.n_steps, self.n_stages, self.m_cand,
                          self.T0 or 0.0, self.TN or 0.0, self.q_auto,
                          PILA_F32 if self.precision in ("f32", PILA_F32) else PILA_F64,
                          self.tn_ratio, self.delta_max, self.f_min, self.f_max, self.resync_every,
                          SCHEDULES[self.schedule], PROPOSALS[self.proposal])


def _stats_dict(s: CSatStats) -> dict:
    return {k: getattr(s, k) for k, _ in CSatStats._fields_}


def sat_workspace(geom: Geometry, params: SatParams, device=None, minimal: bool = False):
    """sat_run's workspace: sat_workspace_size bytes, or with minimal=True
    sat_workspace_min (the chain state alone)."""
    torch = _torch()
    n = C.c_size_t(0)
    p = params.c()
    fn = load().sat_workspace_min if minimal else load().sat_workspace_size
    _check(fn(C.byref(geom.c), C.byref(p), C.byref(n)))
    return torch.empty(int(n.value), dtype=torch.uint8, device=device or "cuda")


def sat_run(pila: Pila, sino, params: SatParams, image, workspace=None, trace: bool = False,
            stats: bool = True):
    """One SAT chain on the device; image (N x N float64) is updated in place.

    Returns (stats dict or None, trace dict of device tensors or None).
    """
    torch = _torch()
    g = pila.geom
    assert image.dtype == torch.float64 and image.is_cuda and image.is_contiguous()
    assert sino.dtype == torch.float64 and sino.is_cuda and sino.is_contiguous()
    ws = workspace if workspace is not None else sat_workspace(g, params, image.device)
    p = params.c()
    tr = None
    ctr = None
    if trace:
        n = params.n_steps
        tr = dict(m_star=torch.empty(n, dtype=torch.int32, device=image.device),
                  accept=torch.empty(n, dtype=torch.uint8, device=image.device),
                  dC=torch.empty(n, dtype=torch.float64, device=image.device))
        ctr = CSatTrace(tr["m_star"].data_ptr(), tr["accept"].data_ptr(), tr["dC"].data_ptr())
    st = CSatStats() if stats else None
    _check(load().sat_run(C.byref(g.c), C.byref(pila.c), sino.data_ptr(), C.byref(p),
                          image.data_ptr(), ws.data_ptr(), ws.numel(),
                          C.byref(st) if st is not None else None,
                          C.byref(ctr) if ctr is not None else None, _stream()))
    return (_stats_dict(st) if st is not None else None), tr


def sat_run_static(pila: Pila, sino, params: SatParams, image, trace: bool = False,
                   stats: bool = True):
    """sat_run on the library's static device scratch (no allocation by the
    library; the trace tensors, if asked for, are allocated here)."""
    torch = _torch()
    g = pila.geom
    assert image.dtype == torch.float64 and image.is_cuda and image.is_contiguous()
    assert sino.dtype == torch.float64 and sino.is_cuda and sino.is_contiguous()
    p = params.c()
    tr = None
    ctr = None
    if trace:
        n = params.n_steps
        tr = dict(m_star=torch.empty(n, dtype=torch.int32, device=image.device),
                  accept=torch.empty(n, dtype=torch.uint8, device=image.device),
                  dC=torch.empty(n, dtype=torch.float64, device=image.device))
        ctr = CSatTrace(tr["m_star"].data_ptr(), tr["accept"].data_ptr(), tr["dC"].data_ptr())
    st = CSatStats() if stats else None
    _check(load().sat_run_static(C.byref(g.c), C.byref(pila.c), sino.data_ptr(), C.byref(p),
                                 image.data_ptr(), C.byref(st) if st is not None else None,
                                 C.byref(ctr) if ctr is not None else None, _stream()))
    return (_stats_dict(st) if st is not None else None), tr


@dataclass
class Job:
    pila: Pila
    sino: object
    image: object
    params: SatParams
    waves_per_chain: int = 0        # 0: the batch's launch shape


MAX_GROUPS = 8


def sat_run_batch(jobs: List[Job], waves_per_chain: int = 4, chains_per_cu: int = 2,
                  lds_residual: bool = True, workspace=None, stats: bool = True,
                  groups: Optional[list] = None):
    """Many independent chains in persistent launches (one per group of chains
    sharing a body and register shape, side by side); images updated in place.
    groups (a list, optional) receives one dict per group: kernel duration in
    ms from HIP events on its stream, body kind, register shape, chain count."""
    torch = _torch()
    n = len(jobs)
    cj = (CSatJob * max(n, 1))()
    keep = []
    for i, j in enumerate(jobs):
        assert j.image.is_contiguous() and j.sino.is_contiguous()
        cj[i].geom = C.pointer(j.pila.geom.c)
        cj[i].csr = C.pointer(j.pila.c)
        cj[i].d_sino = j.sino.data_ptr()
        cj[i].d_image = j.image.data_ptr()
        cj[i].params = j.params.c()
        cj[i].waves_per_chain = j.waves_per_chain
        keep.append(j)
    lib = load()
    nb = C.c_size_t(0)
    _check(lib.sat_batch_workspace_size(n, cj, C.byref(nb)))
    ws = workspace if workspace is not None else torch.empty(int(nb.value), dtype=torch.uint8,
                                                             device="cuda")
    launch = CSatLaunch(waves_per_chain, chains_per_cu, 1 if lds_residual else 0, 0)
    if groups is not None:
        g_ms = (C.c_float * MAX_GROUPS)()
        g_desc = (C.c_int32 * MAX_GROUPS)()
        g_n = (C.c_int32 * MAX_GROUPS)()
        launch.max_groups = MAX_GROUPS
        launch.h_group_ms = C.cast(g_ms, C.POINTER(C.c_float))
        launch.h_group_desc = C.cast(g_desc, C.POINTER(C.c_int32))
        launch.h_group_chains = C.cast(g_n, C.POINTER(C.c_int32))
    st = (CSatStats * max(n, 1))() if stats else None
    _check(lib.sat_run_batch(n, cj, C.byref(launch), ws.data_ptr(), ws.numel(), st, _stream()))
    if groups is not None:
        groups.clear()
        for i in range(MAX_GROUPS):
            d = int(g_desc[i])
            if d:
                groups.append(dict(ms=float(g_ms[i]), kind=d & 255, cpw=(d >> 8) & 255,
                                   e=(d >> 16) & 255, waves=(d >> 24) & 255, chains=int(g_n[i])))
    return [_stats_dict(st[i]) for i in range(n)] if stats else None


class Graph:
    """A chain's or a batch's launches captured once in a HIP graph
    (sat_graph_* ABI).  launch() replays it on torch's current stream; the
    buffers it was made with (images, sinograms, PILAs, workspace) are kept
    alive here and must not be reallocated; copy starting images into them
    before a launch.  stats() returns the last replay's statistics."""

    def __init__(self, handle, n_chains: int, keep):
        self._h = handle
        self.n_chains = n_chains
        self._keep = keep

    def launch(self):
        _check(load().sat_graph_launch(self._h, _stream()))

    def stats(self) -> List[dict]:
        st = (CSatStats * self.n_chains)()
        _check(load().sat_graph_stats(self._h, st, _stream()))
        return [_stats_dict(st[i]) for i in range(self.n_chains)]

    def close(self):
        if self._h:
            _check(load().sat_graph_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sat_graph(pila: Pila, sino, params: SatParams, image, workspace=None, trace=None) -> Graph:
    """Capture sat_run's launches for these buffers into a graph."""
    torch = _torch()
    g = pila.geom
    assert image.dtype == torch.float64 and image.is_cuda and image.is_contiguous()
    ws = workspace if workspace is not None else sat_workspace(g, params, image.device)
    p = params.c()
    ctr = None
    if trace is not None:
        ctr = CSatTrace(trace["m_star"].data_ptr(), trace["accept"].data_ptr(), trace["dC"].data_ptr())
    h = C.c_void_p()
    _check(load().sat_graph_create(C.byref(g.c), C.byref(pila.c), sino.data_ptr(), C.byref(p),
                                   image.data_ptr(), ws.data_ptr(), ws.numel(),
                                   C.byref(ctr) if ctr is not None else None, C.byref(h)))
    return Graph(h, 1, (pila, sino, image, ws, trace))


def sat_batch_graph(jobs: List[Job], waves_per_chain: int = 4, chains_per_cu: int = 2,
                    lds_residual: bool = True, workspace=None) -> Graph:
    """Capture sat_run_batch's launches for these jobs into a graph."""
    torch = _torch()
    n = len(jobs)
    cj = (CSatJob * max(n, 1))()
    for i, j in enumerate(jobs):
        cj[i].geom = C.pointer(j.pila.geom.c)
        cj[i].csr = C.pointer(j.pila.c)
        cj[i].d_sino = j.sino.data_ptr()
        cj[i].d_image = j.image.data_ptr()
        cj[i].params = j.params.c()
        cj[i].waves_per_chain = j.waves_per_chain
    lib = load()
    nb = C.c_size_t(0)
    _check(lib.sat_batch_workspace_size(n, cj, C.byref(nb)))
    ws = workspace if workspace is not None else torch.empty(int(nb.value), dtype=torch.uint8,
                                                             device="cuda")
    launch = CSatLaunch(waves_per_chain, chains_per_cu, 1 if lds_residual else 0, 0)
    h = C.c_void_p()
    _check(lib.sat_batch_graph_create(n, cj, C.byref(launch), ws.data_ptr(), ws.numel(), C.byref(h)))
    return Graph(h, n, (list(jobs), ws))


def sirt_run(pila: Pila, sino, n_iter: int, lam: float, image, workspace=None,
             cost: bool = True, reuse_layout: bool = False):
    """Simultaneous SIRT (Eq. 10-11); image updated in place; returns costs.
    reuse_layout: the workspace holds the layouts of an earlier call on the
    same PILA (PILA_SIRT_REUSE_LAYOUT)."""
    torch = _torch()
    g = pila.geom
    assert image.dtype == torch.float64 and image.is_cuda and image.is_contiguous()
    assert sino.dtype == torch.float64 and sino.is_cuda and sino.is_contiguous()
    assert workspace is not None or not reuse_layout, "reuse_layout needs the earlier workspace"
    p = CSirtParams(int(n_iter), PILA_SIRT_REUSE_LAYOUT if reuse_layout else 0, float(lam))
    lib = load()
    if workspace is None:
        nb = C.c_size_t(0)
        _check(lib.sirt_workspace_size(C.byref(g.c), C.byref(p), C.byref(nb)))
        workspace = torch.empty(int(nb.value), dtype=torch.uint8, device=image.device)
    costs = np.zeros(max(n_iter, 1), dtype=np.float64) if cost else None
    _check(lib.sirt_run(C.byref(g.c), C.byref(pila.c), sino.data_ptr(), C.byref(p), image.data_ptr(),
                        workspace.data_ptr(), workspace.numel(),
                        costs.ctypes.data if costs is not None else None, _stream()))
    return costs[:n_iter] if costs is not None else None


def sat_drt_run(geom: Geometry, sino, params: SatParams, image, trace: bool = False):
    """SAT with the bilinear DRT in the evaluation step (section III-A's
    comparison method).  Returns (final cost, trace dict of device tensors or
    None); image updated in place."""
    torch = _torch()
    assert image.dtype == torch.float64 and image.is_cuda and image.is_contiguous()
    assert sino.dtype == torch.float64 and sino.is_cuda and sino.is_contiguous()
    p = params.c()
    lib = load()
    nb = C.c_size_t(0)
    _check(lib.sat_drt_workspace_size(C.byref(geom.c), C.byref(p), C.byref(nb)))
    ws = torch.empty(int(nb.value), dtype=torch.uint8, device=image.device)
    tr = ctr = None
    if trace:
        n = params.n_steps
        tr = dict(m_star=torch.empty(n, dtype=torch.int32, device=image.device),
                  accept=torch.empty(n, dtype=torch.uint8, device=image.device),
                  dC=torch.empty(n, dtype=torch.float64, device=image.device))
        ctr = CSatTrace(tr["m_star"].data_ptr(), tr["accept"].data_ptr(), tr["dC"].data_ptr())
    c = C.c_double(0.0)
    _check(lib.sat_drt_run(C.byref(geom.c), sino.data_ptr(), C.byref(p), image.data_ptr(), ws.data_ptr(),
                           ws.numel(), C.byref(c), C.byref(ctr) if ctr is not None else None, _stream()))
    return float(c.value), tr


def sirt_seq_run(pila: Pila, sino, n_iter: int, m_per: int, lam: float, image, seed: int = 0,
                 workspace=None, cost: bool = True):
    """Pixel-by-pixel SIRT (section III-D as described); image updated in
    place; returns Eq. 4 after each iteration."""
    torch = _torch()
    g = pila.geom
    assert image.dtype == torch.float64 and image.is_cuda and image.is_contiguous()
    assert sino.dtype == torch.float64 and sino.is_cuda and sino.is_contiguous()
    p = CSirtSeqParams(int(n_iter), 0, int(m_per), float(lam), int(seed))
    lib = load()
    if workspace is None:
        nb = C.c_size_t(0)
        _check(lib.sirt_seq_workspace_size(C.byref(g.c), C.byref(p), C.byref(nb)))
        workspace = torch.empty(int(nb.value), dtype=torch.uint8, device=image.device)
    costs = np.zeros(max(n_iter, 1), dtype=np.float64) if cost else None
    _check(lib.sirt_seq_run(C.byref(g.c), C.byref(pila.c), sino.data_ptr(), C.byref(p), image.data_ptr(),
                            workspace.data_ptr(), workspace.numel(),
                            costs.ctypes.data if costs is not None else None, _stream()))
    return costs[:n_iter] if costs is not None else None


# ---------------------------------------------------------------------------
# serving
# ---------------------------------------------------------------------------

class Server:
    """Chains admitted against a device-memory budget and run by resident
    workgroups that take new requests as earlier ones finish (srv_* ABI).

    submit() returns a ticket, or None when the request is not admissible now
    (EBUSY); poll() returns None while the chain runs, else its stats (the
    image is final then).  The sinogram and image tensors are kept alive
    until their ticket is reaped.
    """

    def __init__(self, mem_budget: int, max_slots: int = 0, waves_per_chain: int = 0,
                 ring_size: int = 0, idle_us: int = 0, general_slots: int = 0,
                 long_slots: int = 0):
        cfg = CSrvConfig(int(mem_budget), int(max_slots), int(waves_per_chain), int(ring_size),
                         int(idle_us), int(general_slots), int(long_slots))
        h = C.c_void_p()
        _check(load().srv_create(C.byref(cfg), C.byref(h)))
        self._h = h
        self._held = {}

    def prepare(self, geom: Geometry):
        _check(load().srv_prepare(self._h, C.byref(geom.c)))

    def submit(self, geom: Geometry, sino, image, params: SatParams) -> Optional[int]:
        assert sino.is_contiguous() and image.is_contiguous()
        req = CSrvRequest(C.pointer(geom.c), sino.data_ptr(), image.data_ptr(), params.c())
        t = C.c_uint64(0)
        rc = load().srv_submit(self._h, C.byref(req), C.byref(t))
        if rc == PILA_EBUSY:
            return None
        _check(rc)
        self._held[t.value] = (geom, sino, image)
        return t.value

    def poll(self, ticket: int) -> Optional[dict]:
        done = C.c_int32(0)
        st = CSatStats()
        _check(load().srv_poll(self._h, ticket, C.byref(done), C.byref(st)))
        if not done.value:
            return None
        self._held.pop(ticket, None)
        return _stats_dict(st)

    def cancel(self, ticket: int):
        _check(load().srv_cancel(self._h, ticket))

    def status(self) -> dict:
        st = CSrvStatus()
        _check(load().srv_get_status(self._h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in CSrvStatus._fields_}

    def close(self):
        if self._h:
            _check(load().srv_destroy(self._h))
            self._h = None
            self._held.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def device_info() -> dict:
    info = CDeviceInfo()
    _check(load().pila_get_device_info(C.byref(info)))
    return dict(cu_count=info.cu_count, lds_per_block=info.lds_per_block, clock_khz=info.clock_khz,
                warp_size=info.warp_size, hbm_bytes=info.hbm_bytes, name=info.name.decode(),
                wallclock_khz=info.wallclock_khz)
