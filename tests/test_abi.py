"""The C-ABI library: symbols and argument errors (CPU only, no device calls)."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pila.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def P():
    import paper_1411_4622_amd as P
    if not os.path.exists(P.LIB_PATH):
        from paper_1411_4622_amd import build
        build.build()
    P.load()
    return P


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("pila_build", "pila_forward", "pila_backproject", "sat_run", "sat_run_batch",
              "sirt_run", "pila_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(P):
    out = subprocess.run(["nm", "-D", "--defined-only", P.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    for n in _declared():
        assert n in exported, n
    lib = P.load()
    for n in _declared():
        assert hasattr(lib, n)


def test_binding_names_match_header(P):
    assert sorted(P.EXPORTED) == _declared()


def _geom(P, n=8, U=4, K=8, dtype="f64", angles=None):
    ang = np.arange(U) * 180.0 / U if angles is None else angles
    return P.Geometry(n, ang, K, None, dtype)


def test_bad_geometry_is_einval(P):
    lib = P.load()
    from paper_1411_4622_amd._binding import CCsr
    csr = CCsr()
    assert lib.pila_build(None, C.byref(csr), None, 0, None) == P._binding.PILA_EINVAL
    assert "NULL" in P.last_error()
    for n, U, K in ((0, 4, 8), (8, 0, 8), (8, 4, 0)):
        g = P.Geometry(max(n, 1), np.zeros(max(U, 1)), max(K, 1))
        g.c.n, g.c.n_angles, g.c.n_bins = n, U, K
        assert lib.pila_build(C.byref(g.c), C.byref(csr), None, 0, None) == P._binding.PILA_EINVAL
    g = _geom(P, angles=np.array([0.0, np.nan, 10.0, 20.0]))
    assert lib.pila_build(C.byref(g.c), C.byref(csr), None, 0, None) == P._binding.PILA_EINVAL
    assert "not finite" in P.last_error()
    g = _geom(P)
    g.c.len_dtype = 7
    assert lib.pila_build(C.byref(g.c), C.byref(csr), None, 0, None) == P._binding.PILA_EINVAL
    g = _geom(P)
    assert lib.pila_build(C.byref(g.c), C.byref(csr), None, 0, None) == P._binding.PILA_EINVAL
    assert "allocated" in P.last_error()
    # caller scratch: size query, then NULL or too small is refused before any device work
    fake = 0x1000
    nb = C.c_size_t(0)
    assert lib.pila_build_scratch_size(C.byref(g.c), C.byref(nb)) == 0 and nb.value == 8 * 8 + 256
    csr = CCsr(0, 0, 0, 0, -1, fake, None, None, None, fake, fake, None, None)
    assert lib.pila_build(C.byref(g.c), C.byref(csr), None, nb.value, None) == P._binding.PILA_EINVAL
    assert lib.pila_build(C.byref(g.c), C.byref(csr), fake, nb.value - 1, None) == P._binding.PILA_ENOMEM
    assert "scratch" in P.last_error()


def test_bad_sat_arguments(P):
    lib = P.load()
    from paper_1411_4622_amd._binding import CCsr, CSatParams, CSatStats
    g = _geom(P)
    csr = CCsr()
    prm = P.SatParams(n_steps=10, T0=1e-2, TN=1e-6).c()
    # missing PILA arrays
    rc = lib.sat_run(C.byref(g.c), C.byref(csr), None, C.byref(prm), None, None, 0, None, None, None)
    assert rc == P._binding.PILA_EINVAL
    fake = 0x1000
    csr = CCsr(10, 5, 4, 0, 3, fake, fake, fake, fake, fake, fake, fake, fake)
    for bad in (dict(m_cand=0), dict(m_cand=65), dict(n_stages=0), dict(precision="f32"),
                dict(T0=None, q_auto=0), dict(T0=1.0, TN=-1.0), dict(delta_max=float("nan")),
                dict(f_min=1.0, f_max=0.0), dict(n_steps=-1)):
        kw = dict(n_steps=10, T0=1e-2, TN=1e-6)
        kw.update(bad)
        p = P.SatParams(**kw).c()
        rc = lib.sat_run(C.byref(g.c), C.byref(csr), fake, C.byref(p), fake, fake, 1 << 30, None,
                         None, None)
        assert rc == P._binding.PILA_EINVAL, bad
    for field, val in (("schedule", 3), ("schedule", -1), ("proposal", 2)):
        p = P.SatParams(n_steps=10, T0=1e-2, TN=1e-6).c()
        setattr(p, field, val)
        rc = lib.sat_run(C.byref(g.c), C.byref(csr), fake, C.byref(p), fake, fake, 1 << 30, None,
                         None, None)
        assert rc == P._binding.PILA_EINVAL and field in P.last_error(), (field, val)
    # workspace too small
    p = P.SatParams(n_steps=10, T0=1e-2, TN=1e-6).c()
    rc = lib.sat_run(C.byref(g.c), C.byref(csr), fake, C.byref(p), fake, fake, 16, None, None, None)
    assert rc == P._binding.PILA_ENOMEM
    assert "workspace" in P.last_error()


def test_static_entry_refuses_oversized_chain(P):
    """sat_run_static checks the chain state against its static array before
    any device work: a 3000 x 3000 ray FP64 residual (72 MB) is above 64 MiB."""
    lib = P.load()
    from paper_1411_4622_amd._binding import CCsr
    g = P.Geometry(8, np.arange(3000) * 180.0 / 3000, 3000, None, "f64")
    fake = 0x1000
    csr = CCsr(10, 5, 4, 0, 3, fake, fake, fake, fake, fake, fake, fake, fake)
    prm = P.SatParams(n_steps=10, T0=1e-2, TN=1e-6).c()
    rc = lib.sat_run_static(C.byref(g.c), C.byref(csr), fake, C.byref(prm), fake, None, None, None)
    assert rc == P._binding.PILA_ENOMEM
    assert "static scratch" in P.last_error()


def test_graph_argument_errors(P):
    lib = P.load()
    h = C.c_void_p()
    assert lib.sat_graph_launch(None, None) == P._binding.PILA_EINVAL
    assert lib.sat_graph_stats(None, None, None) == P._binding.PILA_EINVAL
    assert lib.sat_graph_destroy(None) == 0
    assert lib.sat_graph_create(None, None, None, None, None, None, 0, None, None) == P._binding.PILA_EINVAL
    assert lib.sat_batch_graph_create(0, None, None, None, 0, C.byref(h)) == P._binding.PILA_EINVAL


def test_workspace_sizes(P):
    lib = P.load()
    from paper_1411_4622_amd._binding import CSirtParams
    g = _geom(P, n=64, U=90, K=64)
    n = C.c_size_t(0)
    p64 = P.SatParams(n_steps=1, precision="f64").c()
    assert lib.sat_workspace_size(C.byref(g.c), C.byref(p64), C.byref(n)) == 0
    assert n.value >= 90 * 64 * 8
    # the smallest workspace is the chain state; the full one adds room for
    # a split chain's 15 residual and image copies when the residual may not
    # fit in LDS and M >= 4 (here 90 x 64 x 8 bytes = 45 KB: it fits)
    lo = C.c_size_t(0)
    assert lib.sat_workspace_min(C.byref(g.c), C.byref(p64), C.byref(lo)) == 0
    assert 90 * 64 * 8 <= lo.value <= n.value
    big = _geom(P, n=256, U=720, K=363)
    p32 = P.SatParams(n_steps=1, precision="f32", m_cand=32).c()
    assert lib.sat_workspace_min(C.byref(big.c), C.byref(p32), C.byref(lo)) == 0
    assert lib.sat_workspace_size(C.byref(big.c), C.byref(p32), C.byref(n)) == 0
    r_bytes = 720 * 368 * 4
    assert n.value - lo.value >= 15 * (r_bytes + 256 * 256 * 8)
    assert lib.sat_workspace_min(None, C.byref(p32), C.byref(lo)) == P._binding.PILA_EINVAL
    sp = CSirtParams(10, 0, 0.1)
    assert lib.sirt_workspace_size(C.byref(g.c), C.byref(sp), C.byref(n)) == 0
    assert n.value >= 2 * 90 * 64 * 8
    sp = CSirtParams(-1, 0, 0.1)
    assert lib.sirt_workspace_size(C.byref(g.c), C.byref(sp), C.byref(n)) == P._binding.PILA_EINVAL


def test_sirt_unknown_flags_are_einval(P):
    """Refused before any device work: host-side checks only (the pointers
    are never dereferenced)."""
    from paper_1411_4622_amd._binding import CCsr, CSirtParams
    lib = P.load()
    g = _geom(P, n=16, U=12, K=23)
    fake = 256  # non-NULL placeholders
    csr = CCsr(1, 1, 1, 0, -1, fake, fake, fake, fake, fake, fake, fake, fake)
    sp = CSirtParams(3, 2, 0.5)
    rc = lib.sirt_run(C.byref(g.c), C.byref(csr), C.c_void_p(fake), C.byref(sp), C.c_void_p(fake),
                      C.c_void_p(fake), C.c_size_t(1 << 40), None, None)
    assert rc == P._binding.PILA_EINVAL
    assert "flags" in P.last_error()


def test_batch_argument_errors(P):
    lib = P.load()
    n = C.c_size_t(0)
    assert lib.sat_batch_workspace_size(-1, None, C.byref(n)) == P._binding.PILA_EINVAL
    assert lib.sat_batch_workspace_size(0, None, C.byref(n)) == 0
    assert lib.sat_run_batch(0, None, None, None, 0, None, None) == P._binding.PILA_ENOMEM


def test_server_argument_errors(P):
    from paper_1411_4622_amd._binding import CSrvConfig, CSrvStatus
    lib = P.load()
    h = C.c_void_p()
    E = P._binding.PILA_EINVAL
    assert lib.srv_create(None, C.byref(h)) == E
    assert lib.srv_create(C.byref(CSrvConfig(1 << 30, 0, 5, 0, 0, 0, 0)), C.byref(h)) == E
    assert "waves_per_chain" in P.last_error()
    assert lib.srv_create(C.byref(CSrvConfig(1 << 30, 0, 8, 3, 0, 0, 0)), C.byref(h)) == E
    assert "power of two" in P.last_error()
    assert lib.srv_create(C.byref(CSrvConfig(1 << 10, 0, 8, 0, 0, 0, 0)), C.byref(h)) == P._binding.PILA_ENOMEM
    done = C.c_int32(0)
    assert lib.srv_poll(None, 0, C.byref(done), None) == E
    assert lib.srv_cancel(None, 0) == E
    assert lib.srv_get_status(None, C.byref(CSrvStatus())) == E
    assert lib.srv_submit(None, None, None) == E
    assert lib.srv_prepare(None, None) == E
    assert lib.srv_destroy(None) == 0


def test_product_path_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_1411_4622_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
