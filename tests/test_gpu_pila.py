"""GPU parity: PILA build and PILA projections against the oracle (MI355X)."""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_1411_4622_amd as P
    P.load()
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return P


def _sorted_rays(off, pix, ln):
    """Oracle ray-major listing re-ordered by pixel within each ray."""
    G = len(off) - 1
    rid = np.repeat(np.arange(G), np.diff(off))
    order = np.lexsort((pix, rid))
    return pix[order], ln[order]


def _check_pila(P, N, U, K, ang, mask, dtype, tol=1e-12):
    print("pila parity N=%d U=%d K=%d dtype=%s masked=%s" % (N, U, K, dtype, mask is not None),
          flush=True)
    geom = P.Geometry(N, ang, K, mask, dtype)
    pl = P.pila_build(geom)
    (rp, col, ln), (off, pix, rl) = oracle.pila(N, U, K, ang, mask, with_rays=True)
    assert pl.nnz == len(col)
    assert np.array_equal(pl.row_ptr.cpu().numpy(), rp)
    assert np.array_equal(pl.col.cpu().numpy(), col)
    gl = pl.len.cpu().numpy().astype(np.float64)
    if dtype == "f64":
        assert np.max(np.abs(gl - ln), initial=0.0) <= tol
    else:
        assert np.all(np.abs(gl - ln) <= 6.0e-8 * ln + tol)
    assert np.array_equal(pl.t_row_ptr.cpu().numpy(), off)
    sp, sl = _sorted_rays(off, pix, rl)
    assert np.array_equal(pl.t_col.cpu().numpy(), sp)
    tl = pl.t_len.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(tl - sl), initial=0.0) <= (tol if dtype == "f64" else 6e-8 * 1.5)
    sup = np.flatnonzero(np.ones(N * N) if mask is None else np.asarray(mask).reshape(-1))
    assert np.array_equal(pl.support.cpu().numpy(), sup)
    return pl, (rp, col, ln)


@pytest.mark.parametrize("N,U,K", [(8, 4, 8), (8, 8, 11), (7, 90, 10), (16, 180, 23), (9, 36, 13),
                                   (1, 3, 1), (2, 4, 3), (5, 1, 7)])
def test_pila_small_grids(P, N, U, K):
    _check_pila(P, N, U, K, datagen.angles_deg(U), None, "f64")


def test_pila_odd_angles(P):
    ang = np.array([-30.0, 0.0, 12.5, 45.0, 90.0, 135.0, 180.0, 200.0, 270.0, 333.3, 1e-3])
    _check_pila(P, 10, len(ang), 15, ang, None, "f64")


def test_pila_c1_geometry(P):
    _check_pila(P, 64, 90, 64, datagen.angles_deg(90), None, "f64")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_pila_c2_geometry_masked(P, dtype):
    _check_pila(P, 256, 180, 367, datagen.angles_deg(180), datagen.circle_mask(256), dtype)


def test_pila_ragged_sizes(P):
    # sizes that are not multiples of the wavefront or block shape
    _check_pila(P, 100, 77, 143, datagen.angles_deg(77), datagen.circle_mask(100), "f64")


def test_pila_full_size_1024_sampled(P):
    """The 1024 x 1024, 720-angle, 1449-bin geometry at full size: sampled
    pixel rows and ray rows against the oracle's ray traces, and the
    whole-square chord of every ray."""
    N, U, K = 1024, 720, 1449
    ang = datagen.angles_deg(U)
    mask = datagen.circle_mask(N)
    geom = P.Geometry(N, ang, K, mask, "f64")
    print("full-size build N=%d U=%d K=%d" % (N, U, K), flush=True)
    pl = P.pila_build(geom)
    torch.cuda.synchronize()
    rp = pl.row_ptr.cpu().numpy()
    trp = pl.t_row_ptr.cpu().numpy()
    rng = np.random.default_rng(4)
    sup = np.flatnonzero(mask.reshape(-1))
    # pixels: random support pixels plus boundary and centre pixels
    picks = list(rng.choice(sup, 12, replace=False)) + [int(sup[0]), int(sup[-1]), (N // 2) * N + N // 2]
    for p in picks:
        g_o, l_o = oracle.pixel_row(N, U, K, ang, int(p), mask)
        b, e = int(rp[p]), int(rp[p + 1])
        g_g = pl.col[b:e].cpu().numpy()
        l_g = pl.len[b:e].cpu().numpy()
        assert np.array_equal(g_g, g_o), p
        assert np.max(np.abs(l_g - l_o), initial=0.0) <= 1e-12
    # rays: random rays plus near-axis angles
    rays = list(rng.integers(0, U * K, 40)) + [1 * K + 700, 359 * K + 724, 361 * K + 10, 719 * K + 725]
    for g in rays:
        u, k = divmod(int(g), K)
        pix, ln = oracle.trace_ray(N, K, ang[u], k, mask)
        order = np.argsort(pix)
        b, e = int(trp[g]), int(trp[g + 1])
        assert np.array_equal(pl.t_col[b:e].cpu().numpy(), pix[order]), g
        assert np.max(np.abs(pl.t_len[b:e].cpu().numpy() - ln[order]), initial=0.0) <= 1e-12
    # every ray: projection of the all-ones support equals the chord through the
    # support (checked on the unmasked build below for the closed form)
    del pl
    torch.cuda.empty_cache()


def test_forward_all_ones_is_square_chord_full_size(P):
    N, U, K = 1024, 720, 1449
    ang = datagen.angles_deg(U)
    geom = P.Geometry(N, ang, K, None, "f32")
    pl = P.pila_build(geom)
    ones = torch.ones(N, N, dtype=torch.float64, device="cuda")
    proj = P.pila_forward(pl, ones).cpu().numpy()
    cs = oracle.trig(ang)
    sk = datagen.bin_centres(K)
    # slab clipping of each ray against [-N/2, N/2]^2, vectorised
    h = N / 2.0
    c = cs[:, 0][:, None]
    s = cs[:, 1][:, None]
    px, py, dx, dy = sk[None, :] * c, sk[None, :] * s, -s + 0 * sk[None, :], c + 0 * sk[None, :]
    lo = np.full((U, K), -np.inf)
    hi = np.full((U, K), np.inf)
    ok = np.ones((U, K), bool)
    for p_, d_ in ((px, dx), (py, dy)):
        par = d_ == 0.0
        ok &= ~par | ((p_ >= -h) & (p_ < h))
        with np.errstate(divide="ignore", invalid="ignore"):
            t1 = np.where(par, -np.inf, (-h - p_) / np.where(par, 1.0, d_))
            t2 = np.where(par, np.inf, (h - p_) / np.where(par, 1.0, d_))
        lo = np.maximum(lo, np.minimum(t1, t2))
        hi = np.minimum(hi, np.maximum(t1, t2))
    want = np.where(ok, np.maximum(hi - lo, 0.0), 0.0)
    # float32 lengths: relative 6e-8 per entry
    assert np.all(np.abs(proj - want) <= 1e-12 * N + 1.2e-7 * want)


@pytest.mark.parametrize("N,U,K,masked", [(64, 90, 64, False), (96, 60, 137, True), (33, 45, 47, True)])
def test_forward_and_back_projection(P, N, U, K, masked):
    ang = datagen.angles_deg(U)
    mask = datagen.circle_mask(N) if masked else None
    geom = P.Geometry(N, ang, K, mask, "f64")
    pl = P.pila_build(geom)
    csr = oracle.pila(N, U, K, ang, mask)
    rng = np.random.default_rng(N + U)
    f = rng.random((N, N))
    y = rng.standard_normal((U, K))
    pf = P.pila_forward(pl, torch.from_numpy(f).cuda()).cpu().numpy()
    of = oracle.forward(N, U, K, csr, f)
    scale = oracle.forward(N, U, K, csr, np.abs(f))
    assert np.all(np.abs(pf - of) <= 1e-12 * scale + 1e-300)
    pb = P.pila_backproject(pl, torch.from_numpy(y).cuda()).cpu().numpy()
    ob = oracle.backward(N, csr, y)
    bscale = oracle.backward(N, csr, np.abs(y))
    assert np.all(np.abs(pb - ob) <= 1e-12 * bscale + 1e-300)


def test_projection_deterministic(P):
    N, U, K = 128, 90, 182
    geom = P.Geometry(N, datagen.angles_deg(U), K, datagen.circle_mask(N), "f32")
    pl = P.pila_build(geom)
    f = torch.rand(N, N, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(1))
    a = P.pila_forward(pl, f)
    b = P.pila_forward(pl, f)
    assert torch.equal(a, b)
