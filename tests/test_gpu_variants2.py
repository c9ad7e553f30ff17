"""GPU parity of the pixel-by-pixel SIRT (section III-D as described) and of
the DRT comparison chain (section III-A) against the oracle (MI355X)."""
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


# 32 x 32: projections in LDS; 96 x 96 x 180 angles: in global memory
@pytest.mark.parametrize("N,U,K,lam,iters,masked", [(32, 30, 46, 1.0, 3, True), (96, 180, 136, 0.5, 2, True),
                                                    (24, 12, 37, 1.0, 4, False)])
def test_sirt_seq_matches_oracle(P, N, U, K, lam, iters, masked):
    ell = datagen.random_ellipses(N + 3, N, 6)
    sl = datagen.make_slice(N, U, K, ell, masked=masked, I0=1e4, noise_seed=4)
    m_per = int(sl.mask.sum()) if masked else N * N
    csr = oracle.pila(N, U, K, sl.angles, sl.mask)
    f_o, c_o = oracle.sirt_seq_run(N, U, K, csr, sl.sino, sl.f0, iters, m_per, lam, seed=21, mask=sl.mask)
    print("sirt_seq N=%d U=%d" % (N, U), flush=True)
    pl = P.pila_build(P.Geometry(N, sl.angles, K, sl.mask, "f64"))
    img = torch.from_numpy(sl.f0.copy()).cuda()
    cost = P.sirt_seq_run(pl, torch.from_numpy(sl.sino).cuda(), iters, m_per, lam, img, seed=21)
    f_g = img.cpu().numpy()
    assert np.max(np.abs(f_g - f_o)) <= 1e-10 * max(1.0, np.max(np.abs(f_o)))
    assert np.max(np.abs(cost - c_o) / c_o) <= 1e-10
    assert cost[-1] < cost[0]


def test_sirt_seq_f32_lengths_and_edge_cases(P):
    N, U, K = 40, 36, 57
    ell = datagen.random_ellipses(12, N, 6)
    sl = datagen.make_slice(N, U, K, ell, masked=True, I0=1e4, noise_seed=5)
    csr = oracle.pila(N, U, K, sl.angles, sl.mask)
    csr32 = (csr[0], csr[1], csr[2].astype(np.float32).astype(np.float64))
    f_o, _ = oracle.sirt_seq_run(N, U, K, csr32, sl.sino, sl.f0, 2, 500, 1.0, seed=2, mask=sl.mask)
    pl = P.pila_build(P.Geometry(N, sl.angles, K, sl.mask, "f32"))
    img = torch.from_numpy(sl.f0.copy()).cuda()
    P.sirt_seq_run(pl, torch.from_numpy(sl.sino).cuda(), 2, 500, 1.0, img, seed=2)
    assert np.max(np.abs(img.cpu().numpy() - f_o)) <= 1e-8
    # no iterations / no updates: the image is untouched
    img = torch.from_numpy(sl.f0.copy()).cuda()
    assert len(P.sirt_seq_run(pl, torch.from_numpy(sl.sino).cuda(), 0, 100, 1.0, img)) == 0
    P.sirt_seq_run(pl, torch.from_numpy(sl.sino).cuda(), 3, 0, 1.0, img)
    assert np.array_equal(img.cpu().numpy(), sl.f0)


@pytest.mark.parametrize("N,U,K,M,masked", [(16, 12, 23, 1, True), (24, 18, 35, 4, False),
                                            (20, 30, 29, 3, True)])
def test_satdrt_matches_oracle(P, N, U, K, M, masked):
    ell = datagen.random_ellipses(N, N, 5)
    sl = datagen.make_slice(N, U, K, ell, masked=masked, I0=1e4, noise_seed=6)
    kw = dict(seed=3, chain_id=1, n_steps=300, n_stages=10, m_cand=M, T0=5e-3, TN=5e-6, delta_max=0.2)
    f_o, c_o, tr_o = oracle.satdrt_run(N, U, K, sl.angles, sl.sino, sl.f0, mask=sl.mask, **kw)
    geom = P.Geometry(N, sl.angles, K, sl.mask, "f64")
    prm = P.SatParams(n_steps=300, seed=3, chain_id=1, n_stages=10, m_cand=M, T0=5e-3, TN=5e-6,
                      delta_max=0.2)
    img = torch.from_numpy(sl.f0.copy()).cuda()
    print("satdrt N=%d M=%d" % (N, M), flush=True)
    c_g, tr = P.sat_drt_run(geom, torch.from_numpy(sl.sino).cuda(), prm, img, trace=True)
    tr = {k: v.cpu().numpy() for k, v in tr.items()}
    assert np.array_equal(tr["m_star"], tr_o["m_star"])
    assert np.array_equal(tr["accept"], tr_o["accept"])
    # Delta C is a difference of two costs: its rounding scales with C
    assert np.max(np.abs(tr["dC"] - tr_o["dC"])) <= 1e-12 * c_o
    assert np.max(np.abs(img.cpu().numpy() - f_o)) <= 1e-12
    assert abs(c_g - c_o) <= 1e-12 * c_o
    assert 0 < int(tr["accept"].sum()) < 300
