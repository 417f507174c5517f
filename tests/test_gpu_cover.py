"""The cover-all list on the GPU (grid recording and every query form) against
the FP64 oracle: a heightfield on a 64 x 64 grid with cover_frac = 0.002 puts
about half of the tuples in the list.  The cells' lists and the cover-all list
must equal the oracle's, the candidate counts |U| and the Bernoulli decisions
must be identical, estimates agree to 1e-5; with cover_frac = 0 the exhaustive
estimates are those of the list-free grid."""
import gpu_checks
import numpy as np
import pytest

from paper_2504_19163_amd import scenes as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

G = 64
PARAMS = dict(max_depth=4, grid_res=G, cover_frac=0.002)


@pytest.fixture(scope="module")
def bbc():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2504_19163_amd import bbc as B
    B.lib()
    return B


@pytest.fixture(scope="module")
def built(bbc, orc):
    sc = S.heightfield_mirror(16)
    B = bbc.Bounds(bbc.DeviceScene(sc), PARAMS)
    Ob = orc.OracleBuild(orc.OracleScene(sc), PARAMS)
    return sc, B, Ob


def test_grid_and_cover_list_match_oracle(bbc, built):
    sc, B, Ob = built
    info = B.info()
    st = Ob.stats()
    assert info["n_cover_tuples"] == st["cover_tuples"] > 0
    assert info["n_grid_entries"] == st["grid_entries"]
    off, gt, ge = B.grid()
    for c in range(G * G):
        ot, oe = Ob.cell_list(*divmod(c, G))
        a, b = off[c], off[c + 1]
        assert np.array_equal(gt[a:b].astype(np.int64), ot), c
        e = ge[a:b].astype(np.float64)
        fin = np.isfinite(oe)
        assert np.array_equal(np.isfinite(e), fin)
        assert np.all(e[fin] >= oe[fin] * (1 - 1e-12)) and np.all(e[fin] <= oe[fin] * (1 + gpu_checks.BOUND_TOL))
    gpu_checks.check_cover_list(off, gt, ge, Ob, G)


@pytest.mark.parametrize("form", ["fused", "staged"])
@pytest.mark.parametrize("exhaustive", [False, True])
def test_queries_with_cover_list_match_oracle(bbc, built, form, exhaustive):
    sc, B, Ob = built
    pts = S.receiver_points(sc, 96, grid_res=G)
    m = bbc.QUERY_FUSED if form == "fused" else bbc.QUERY_STAGED
    if exhaustive:
        m |= bbc.QUERY_EXHAUSTIVE
    W = 8
    print(form, "exhaustive" if exhaustive else "sampled", pts.shape[1], flush=True)
    E, st = B.query(torch.as_tensor(pts, device="cuda"), W, 5, mode=m, stats=True)
    E = E.cpu().numpy().astype(np.float64)
    st = st.cpu().numpy()
    OE, ost = Ob.query(pts, W, 5, mode=1 if exhaustive else 0)
    assert np.array_equal(st[:, 0], ost[:, 0])  # |U| = cell list + cover-all list
    assert np.array_equal(st[:, 1], ost[:, 1])  # identical Bernoulli decisions
    assert np.array_equal(st[:, 2], ost[:, 2])  # roots
    assert np.count_nonzero(OE) > 20
    np.testing.assert_allclose(E, OE, rtol=1e-5, atol=1e-12)


def test_exhaustive_estimates_equal_list_free_grid(bbc, built):
    sc, B, Ob = built
    B0 = bbc.Bounds(bbc.DeviceScene(sc), dict(PARAMS, cover_frac=0.0))
    assert B0.info()["n_cover_tuples"] == 0
    pts = torch.as_tensor(S.random_points(sc, 5000, seed=4, grid_res=G), device="cuda")
    m = bbc.QUERY_STAGED | bbc.QUERY_EXHAUSTIVE
    E1, s1 = B.query(pts, 1, 0, mode=m, stats=True)
    E0, s0 = B0.query(pts, 1, 0, mode=m, stats=True)
    assert torch.all(s1[:, 0] >= s0[:, 0])
    np.testing.assert_allclose(E1.cpu().numpy(), E0.cpu().numpy(), rtol=1e-6, atol=0)
    B0.free()
