"""GPU parity of the single-refraction chain (T) against the FP64 oracle:
tree shape, every leaf's position and irradiance bound against the oracle's
bound of the same box, the receiver grid, and the estimates.

Cases: a curved refractor entering a denser medium (eta' = 1/1.5) refined to
an irradiance ratio of 1.1; a refractor leaving a denser medium (eta' = 2),
where part of the domain has total internal reflection and the square root
cannot be bounded (universal bounds and infinite irradiance bounds); and a
4 x 4 water surface with four lights at the default ratio 2.
"""
import gpu_checks
import numpy as np
import pytest

from paper_2504_19163_amd import scenes as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EST_TOL = 1e-5

CASES = {
    "curved": (lambda: S.curved_triangles(8, seed=3, chain="T", eta=1 / 1.5), dict(max_depth=4, alpha=1.1)),
    "steep": (lambda: S.curved_triangles(6, seed=5, chain="T", eta=2.0), dict(max_depth=4, alpha=1.1)),
    "water": (lambda: S.water_surface(m=4, amp_scale=0.04), dict(max_depth=3)),
}


@pytest.fixture(scope="module")
def bbc():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2504_19163_amd import bbc as B
    B.lib()
    return B


@pytest.fixture(scope="module")
def built(bbc, orc):
    out = {}
    for name, (make, params) in CASES.items():
        sc = make()
        osc = orc.OracleScene(sc)
        out[name] = (sc, osc, bbc.Bounds(bbc.DeviceScene(sc), params), orc.OracleBuild(osc, params), params)
    return out


@pytest.mark.parametrize("case", list(CASES))
def test_refraction_tree_and_bounds(bbc, orc, built, case):
    sc, osc, B, Ob, _ = built[case]
    L, OL = B.leaves(), Ob.leaves()
    print(case, "leaves", len(L["tuple"]), "oracle", len(OL["tuple"]), flush=True)
    assert gpu_checks.keyset(L) == gpu_checks.keyset(OL)
    gpu_checks.check_leaf_bounds(orc, osc, L, range(len(L["tuple"])))
    info, st = B.info(), Ob.stats()
    assert info["n_live_tuples"] == st["live_tuples"]
    assert info["n_inf_leaves"] == st["inf_leaves"]


def test_refraction_grid_matches_oracle(bbc, orc, built):
    sc, osc, B, Ob, _ = built["water"]
    off, gt, ge = B.grid()
    G = 512
    rng = np.random.default_rng(2)
    for c in rng.choice(G * G, 4000, replace=False):
        cu, cv = divmod(int(c), G)
        ot, oe = Ob.cell_list(cu, cv)
        a, b = off[c], off[c + 1]
        assert np.array_equal(gt[a:b].astype(np.int64), ot), c
        e = ge[a:b].astype(np.float64)
        fin = np.isfinite(oe)
        assert np.array_equal(np.isfinite(e), fin)
        assert np.all(e[fin] >= oe[fin] * (1 - 1e-12)) and np.all(e[fin] <= oe[fin] * (1 + gpu_checks.BOUND_TOL))
    gpu_checks.check_cover_list(off, gt, ge, Ob, G)


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("mode,omode", [("exhaustive", 1), ("sample", 0)])
def test_refraction_query_matches_oracle(bbc, orc, built, case, mode, omode):
    sc, osc, B, Ob, _ = built[case]
    pts = S.receiver_points(sc, 48)
    m = bbc.QUERY_STAGED | (bbc.QUERY_EXHAUSTIVE if mode == "exhaustive" else 0)
    E, st = B.query(torch.as_tensor(pts, device="cuda"), 8, 21, mode=m, stats=True)
    E = E.cpu().numpy().astype(np.float64)
    st = st.cpu().numpy()
    OE, ost = Ob.query(pts, 8, 21, mode=omode)
    assert np.array_equal(st[:, 0], ost[:, 0])
    assert np.array_equal(st[:, 1], ost[:, 1])
    assert np.array_equal(st[:, 2], ost[:, 2])
    np.testing.assert_allclose(E, OE, rtol=EST_TOL, atol=1e-12)
    Ef, _ = B.query(torch.as_tensor(pts, device="cuda"), 8, 21, mode=m & ~bbc.QUERY_STAGED)
    assert np.array_equal(Ef.cpu().numpy().astype(np.float64), E)


def test_refraction_roots_match_brute_force(bbc, orc, built):
    """Test (c) for the refraction chain: every admissible path found by a
    dense multi-start search over all tuples is found by the GPU estimator
    (exhaustive mode sums exactly these paths)."""
    sc, osc, B, Ob, _ = built["curved"]
    pts = S.random_points(sc, 200, seed=8)
    E, _ = B.query(torch.as_tensor(pts, device="cuda"), 8, 0, mode=bbc.QUERY_EXHAUSTIVE)
    Eb = orc.true_irradiance(osc, pts, lattice=24)  # lattice multi-start over every tuple
    np.testing.assert_allclose(E.cpu().numpy().astype(np.float64), Eb, rtol=1e-5, atol=1e-12)
