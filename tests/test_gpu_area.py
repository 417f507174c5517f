"""GPU parity of area lights (single reflection; the light's two parameters
are two more axes of every polynomial, and a query draws one light point per
selected pair from Philox streams 3 and 4) against the FP64 oracle: tree
shape, every leaf's position and irradiance bound against the oracle's bound
of the same box (rounded outward: containing the oracle's, within the bound
tolerance), the grid and the estimates with the same light-point draws (the
polish takes the FP64 light point, so estimates agree to 1e-5)."""
import gpu_checks
import numpy as np
import pytest

from paper_2504_19163_amd import scenes as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = {
    "heightfield": (lambda: S.area_light(S.heightfield_mirror(8), [0.6, 0.0, 0.0], [0.0, 0.4, 0.0]),
                    dict(max_depth=3)),
    "flat": (lambda: S.area_light(S.flat_mirror(), [0.5, 0.0, 0.0], [0.0, 0.3, 0.0]), dict(max_depth=4)),
    "curved": (lambda: S.area_light(S.curved_triangles(4, seed=7), [0.3, 0.1, 0.0], [0.0, 0.3, 0.05]),
               dict(max_depth=3)),
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
        out[name] = (sc, osc, bbc.Bounds(bbc.DeviceScene(sc), params), orc.OracleBuild(osc, params))
    return out


@pytest.mark.parametrize("case", list(CASES))
def test_area_tree_and_bounds(bbc, orc, built, case):
    sc, osc, B, Ob = built[case]
    L, OL = B.leaves(), Ob.leaves()
    print(case, "leaves", len(L["tuple"]), "oracle", len(OL["tuple"]), flush=True)
    assert len(L["tuple"]) > 0
    assert gpu_checks.keyset(L) == gpu_checks.keyset(OL)
    # position and irradiance bounds carry rounding control: they contain the
    # oracle's and exceed them by at most the tolerance
    gpu_checks.check_leaf_bounds(orc, osc, L, range(len(L["tuple"])))
    info, st = B.info(), Ob.stats()
    assert info["n_live_tuples"] == st["live_tuples"]
    assert info["n_inf_leaves"] == st["inf_leaves"]


def test_area_grid_matches_oracle(bbc, orc, built):
    sc, osc, B, Ob = built["heightfield"]
    off, gt, ge = B.grid()
    G = 512
    rng = np.random.default_rng(5)
    for c in rng.choice(G * G, 3000, replace=False):
        cu, cv = divmod(int(c), G)
        ot, oe = Ob.cell_list(cu, cv)
        a, b = off[c], off[c + 1]
        assert np.array_equal(gt[a:b].astype(np.int64), ot), c
        e = ge[a:b].astype(np.float64)
        fin = np.isfinite(oe)
        assert np.array_equal(np.isfinite(e), fin), c
        assert np.all(np.abs(e[fin] - oe[fin]) <= gpu_checks.BOUND_TOL * np.abs(oe[fin])), c
    gpu_checks.check_cover_list(off, gt, ge, Ob, G)


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("mode,omode", [("exhaustive", 1), ("sample", 0)])
def test_area_query_matches_oracle(bbc, orc, built, case, mode, omode):
    sc, osc, B, Ob = built[case]
    pts = S.receiver_points(sc, 48)
    m = bbc.QUERY_STAGED | (bbc.QUERY_EXHAUSTIVE if mode == "exhaustive" else 0)
    E, st = B.query(torch.as_tensor(pts, device="cuda"), 8, 13, mode=m, stats=True)
    E = E.cpu().numpy().astype(np.float64)
    st = st.cpu().numpy()
    OE, ost = Ob.query(pts, 8, 13, mode=omode)
    assert np.array_equal(st[:, 0], ost[:, 0])
    assert np.array_equal(st[:, 1], ost[:, 1])
    assert np.count_nonzero(OE) > 50
    np.testing.assert_allclose(E, OE, rtol=1e-5, atol=1e-12)
    Ef, _ = B.query(torch.as_tensor(pts, device="cuda"), 8, 13, mode=m & ~bbc.QUERY_STAGED)
    np.testing.assert_allclose(Ef.cpu().numpy().astype(np.float64), E, rtol=1e-6, atol=1e-12)


def test_area_light_needs_single_reflection(bbc):
    sc = S.area_light(S.curved_triangles(3, seed=9, chain="T", eta=1.0 / 1.5), [0.3, 0, 0], [0, 0.3, 0])
    with pytest.raises(Exception):
        bbc.Bounds(bbc.DeviceScene(sc), dict(max_depth=2))
