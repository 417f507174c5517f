"""GPU parity of the two-reflection chain (RR) against the FP64 oracle: tuple
construction and the tree (same live tuples and leaves), every leaf's
position bound against the oracle's bound of the same box, the grid, the
estimates, the double-mirror image source and brute-force enumeration."""
import gpu_checks
import numpy as np
import pytest

from paper_2504_19163_amd import scenes as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bbc():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2504_19163_amd import bbc as B
    B.lib()
    return B


@pytest.fixture(scope="module")
def walls(bbc, orc):
    sc = S.facing_walls(4)
    params = dict(max_depth=4)
    osc = orc.OracleScene(sc)
    return sc, osc, bbc.Bounds(bbc.DeviceScene(sc), params), orc.OracleBuild(osc, params)


def test_rr_double_mirror_image_source_on_gpu(bbc):
    sc = S.double_mirror()
    B = bbc.Bounds(bbc.DeviceScene(sc), dict(max_depth=3))
    pts = S.receiver_points(sc, 24)
    E, st = B.query(torch.as_tensor(pts, device="cuda"), 4, 0, mode=bbc.QUERY_EXHAUSTIVE | bbc.QUERY_STAGED,
                    stats=True)
    lx, ly, lz = sc["epos"][:, 0].astype(float)
    d = pts.astype(float) - np.array([lx, ly, 4.0 + lz])[:, None]
    ref = np.abs(d[2]) / np.linalg.norm(d, axis=0) ** 3
    np.testing.assert_allclose(E.cpu().numpy().astype(np.float64), ref, rtol=1e-5)
    assert np.all(st.cpu().numpy()[:, 2] == 1)


def test_rr_tree_and_bounds(bbc, orc, walls):
    sc, osc, B, Ob = walls
    L, OL = B.leaves(), Ob.leaves()
    print("leaves", len(L["tuple"]), "oracle", len(OL["tuple"]), flush=True)
    assert gpu_checks.keyset(L) == gpu_checks.keyset(OL)
    gpu_checks.check_leaf_bounds(orc, osc, L, range(len(L["tuple"])), e_face_value=True)
    info, st = B.info(), Ob.stats()
    assert info["n_tuples"] == st["tuples"]
    assert info["n_live_tuples"] == st["live_tuples"]
    assert info["n_leaves"] == st["leaves"]


def test_rr_grid_matches_oracle(bbc, orc, walls):
    sc, osc, B, Ob = walls
    off, gt, ge = B.grid()
    G = 512
    rng = np.random.default_rng(3)
    for c in rng.choice(G * G, 4000, replace=False):
        cu, cv = divmod(int(c), G)
        ot, oe = Ob.cell_list(cu, cv)
        a, b = off[c], off[c + 1]
        assert np.array_equal(gt[a:b].astype(np.int64), ot), c
        # E~ from a ratio taken at face value on both sides: equal up to the
        # order of the FP64 sums and the outward FP32 rounding
        e = ge[a:b].astype(np.float64)
        fin = np.isfinite(oe)
        assert np.array_equal(np.isfinite(e), fin), c
        assert np.all(np.abs(e[fin] - oe[fin]) <= gpu_checks.BOUND_TOL * np.abs(oe[fin])), c
    gpu_checks.check_cover_list(off, gt, ge, Ob, G)


@pytest.mark.parametrize("form", ["staged", "fused"])
@pytest.mark.parametrize("mode,omode", [("exhaustive", 1), ("sample", 0)])
def test_rr_query_matches_oracle(bbc, orc, walls, form, mode, omode):
    sc, osc, B, Ob = walls
    pts = S.random_points(sc, 2000, seed=7)
    m = (bbc.QUERY_STAGED if form == "staged" else bbc.QUERY_FUSED) | (bbc.QUERY_EXHAUSTIVE if mode == "exhaustive"
                                                                         else 0)
    E, st = B.query(torch.as_tensor(pts, device="cuda"), 16, 4, mode=m, stats=True)
    E = E.cpu().numpy().astype(np.float64)
    st = st.cpu().numpy()
    OE, ost = Ob.query(pts, 16, 4, mode=omode)
    assert np.array_equal(st[:, 0], ost[:, 0])
    assert np.array_equal(st[:, 1], ost[:, 1])
    assert np.array_equal(st[:, 2], ost[:, 2])
    np.testing.assert_allclose(E, OE, rtol=1e-5, atol=1e-12)
    assert (OE > 0).sum() > 200


def test_rr_exhaustive_close_to_brute_force(bbc, orc, walls):
    sc, osc, B, Ob = walls
    pts = S.random_points(sc, 150, seed=9)
    E, _ = B.query(torch.as_tensor(pts, device="cuda"), 1, 0, mode=bbc.QUERY_EXHAUSTIVE)
    E = E.cpu().numpy().astype(np.float64)
    Et = orc.true_irradiance(osc, pts, lattice=16)
    assert np.all(E <= Et * (1 + 1e-5) + 1e-12)
    assert np.isclose(E, Et, rtol=1e-5, atol=1e-12).mean() >= 0.95


def test_rr_called_box_evaluation_gives_the_same_build(bbc):
    """The subdivision kernel with the box evaluation as a called function
    (BBC_TUNE_RR_OUTLINED; the LDS block and the helpers' reduction buffers
    then go through the lowering of non-kernel functions) builds exactly the
    tree, bounds and grid of the inlined kernel, with and without the degree
    reduction."""
    sc = S.facing_walls(8)
    for flags in (0, bbc.FLAG_DEGREE_REDUCTION):
        p = dict(max_depth=5, alpha=10.0, flags=flags)
        B1, B2 = bbc.Bounds(bbc.DeviceScene(sc), p), bbc.Bounds(bbc.DeviceScene(sc), p)
        B2.set_tuning(bbc.TUNE_RR_OUTLINED, 1)
        B2.rebuild()
        L1, L2 = B1.leaves(), B2.leaves()
        print("flags", flags, "leaves", len(L1["tuple"]), flush=True)
        assert len(L1["tuple"]) > 1000
        for k in ("tuple", "box", "uk", "E"):
            assert np.array_equal(np.asarray(L1[k]).view(np.uint8), np.asarray(L2[k]).view(np.uint8)), k
        g1, g2 = B1.grid(), B2.grid()
        for a, b in zip(g1, g2):
            assert np.array_equal(np.asarray(a).view(np.uint8), np.asarray(b).view(np.uint8))
        B1.free()
        B2.free()
