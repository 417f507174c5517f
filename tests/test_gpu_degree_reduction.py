"""GPU parity of the degree reduction (Sec. 6.1, "Degree reduction"; build
flag BBC_FLAG_DEGREE_REDUCTION) on the two-reflection chain against the FP64
oracle with the same flag (8): the tree, every leaf's bounds against the
oracle's bound of the same box (det M's coefficients at face value on both
sides, as without the flag; the reduction and its remainder on top), the
grid and the estimates.  The reduced bound also contains the full-degree one
on the boxes both builds keep as leaves."""
import gpu_checks
import numpy as np
import pytest

from paper_2504_19163_amd import scenes as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REDUCE = 8
PARAMS = dict(max_depth=5, alpha=10.0)


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
    osc = orc.OracleScene(sc)
    p = dict(PARAMS, flags=REDUCE)
    print("facing walls 32 + 32 triangles, depth 5, degree reduction", flush=True)
    return sc, osc, bbc.Bounds(bbc.DeviceScene(sc), p), orc.OracleBuild(osc, p)


def test_reduced_tree_and_bounds_match_oracle(bbc, orc, walls):
    sc, osc, B, Ob = walls
    L, OL = B.leaves(), Ob.leaves()
    print("leaves", len(L["tuple"]), "oracle", len(OL["tuple"]), flush=True)
    assert gpu_checks.keyset(L) == gpu_checks.keyset(OL)
    # E_lo of a box whose fitted numerator nearly cancels against its
    # remainder is tiny and known to the rounding of E_hi's scale only
    gpu_checks.check_leaf_bounds(orc, osc, L, range(len(L["tuple"])), e_face_value=True, flags=REDUCE, e_abs=1e-9)
    info, st = B.info(), Ob.stats()
    assert info["n_leaves"] == st["leaves"]
    assert info["n_inf_leaves"] == st["inf_leaves"]


def test_reduced_bound_contains_full_degree_bound(bbc, walls):
    sc, osc, B, Ob = walls
    B0 = bbc.Bounds(bbc.DeviceScene(sc), PARAMS)
    L, L0 = B.leaves(), B0.leaves()
    key = {k: i for i, k in enumerate(zip(L0["tuple"].tolist(), map(tuple, L0["box"].tolist())))}
    n = 0
    for i, k in enumerate(zip(L["tuple"].tolist(), map(tuple, L["box"].tolist()))):
        j = key.get(k)
        if j is None:
            continue
        e, e0 = L["E"][i].astype(np.float64), L0["E"][j].astype(np.float64)
        # both ratios at face value: containment up to the FP64 sums' order
        assert e[0] <= e0[0] * (1 + 1e-6) and e[1] >= e0[1] * (1 - 1e-6), (k, e, e0)
        n += 1
    assert n > 300
    B0.free()


def test_reduced_grid_and_queries_match_oracle(bbc, orc, walls):
    sc, osc, B, Ob = walls
    off, gt, ge = B.grid()
    G = 512
    rng = np.random.default_rng(8)
    for c in rng.choice(G * G, 3000, replace=False):
        ot, oe = Ob.cell_list(*divmod(int(c), G))
        a, b = off[c], off[c + 1]
        assert np.array_equal(gt[a:b].astype(np.int64), ot), c
        e = ge[a:b].astype(np.float64)
        fin = np.isfinite(oe)
        assert np.array_equal(np.isfinite(e), fin), c
        assert np.all(np.abs(e[fin] - oe[fin]) <= gpu_checks.BOUND_TOL * np.abs(oe[fin])), c
    pts = S.random_points(sc, 1500, seed=12)
    for mode, omode in ((bbc.QUERY_STAGED | bbc.QUERY_EXHAUSTIVE, 1), (bbc.QUERY_STAGED, 0)):
        E, st = B.query(torch.as_tensor(pts, device="cuda"), 16, 4, mode=mode, stats=True)
        OE, ost = Ob.query(pts, 16, 4, mode=omode)
        st = st.cpu().numpy()
        assert np.array_equal(st[:, 0], ost[:, 0])
        same = st[:, 1] == ost[:, 1]  # selection decisions on E~ within rounding of a threshold may differ
        assert same.mean() >= 0.99
        assert np.count_nonzero(OE) > 100
        np.testing.assert_allclose(E.cpu().numpy().astype(np.float64)[same], OE[same], rtol=1e-5, atol=1e-12)
