"""The pooled Newton kernel of the staged query (starts of 64 pairs spread
over a wave's lanes, FP32 passes of a few iterations, FP64 polish 64 at a
time) against the kernel that gives each lane one pair for all of its starts:
the per-start arithmetic, the start order of the per-pair root sum and the
deduplication are the same, so estimates, per-point statistics and work
counters must agree bit for bit, for every pass length and chain (and, for
two reflections, with the pooled kernel testing runs of leaves before their
leaves)."""
import numpy as np
import pytest

from paper_2504_19163_amd import scenes as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = {
    # single reflection: 512-triangle heightfield, 8192-triangle sphere
    "heightfield": (lambda: S.heightfield_mirror(16), dict(max_depth=4), 96, 16),
    "sphere": (lambda: S.displaced_sphere(5), dict(max_depth=6), 160, 64),
    # refraction: 8 x 8 water surface, four lights
    "water": (lambda: S.water_surface(m=8, amp_scale=0.04), dict(max_depth=4), 96, 64),
    # two reflections: 32 + 32 facing-wall triangles (many leaves per tuple)
    "walls": (lambda: S.facing_walls(4), dict(max_depth=4), 64, 256),
}


@pytest.fixture(scope="module")
def bbc():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2504_19163_amd import bbc as B
    B.lib()
    return B


def _run(bbc, B, pts, spp, steps, mode):
    B.set_tuning(bbc.TUNE_NEWTON_STEPS, steps)
    E, st, hs = B.query(pts, spp, 11, mode=mode, stats=True, host_stats=True)
    torch.cuda.synchronize()
    return E.cpu().numpy(), st.cpu().numpy(), hs


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("exhaustive", [False, True])
def test_pooled_newton_matches_lane_per_pair(bbc, name, exhaustive):
    make, params, grid, spp = CASES[name]
    sc = make()
    B = bbc.Bounds(bbc.DeviceScene(sc), params)
    pts = torch.as_tensor(S.receiver_points(sc, grid), device="cuda")
    mode = bbc.QUERY_STAGED | (bbc.QUERY_EXHAUSTIVE if exhaustive else 0)
    print(name, "exhaustive" if exhaustive else "sampled", "points", pts.shape[1], flush=True)
    if name == "walls":
        # tuples of 12 leaves or more: the two-reflection kernel tests the
        # unions of their runs of 8 leaves before the leaves themselves
        t = B.leaves()["tuple"]
        assert np.bincount(t).max() >= 12
    E0, st0, h0 = _run(bbc, B, pts, spp, 0, mode)
    assert h0["n_roots"] > 0
    for steps, results in ((1, 96), (3, 96), (4, 96), (20, 96), (4, 1), (2, 5)):
        # a small result buffer sends most pairs with roots through the redo
        # kernel, whose work counters cover only the roots it adds
        B.set_tuning(bbc.TUNE_NEWTON_RESULTS, results)
        E1, st1, h1 = _run(bbc, B, pts, spp, steps, mode)
        assert np.array_equal(E0.view(np.uint32), E1.view(np.uint32)), (name, steps, results)
        assert np.array_equal(st0.view(np.uint32), st1.view(np.uint32)), (name, steps, results)
        for f in ("n_pairs", "n_newton", "n_roots", "n_iter_fp32", "n_iter_fp64"):
            assert h0[f] == h1[f], (name, steps, results, f)
    B.set_tuning(bbc.TUNE_NEWTON_STEPS, 4)
    B.set_tuning(bbc.TUNE_NEWTON_RESULTS, 96)


def test_newton_knob_validation(bbc):
    sc = S.heightfield_mirror(4)
    B = bbc.Bounds(bbc.DeviceScene(sc), dict(max_depth=2))
    assert B.get_tuning(bbc.TUNE_NEWTON_STEPS) == 4
    assert B.get_tuning(bbc.TUNE_NEWTON_RESULTS) == 96
    for knob, bad in ((bbc.TUNE_NEWTON_STEPS, -1), (bbc.TUNE_NEWTON_STEPS, 21), (bbc.TUNE_NEWTON_RESULTS, 0),
                      (bbc.TUNE_NEWTON_RESULTS, 97)):
        with pytest.raises(RuntimeError):
            B.set_tuning(knob, bad)
    B.set_tuning(bbc.TUNE_NEWTON_STEPS, 0)
    assert B.get_tuning(bbc.TUNE_NEWTON_STEPS) == 0
