"""The cover-all list of the bound storage (Sec. 6.1, bound storage, with the
cover-all reading): a tuple whose leaves would be splatted into at least
cover_frac * G^2 cells is stored once, in a list every shading point reads
after its cell's list, with the largest E_hi of its leaves.

Pins, independent of how the oracle stores the grid:
  * conservative storage: for every leaf and every cell its closed position
    bound touches, the leaf's tuple is a candidate of that cell with a
    per-tuple bound >= the leaf's E_hi (the property Eq. eq_pertuple_b needs);
  * the decision is the stated footprint rule, recomputed here from the
    exported leaves; cover_frac = 0 keeps every tuple in the cells, a tiny
    cover_frac moves every tuple with leaves to the list;
  * the cover-all tuples' bound is the maximum over all of their leaves;
  * the exhaustive estimate (every candidate with P = 1) is the same with and
    without the list: a tuple added to a far cell has no leaf covering the
    point, hence no Newton start and no contribution;
  * the sampled estimator stays unbiased with the list (mean over 400 seeds
    within 4 standard errors of the exhaustive sum at each of 24 points)."""
import numpy as np
import pytest

from paper_2504_19163_amd import scenes as S


def _cell(x, G):
    return np.minimum(G - 1, np.floor(np.clip(x, 0.0, 1.0) * G).astype(np.int64))


def _footprints(L, G):
    cu0, cu1 = _cell(L["uk"][:, 0], G), _cell(L["uk"][:, 1], G)
    cv0, cv1 = _cell(L["uk"][:, 2], G), _cell(L["uk"][:, 3], G)
    return cu0, cu1, cv0, cv1, (cu1 - cu0 + 1) * (cv1 - cv0 + 1)


@pytest.fixture(scope="module")
def scene(orc):
    sc = S.heightfield_mirror(16)
    return sc, orc.OracleScene(sc)


@pytest.mark.parametrize("frac", [0.0, 0.002, 0.5, 1e-9])
def test_cover_decision_and_conservative_storage(orc, scene, frac):
    sc, osc = scene
    G = 64
    b = orc.OracleBuild(osc, dict(max_depth=4, grid_res=G, cover_frac=frac))
    L = b.leaves()
    cu0, cu1, cv0, cv1, fp = _footprints(L, G)
    tuples = np.unique(L["tuple"])
    per = {int(t): fp[L["tuple"] == t].sum() for t in tuples}
    emax = {int(t): L["E"][L["tuple"] == t, 1].max() for t in tuples}
    want = sorted(t for t in per if frac > 0 and per[t] >= frac * G * G)
    ct, ce = b.cover_list()
    assert ct.tolist() == want
    for t, e in zip(ct, ce):
        assert e == emax[int(t)]
    if frac == 1e-9:
        assert ct.tolist() == sorted(per)
    if frac == 0.0:
        assert len(ct) == 0
    if frac == 0.002:
        assert 0 < len(ct) < len(per)  # the rule splits this scene's tuples
    st = b.stats()
    assert st["cover_tuples"] == len(ct)
    cover = set(ct.tolist())
    n_cell_entries = 0
    for cu in range(G):
        for cv in range(G):
            t, e = b.cell_list(cu, cv)
            assert not (set(t.tolist()) & cover)  # a tuple is in the cells or in the list, never both
            n_cell_entries += len(t)
    assert st["grid_entries"] == n_cell_entries + len(ct)
    # every leaf is found under each cell it touches, with a bound >= its E_hi
    rng = np.random.default_rng(3)
    for k in rng.choice(len(L["tuple"]), min(300, len(L["tuple"])), replace=False):
        t = int(L["tuple"][k])
        for cu in range(cu0[k], cu1[k] + 1, max(1, (cu1[k] - cu0[k]) // 3)):
            for cv in range(cv0[k], cv1[k] + 1, max(1, (cv1[k] - cv0[k]) // 3)):
                U, Et = b.candidates(cu, cv)
                hit = np.nonzero(U == t)[0]
                assert len(hit) == 1, (k, cu, cv)
                assert Et[hit[0]] >= L["E"][k, 1]


def test_exhaustive_estimate_is_unchanged_by_the_list(orc, scene):
    sc, osc = scene
    pts = S.random_points(sc, 400, seed=11, grid_res=64)
    off = orc.OracleBuild(osc, dict(max_depth=4, grid_res=64, cover_frac=0.0))
    on = orc.OracleBuild(osc, dict(max_depth=4, grid_res=64, cover_frac=0.002))
    assert on.stats()["cover_tuples"] > 0
    E0, s0 = off.query(pts, 1, 0, mode=1)
    E1, s1 = on.query(pts, 1, 0, mode=1)
    assert np.all(s1[:, 0] >= s0[:, 0])  # U only grows
    assert np.count_nonzero(E0) > 50
    np.testing.assert_allclose(E1, E0, rtol=1e-12, atol=0)


def test_sampled_estimator_with_the_list_is_unbiased(orc, scene):
    sc, osc = scene
    pts = S.random_points(sc, 24, seed=12, grid_res=64)
    on = orc.OracleBuild(osc, dict(max_depth=4, grid_res=64, cover_frac=0.002))
    ex, _ = on.query(pts, 1, 0, mode=1)
    W = 4
    runs = np.stack([on.query(pts, W, s, mode=0)[0] for s in range(400)])
    mean = runs.mean(0)
    se = runs.std(0, ddof=1) / np.sqrt(runs.shape[0])
    lit = ex > 0
    assert lit.sum() >= 5
    z = np.abs(mean - ex) / np.maximum(se, 1e-30)
    assert np.all(z[lit & (se > 0)] < 4.0), z[lit]
    assert np.all(mean[~lit] == 0.0)
