"""Test (b) of the oracle: every leaf's position and irradiance bound contains
the true u_k and E_k of every admissible path through a dense grid of its box
(Sec. 4.2, Eq. eq_bbound; Sec. 6.1 subdivision), including pieces around a
fold, where the only valid bound is infinite (Fig. 2D examples, case (c)), and
refraction, whose bound relies on the remainder variables (Sec. 4.3)."""
import numpy as np
import pytest

from paper_2504_19163_amd import scenes as S


def _check_containment(orc, osc, build, tuples=None, n=17):
    L = build.leaves()
    keep = np.ones(len(L["tuple"]), bool) if tuples is None else np.isin(L["tuple"], tuples)
    n_paths = 0
    n_inf = 0
    for k in np.nonzero(keep)[0]:
        t = L["tuple"][k]
        u0, u1, v0, v1 = L["box"][k]
        ulo, uhi, vlo, vhi = L["uk"][k]
        Elo, Ehi = L["E"][k]
        n_inf += np.isinf(Ehi)
        for u in np.linspace(u0, u1, n):
            for v in np.linspace(v0, v1, n):
                e = orc.eval_path(osc, t, u, v)
                if not e["admissible"]:
                    continue
                if not (0 <= e["uk"] <= 1 and 0 <= e["vk"] <= 1):
                    continue
                n_paths += 1
                tol = 1e-9
                assert ulo - tol <= e["uk"] <= uhi + tol, (t, u, v, e["uk"], ulo, uhi)
                assert vlo - tol <= e["vk"] <= vhi + tol, (t, u, v, e["vk"], vlo, vhi)
                assert e["Ek"] <= Ehi * (1 + 1e-9), (t, u, v, e["Ek"], Ehi)
                assert e["Ek"] >= Elo * (1 - 1e-9), (t, u, v, e["Ek"], Elo)
    return n_paths, n_inf


def test_containment_heightfield(orc):
    sc = S.heightfield_mirror(16)
    osc = orc.OracleScene(sc)
    b = orc.OracleBuild(osc, dict(max_depth=4))
    n_paths, n_inf = _check_containment(orc, osc, b, tuples=np.arange(0, 512, 16))
    assert n_paths > 5000


def test_containment_fixed_depth_and_folds(orc):
    # strongly tilted normals fold the caustic; fixed-depth subdivision keeps
    # pieces straddling the fold, whose irradiance bound must be infinite
    sc = S.curved_triangles(4, seed=3)
    sc["nrm"] = sc["nrm"].copy()
    rng = np.random.default_rng(5)
    for t in range(4):
        for k in range(3):
            nn = np.array([rng.uniform(-0.8, 0.8), rng.uniform(-0.8, 0.8), 1.0])
            sc["nrm"][3 * k:3 * k + 3, t] = nn / np.linalg.norm(nn)
    osc = orc.OracleScene(sc)
    b = orc.OracleBuild(osc, dict(max_depth=3, flags=1))
    n_paths, n_inf = _check_containment(orc, osc, b, n=21)
    assert n_paths > 1000
    # a fold exists inside a piece iff det J changes sign there; such pieces
    # must carry an infinite irradiance bound
    L = b.leaves()
    found_fold = 0
    for k in range(len(L["tuple"])):
        t = L["tuple"][k]
        u0, u1, v0, v1 = L["box"][k]
        signs = set()
        for u in np.linspace(u0, u1, 9):
            for v in np.linspace(v0, v1, 9):
                if u + v <= 1:
                    signs.add(np.sign(orc.eval_path(osc, t, u, v)["detJ"]))
        if len(signs - {0.0}) == 2:
            found_fold += 1
            assert np.isinf(L["E"][k][1])
    assert found_fold > 0


@pytest.mark.parametrize("eta", [1.0 / 1.5, 1.33])
def test_containment_refraction(orc, eta):
    sc = S.curved_triangles(3, seed=9, chain="T", eta=eta)
    osc = orc.OracleScene(sc)
    b = orc.OracleBuild(osc, dict(max_depth=3))
    n_paths, _ = _check_containment(orc, osc, b, n=15)
    assert n_paths > 500
