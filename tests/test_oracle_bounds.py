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


def _small_box_ratios(orc, osc, build, divs=(32, 64), n_max=40):
    """For leaves with a finite bound around an admissible centre: on boxes of
    half-width w/d around that centre, E_lo / min E_k, E_hi / max E_k and
    (E_hi - E_lo) / (max - min) over a 9 x 9 sample of the box."""
    L = build.leaves()
    rows = []
    for k in np.nonzero(np.isfinite(L["E"][:, 1]))[0]:
        t = L["tuple"][k]
        u0, u1, v0, v1 = L["box"][k]
        uc, vc = 0.5 * (u0 + u1), 0.5 * (v0 + v1)
        if not orc.eval_path(osc, t, uc, vc)["admissible"]:
            continue
        res = []
        for d in divs:
            h = (u1 - u0) / d
            bb = orc.box_bound(osc, t, [uc - h, uc + h, vc - h, vc + h])
            if not (bb["live"] and np.isfinite(bb["E"][1])):
                break
            E = [orc.eval_path(osc, t, u, v) for u in np.linspace(uc - h, uc + h, 9)
                 for v in np.linspace(vc - h, vc + h, 9)]
            if not all(e["admissible"] for e in E):
                break
            E = np.array([e["Ek"] for e in E])
            res.append((bb["E"][0] / E.min(), bb["E"][1] / E.max(), (bb["E"][1] - bb["E"][0]) / (E.max() - E.min())))
        if len(res) == len(divs):
            rows.append(res)
        if len(rows) >= n_max:
            break
    return np.array(rows)


@pytest.mark.parametrize("case", ["reflection", "refraction"])
def test_irradiance_bound_is_tight_on_small_boxes(orc, case):
    """The explicit irradiance bound (Sec. 4.4, Eq. eq_irr_term3a with the
    factor-wise bound of |n_g.d0| / |d0|^3) on small boxes around admissible
    paths: it contains the sampled E_k, its ends sit within 1 % of the
    sampled extremes at half-width w/32, its width is within a small factor
    of the sampled range, and its excess over the sampled extremes halves
    (at least) when the box halves -- the product of the factors' ranges
    converges linearly, each factor's Bernstein range quadratically (Sec.
    4.1).  A lower end collapsing to 0, an extra factor on the upper end or a
    wrong term in det M or Q^3 fails one of these."""
    if case == "reflection":
        sc, params, wmax = S.heightfield_mirror(16), dict(max_depth=4), 1.5
    else:
        sc, params, wmax = S.water_surface(m=8, amp_scale=0.04), dict(max_depth=4), 2.5
    osc = orc.OracleScene(sc)
    rows = _small_box_ratios(orc, osc, orc.OracleBuild(osc, params))
    assert len(rows) >= 20
    lo, hi, width = rows[:, :, 0], rows[:, :, 1], rows[:, :, 2]
    assert np.all(lo <= 1 + 1e-9) and np.all(hi >= 1 - 1e-9)  # containment
    assert lo[:, 0].min() >= 0.99 and hi[:, 0].max() <= 1.01
    assert np.all(width <= wmax)
    shrink_hi = (hi[:, 0] - 1) / np.maximum(hi[:, 1] - 1, 1e-300)
    shrink_lo = (1 - lo[:, 0]) / np.maximum(1 - lo[:, 1], 1e-300)
    assert np.median(shrink_hi) >= 1.7 and np.median(shrink_lo) >= 1.7
