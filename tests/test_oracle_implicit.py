"""The oracle's irradiance bound of refraction by implicit differentiation
(Sec. 4.4, "Implicit differentiation"; build flag 4).

Pins: (a) at admissible paths of the forward map, the specular polynomials F
(Snell's law along b) and G (coplanarity) vanish and -J_1^{-1} J_k, formed here
in numpy from finite differences of F and G, reproduces the forward map's
1/|det du_k/du1|: the formula the bound is built from, checked against the
path evaluator rather than against itself; (b) every leaf's implicit bound
contains E_k of every admissible path through its box, and most leaves are
bounded; (c) on small boxes approaching total internal reflection the bound is
close to the sampled range of E_k."""
import numpy as np
import pytest

from paper_2504_19163_amd import scenes as S
from test_oracle_bounds import _check_containment

IMPLICIT = 4


def _tir_scene():
    # one flat refracting triangle (eta = n_i / n_t = 1.33) lit obliquely: the
    # incidence angle reaches the critical angle inside the triangle
    pos = np.zeros((9, 1))
    nrm = np.zeros((9, 1))
    P = np.array([[0.0, -0.2, 0.0], [0.4, -0.2, 0.0], [0.0, 0.2, 0.0]])
    for k in range(3):
        pos[3 * k:3 * k + 3, 0] = P[k]
        nrm[3 * k:3 * k + 3, 0] = [0.0, 0.0, 1.0]
    return S._scene("T", pos, nrm, [-1.0, 0.0, 1.1], [1.0], [-10.0, -10.0, -1.0], [20.0, 0.0, 0.0],
                    [0.0, 20.0, 0.0], eta=1.33, name="tir1")


def _geom(sc, t):
    f = lambda a, k: a[3 * k:3 * k + 3, t].astype(np.float64)
    p0, p1, p2 = f(sc["pos"], 0), f(sc["pos"], 1), f(sc["pos"], 2)
    n0, n1, n2 = f(sc["nrm"], 0), f(sc["nrm"], 1), f(sc["nrm"], 2)
    return p0, p1 - p0, p2 - p0, n0, n1 - n0, n2 - n0


def _FG(sc, t, p, b):
    p0, e1, e2, n0, dn1, dn2 = _geom(sc, t)
    u, v, uk, vk = p
    x0 = sc["epos"][:, 0].astype(np.float64)
    xk = sc["q0"].astype(np.float64) + uk * sc["f1"].astype(np.float64) + vk * sc["f2"].astype(np.float64)
    x1 = p0 + u * e1 + v * e2
    n = n0 + u * dn1 + v * dn2
    d0, d1 = x1 - x0, xk - x1
    c0, c1 = np.cross(d0, n), np.cross(d1, n)
    eta = float(sc["eta"])
    return np.array([(d0 @ d0) * (c1 @ b) ** 2 - eta ** 2 * (d1 @ d1) * (c0 @ b) ** 2, c0 @ d1])


@pytest.mark.parametrize("which", ["tir", "curved"])
def test_specular_polynomials_give_the_forward_jacobian(orc, which):
    sc = _tir_scene() if which == "tir" else S.curved_triangles(3, seed=9, chain="T", eta=1.0 / 1.5)
    osc = orc.OracleScene(sc)
    rng = np.random.default_rng(11)
    checked = 0
    for _ in range(300):
        t = int(rng.integers(0, sc["pos"].shape[1]))
        u, v = rng.uniform(0, 1, 2)
        if u + v > 1:
            continue
        e = orc.eval_path(osc, t, u, v)
        if not e["admissible"]:
            continue
        p = np.array([u, v, e["uk"], e["vk"]])
        for b in (np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0])):
            FG = _FG(sc, t, p, b)
            h = 1e-6
            J = np.zeros((2, 4))
            for a in range(4):
                dp = np.zeros(4)
                dp[a] = h
                J[:, a] = (_FG(sc, t, p + dp, b) - _FG(sc, t, p - dp, b)) / (2 * h)
            scale = np.abs(J).max(axis=1)
            assert np.all(np.abs(FG) <= 1e-6 * scale), (which, t, u, v, FG, scale)
            ratio = abs(np.linalg.det(J[:, 2:]) / np.linalg.det(J[:, :2]))
            assert ratio == pytest.approx(1.0 / abs(e["detJ"]), rel=1e-5), (which, t, u, v)
        checked += 1
    assert checked > 40


@pytest.mark.parametrize("eta", [1.0 / 1.5, 1.33])
def test_implicit_bounds_contain_paths(orc, eta):
    sc = S.curved_triangles(3, seed=9, chain="T", eta=eta)
    osc = orc.OracleScene(sc)
    b = orc.OracleBuild(osc, dict(max_depth=3, flags=IMPLICIT))
    n_paths, n_inf = _check_containment(orc, osc, b, n=15)
    n_leaves = len(b.leaves()["tuple"])
    assert n_paths > 5000
    assert n_inf < 0.5 * n_leaves


def test_implicit_bound_tight_near_critical_angle(orc):
    sc = _tir_scene()
    osc = orc.OracleScene(sc)
    for u0 in np.arange(0.30, 0.52, 0.04):
        box = [u0, u0 + 0.02, 0.0, 0.02]
        ob = orc.box_bound(osc, 0, box, True, IMPLICIT)
        Es = []
        for u in np.linspace(box[0], box[1], 7):
            for v in np.linspace(box[2], box[3], 7):
                e = orc.eval_path(osc, 0, u, v)
                if e["admissible"] and 0 <= e["uk"] <= 1 and 0 <= e["vk"] <= 1:
                    Es.append(e["Ek"])
        lo, hi = ob["E"]
        assert ob["live"] and np.isfinite(hi) and lo > 0, (u0, ob)
        assert lo <= min(Es) * (1 + 1e-9) and max(Es) <= hi * (1 + 1e-9), (u0, lo, hi, min(Es), max(Es))
        assert hi / lo <= 1.25 * max(Es) / min(Es), (u0, lo, hi, min(Es), max(Es))
