"""Pins of the oracle's path evaluation (Sec. 4.3-4.4) against closed forms and
first principles that do not reuse its formulas:

* a flat mirror reflects like the mirror image of the light (image source);
* refraction with eta' = 1 leaves rays straight (direct light);
* the irradiance E_k = I0 dOmega0/dA_k equals the solid angle of a tiny ray
  triangle at the light divided by the area it lands on (finite geometry,
  not the chain rule of Eq. eq_dwda);
* the receiver Jacobian matches finite differences of u_k(u1);
* the secant remainder of sqrt is attained and never exceeded (Sec. 4.3).
"""
import numpy as np
import pytest

from paper_2504_19163_amd import scenes as S


def _solid_angle(a, b, c):
    """Solid angle of the spherical triangle spanned by vectors a, b, c
    (Van Oosterom and Strackee, 1983)."""
    la, lb, lc = np.linalg.norm(a), np.linalg.norm(b), np.linalg.norm(c)
    num = abs(np.dot(a, np.cross(b, c)))
    den = la * lb * lc + np.dot(a, b) * lc + np.dot(a, c) * lb + np.dot(b, c) * la
    return 2.0 * np.arctan2(num, den)


def test_flat_mirror_image_source(orc):
    sc = S.flat_mirror()
    osc = orc.OracleScene(sc)
    x0 = sc["epos"][:, 0].astype(float)
    x0m = x0 * np.array([1, 1, -1])  # image of the light in the plane z = 0
    pts = S.receiver_points(sc, 24)
    E = orc.true_irradiance(osc, pts, lattice=8)
    n_lit = 0
    for i in range(pts.shape[1]):
        x = pts[:, i].astype(float)
        d = x - x0m
        hit = x0m + (-x0m[2] / d[2]) * d
        u, v = (hit[0] + 1) / 2, (hit[1] + 1) / 2
        inside = u >= 0 and v >= 0 and u + v <= 1
        ref = abs(d[2]) / np.linalg.norm(d) ** 3 if inside else 0.0
        n_lit += inside
        assert abs(E[i] - ref) <= 1e-10 * max(ref, 1e-3)
    assert n_lit > 50


def test_refraction_unit_eta_is_direct_light(orc):
    # eta' = 1: beta = (d.n)^2, the refracted direction is d itself
    sc = S.curved_triangles(1, chain="T", eta=1.0)
    sc["nrm"][:] = np.array([0, 0, 1] * 3, np.float32).reshape(9, 1)  # flat interface
    osc = orc.OracleScene(sc)
    x0 = sc["epos"][:, 0].astype(float)
    P = sc["pos"].astype(float)[:, 0].reshape(3, 3)
    pts = S.receiver_points(sc, 20)
    E = orc.true_irradiance(osc, pts, lattice=8)
    n_lit = 0
    for i in range(pts.shape[1]):
        x = pts[:, i].astype(float)
        d = x - x0
        hit = x0 + (-x0[2] / d[2]) * d
        # barycentric coordinates of hit in the triangle
        M = np.stack([P[1] - P[0], P[2] - P[0]], 1)[:2]
        u, v = np.linalg.solve(M, (hit - P[0])[:2])
        inside = u >= 0 and v >= 0 and u + v <= 1
        ref = abs(d[2]) / np.linalg.norm(d) ** 3 if inside else 0.0
        n_lit += inside
        assert abs(E[i] - ref) <= 1e-9 * max(ref, 1e-3)
    assert n_lit > 20


@pytest.mark.parametrize("chain,eta", [("R", 1.0), ("T", 1.0 / 1.5)])
def test_irradiance_equals_solid_angle_over_area(orc, chain, eta):
    sc = S.curved_triangles(3, chain=chain, eta=eta)
    osc = orc.OracleScene(sc)
    x0 = sc["epos"][:, 0].astype(float)
    q0, f1, f2 = (sc[k].astype(float) for k in ("q0", "f1", "f2"))
    rng = np.random.default_rng(11)
    checked = 0
    for t in range(osc.n_tuples):
        for _ in range(6):
            u, v = rng.uniform(0.1, 0.45, 2)
            e = orc.eval_path(osc, t, u, v)
            if not e["admissible"]:
                continue
            h = 2e-5
            cs = [(u, v), (u + h, v), (u, v + h)]
            ev = [orc.eval_path(osc, t, a, b) for a, b in cs]
            xk = [q0 + p["uk"] * f1 + p["vk"] * f2 for p in ev]
            area = 0.5 * np.linalg.norm(np.cross(xk[1] - xk[0], xk[2] - xk[0]))
            om = _solid_angle(*(p["x1"] - x0 for p in ev))
            assert abs(om / area - e["Ek"]) <= 2e-3 * e["Ek"], (t, u, v)
            checked += 1
    assert checked >= 5


def test_jacobian_matches_finite_differences(orc):
    sc = S.heightfield_mirror(4)
    osc = orc.OracleScene(sc)
    rng = np.random.default_rng(12)
    for t in range(0, osc.n_tuples, 3):
        u, v = rng.uniform(0.1, 0.4, 2)
        e = orc.eval_path(osc, t, u, v)
        h = 1e-6
        ep = orc.eval_path(osc, t, u + h, v)
        em = orc.eval_path(osc, t, u - h, v)
        fp = orc.eval_path(osc, t, u, v + h)
        fm = orc.eval_path(osc, t, u, v - h)
        J = np.array([[ep["uk"] - em["uk"], fp["uk"] - fm["uk"]], [ep["vk"] - em["vk"], fp["vk"] - fm["vk"]]]) / (2 * h)
        assert abs(np.linalg.det(J) - e["detJ"]) <= 1e-5 * max(1.0, abs(e["detJ"]))


def test_sqrt_secant_remainder_is_tight(orc):
    for blo, bhi in [(0.01, 1.0), (0.5, 0.6), (1e-4, 4.0), (2.0, 2.0000001)]:
        a, b, dlo, dhi = orc.sqrt_secant(blo, bhi)
        x = np.linspace(blo, bhi, 20001)
        r = np.sqrt(x) - (a * x + b)
        assert r.min() >= dlo - 1e-12 and r.max() <= dhi + 1e-12
        # the bounds are attained: at the interval ends and at the tangent point
        assert abs(r.min() - dlo) < 1e-12
        assert abs(r.max() - dhi) <= max(1e-12, 1e-6 * dhi)
