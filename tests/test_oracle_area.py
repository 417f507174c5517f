"""Area lights in the oracle (the emitter variable of the area-light remark
in the implementation section and the area-light figure): the light is a
parallelogram x0 + z1 a + z2 b, every point of which emits with the light's
intensity, and the irradiance is the mean over (z1, z2) in [0,1]^2.  Bounds
hold over the box times the whole light (axes u, v, z1, z2); the estimator
draws one light point per selected pair.

Pins: (a) a light of zero extent reproduces the point light's leaves, bounds
and estimates; (b) every leaf's bound contains u_k and E_k of every admissible
path through its box from every sampled light point; (c) over a flat mirror
the estimator's mean matches the image-source irradiance averaged over the
light by quadrature (numpy), within 4 standard errors."""
import numpy as np
import pytest

from paper_2504_19163_amd import scenes as S


def test_point_sized_area_light_equals_point_light(orc):
    sc = S.heightfield_mirror(8)
    scz = S.area_light(sc, [0.0, 0.0, 0.0], [0.0, 0.0, 0.0])
    osc, oscz = orc.OracleScene(sc), orc.OracleScene(scz)
    p = dict(max_depth=3)
    b, bz = orc.OracleBuild(osc, p), orc.OracleBuild(oscz, p)
    L, Lz = b.leaves(), bz.leaves()
    key = lambda L: np.lexsort((L["code"][:, 2], L["code"][:, 1], L["code"][:, 0], L["tuple"]))
    i, iz = key(L), key(Lz)
    assert np.array_equal(L["tuple"][i], Lz["tuple"][iz]) and np.array_equal(L["code"][i], Lz["code"][iz])
    np.testing.assert_allclose(Lz["uk"][iz], L["uk"][i], rtol=1e-12, atol=1e-14)
    fin = np.isfinite(L["E"][i])
    assert np.array_equal(fin, np.isfinite(Lz["E"][iz]))
    np.testing.assert_allclose(Lz["E"][iz][fin], L["E"][i][fin], rtol=1e-9)
    pts = S.random_points(sc, 300, seed=3)
    E, _ = b.query(pts, 8, 5, mode=0)
    Ez, _ = bz.query(pts, 8, 5, mode=0)
    np.testing.assert_allclose(Ez, E, rtol=1e-9, atol=1e-15)


def test_area_bounds_contain_paths_from_every_light_point(orc):
    sc = S.area_light(S.heightfield_mirror(8), [0.6, 0.0, 0.0], [0.0, 0.4, 0.0])
    osc = orc.OracleScene(sc)
    b = orc.OracleBuild(osc, dict(max_depth=3))
    L = b.leaves()
    rng = np.random.default_rng(2)
    zs = [(0, 0), (1, 0), (0, 1), (1, 1), (0.5, 0.5)] + [tuple(z) for z in rng.uniform(0, 1, (3, 2))]
    n_paths = 0
    for k in range(0, len(L["tuple"]), 3):
        t = L["tuple"][k]
        u0, u1, v0, v1 = L["box"][k]
        ulo, uhi, vlo, vhi = L["uk"][k]
        Elo, Ehi = L["E"][k]
        for u in np.linspace(u0, u1, 5):
            for v in np.linspace(v0, v1, 5):
                for z in zs:
                    e = orc.eval_path(osc, t, u, v, z)
                    if not e["admissible"] or not (0 <= e["uk"] <= 1 and 0 <= e["vk"] <= 1):
                        continue
                    n_paths += 1
                    assert ulo - 1e-9 <= e["uk"] <= uhi + 1e-9 and vlo - 1e-9 <= e["vk"] <= vhi + 1e-9, (t, u, v, z)
                    assert Elo * (1 - 1e-9) <= e["Ek"] <= Ehi * (1 + 1e-9), (t, u, v, z, e["Ek"], Elo, Ehi)
    assert n_paths > 3000


def test_flat_mirror_area_light_closed_form(orc):
    a, bvec = np.array([0.5, 0.0, 0.0]), np.array([0.0, 0.3, 0.0])
    base = S.flat_mirror()
    sc = S.area_light(base, a, bvec)
    osc = orc.OracleScene(sc)
    b = orc.OracleBuild(osc, dict(max_depth=4))
    # shading points over the part of the receiver the mirror lights
    rng = np.random.default_rng(9)
    uv = rng.uniform(0.32, 0.56, (2, 40))
    pts = (sc["q0"][:, None] + uv[0] * sc["f1"][:, None] + uv[1] * sc["f2"][:, None]).astype(np.float32)
    corner = sc["epos"][:, 0].astype(np.float64)
    tri = base["pos"][:, 0].astype(np.float64).reshape(3, 3)

    def inside(p):  # reflection point inside the mirror triangle (z = 0)
        l1 = (p[0] - tri[0, 0]) / (tri[1, 0] - tri[0, 0])
        l2 = (p[1] - tri[0, 1]) / (tri[2, 1] - tri[0, 1])
        return l1 >= 0 and l2 >= 0 and l1 + l2 <= 1

    # image-source irradiance averaged over the light (midpoint rule, 60 x 60)
    g = (np.arange(60) + 0.5) / 60
    exact = np.zeros(pts.shape[1])
    cover = np.zeros(pts.shape[1])  # fraction of the light that reaches the point via the mirror
    for i in range(pts.shape[1]):
        x = pts[:, i].astype(np.float64)
        acc, hit = 0.0, 0
        for z1 in g:
            for z2 in g:
                x0 = corner + z1 * a + z2 * bvec
                img = x0 * np.array([1.0, 1.0, -1.0])
                d = x - img
                p = img + d * (-img[2] / d[2])  # where the image ray crosses z = 0
                if inside(p):
                    acc += abs(d[2]) / np.linalg.norm(d) ** 3
                    hit += 1
        exact[i] = acc / g.size ** 2
        cover[i] = hit / g.size ** 2
    K = 300
    runs = np.stack([b.query(pts, 1, s, mode=1)[0] for s in range(K)])
    mean, se = runs.mean(0), runs.std(0, ddof=1) / np.sqrt(K)
    # fully lit points: every draw finds the path, only its value varies
    full = cover == 1.0
    assert full.sum() > 25
    err = np.abs(mean[full] - exact[full])
    assert np.all(err <= 4 * se[full] + 5e-3 * exact[full]), (err / exact[full]).max()
    # penumbra points included: the sum over all points
    tot_se = np.sqrt(np.sum(se ** 2))
    assert abs(mean.sum() - exact.sum()) <= 4 * tot_se + 5e-3 * exact.sum()
