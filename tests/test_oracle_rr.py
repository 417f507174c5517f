"""The oracle's two-reflection chain (RR): the rational map of Eq. eq_rct
applied twice against an ordinary ray tracer, its Jacobian against finite
differences, its irradiance against the solid angle of a ray triangle over
the receiver area it lands on, the double-mirror image source, containment of
every leaf's position and irradiance bound (Sec. 4.2, 4.4) and the
irradiance bound's tightness on small boxes, and test (c) over all tuples: every
admissible path lies in a tuple of its cell list (so pair culling and the
bounds lose nothing) and the leaf-seeded search finds almost all of them."""
import numpy as np
import pytest

from paper_2504_19163_amd import scenes as S


def _tri(pos, nrm, t):
    P = pos[:, t].astype(float).reshape(3, 3)
    N = nrm[:, t].astype(float).reshape(3, 3)
    return P, N


def _oriented_normal(P, N):
    g = np.cross(P[1] - P[0], P[2] - P[0])
    g = g / np.linalg.norm(g)
    return -g if g @ N.sum(0) < 0 else g


def _trace(sc, t1, t2, u, v):
    """Ordinary ray tracing with normalised normals: returns (uk, vk, admissible)."""
    P, N = _tri(sc["pos"], sc["nrm"], t1)
    Pb, Nb = _tri(sc["pos2"], sc["nrm2"], t2)
    x0 = sc["epos"][:, 0].astype(float)
    x1 = P[0] + u * (P[1] - P[0]) + v * (P[2] - P[0])
    n1 = N[0] + u * (N[1] - N[0]) + v * (N[2] - N[0])
    n1 /= np.linalg.norm(n1)
    d = x1 - x0
    r1 = d - 2 * (d @ n1) * n1
    g2 = np.cross(Pb[1] - Pb[0], Pb[2] - Pb[0])
    s = ((Pb[0] - x1) @ g2) / (r1 @ g2)
    x2 = x1 + s * r1
    M = np.stack([Pb[1] - Pb[0], Pb[2] - Pb[0]], 1)
    u2, v2 = np.linalg.lstsq(M, x2 - Pb[0], rcond=None)[0]
    n2 = Nb[0] + u2 * (Nb[1] - Nb[0]) + v2 * (Nb[2] - Nb[0])
    n2 /= np.linalg.norm(n2)
    r2 = r1 - 2 * (r1 @ n2) * n2
    q0, f1, f2 = (sc[k].astype(float) for k in ("q0", "f1", "f2"))
    fk = np.cross(f1, f2)
    t = ((q0 - x2) @ fk) / (r2 @ fk)
    xk = x2 + t * r2
    uk, vk = np.linalg.lstsq(np.stack([f1, f2], 1), xk - q0, rcond=None)[0]
    front1 = (x0 - P[0]) @ _oriented_normal(P, N) > 0
    front2 = r1 @ _oriented_normal(Pb, Nb) < 0
    ok = (front1 and front2 and u >= 0 and v >= 0 and u + v <= 1 and s > 0 and u2 >= 0 and v2 >= 0
          and u2 + v2 <= 1 and t > 0)
    return uk, vk, ok


def _solid_angle(a, b, c):
    la, lb, lc = (np.linalg.norm(x) for x in (a, b, c))
    num = abs(a @ np.cross(b, c))
    den = la * lb * lc + (a @ b) * lc + (a @ c) * lb + (b @ c) * la
    return 2 * np.arctan2(num, den)


@pytest.fixture(scope="module")
def walls(orc):
    sc = S.facing_walls(4)
    osc = orc.OracleScene(sc)
    b = orc.OracleBuild(osc, dict(max_depth=4))
    return sc, osc, b


def _admissible_samples(orc, osc, sc, n_want, seed):
    rng = np.random.default_rng(seed)
    n2 = sc["pos2"].shape[1]
    out = []
    tries = 0
    while len(out) < n_want and tries < 200000:
        tries += 1
        t = int(rng.integers(0, osc.n_tuples))
        u, v = rng.uniform(0, 1, 2)
        if u + v > 1:
            continue
        e = orc.eval_path(osc, t, u, v)
        if e["admissible"]:
            out.append((t, t // n2, t % n2, u, v, e))
    return out


def test_rr_double_mirror_image_source(orc):
    sc = S.double_mirror()
    osc = orc.OracleScene(sc)
    b = orc.OracleBuild(osc, dict(max_depth=3))
    pts = S.receiver_points(sc, 16)
    E, st = b.query(pts, 4, 0, mode=1)
    lx, ly, lz = sc["epos"][:, 0].astype(float)
    img = np.array([lx, ly, 2 * 2.0 + lz])  # the light mirrored in z = 0, then in z = 2
    d = pts.astype(float) - img[:, None]
    ref = np.abs(d[2]) / np.linalg.norm(d, axis=0) ** 3
    np.testing.assert_allclose(E, ref, rtol=1e-8)
    assert np.all(st[:, 2] == 1)


def test_rr_map_matches_ray_tracing(orc, walls):
    sc, osc, b = walls
    samples = _admissible_samples(orc, osc, sc, 60, seed=1)
    assert len(samples) >= 60
    for t, t1, t2, u, v, e in samples:
        uk, vk, ok = _trace(sc, t1, t2, u, v)
        assert ok, (t, u, v)
        assert abs(uk - e["uk"]) <= 1e-9 and abs(vk - e["vk"]) <= 1e-9, (t, u, v, uk, vk, e)
    # and a path the tracer rejects is not admissible either
    rng = np.random.default_rng(2)
    n2 = sc["pos2"].shape[1]
    for _ in range(300):
        t = int(rng.integers(0, osc.n_tuples))
        u, v = rng.uniform(0, 0.5, 2)
        e = orc.eval_path(osc, t, u, v)
        _, _, ok = _trace(sc, t // n2, t % n2, u, v)
        assert bool(e["admissible"]) == bool(ok), (t, u, v)


def test_rr_jacobian_and_irradiance_first_principles(orc, walls):
    sc, osc, b = walls
    x0 = sc["epos"][:, 0].astype(float)
    q0, f1, f2 = (sc[k].astype(float) for k in ("q0", "f1", "f2"))
    for t, t1, t2, u, v, e in _admissible_samples(orc, osc, sc, 25, seed=3):
        h = 1e-6
        ep, em = orc.eval_path(osc, t, u + h, v), orc.eval_path(osc, t, u - h, v)
        fp, fm = orc.eval_path(osc, t, u, v + h), orc.eval_path(osc, t, u, v - h)
        J = np.array([[ep["uk"] - em["uk"], fp["uk"] - fm["uk"]], [ep["vk"] - em["vk"], fp["vk"] - fm["vk"]]]) / (2 * h)
        assert abs(np.linalg.det(J) - e["detJ"]) <= 1e-4 * max(1.0, abs(e["detJ"])), (t, u, v)
        # irradiance = solid angle at the light of a small ray triangle / its area on the receiver
        h = 2e-6
        ev = [orc.eval_path(osc, t, a, c) for a, c in ((u, v), (u + h, v), (u, v + h))]
        xk = [q0 + p["uk"] * f1 + p["vk"] * f2 for p in ev]
        area = 0.5 * np.linalg.norm(np.cross(xk[1] - xk[0], xk[2] - xk[0]))
        om = _solid_angle(*(p["x1"] - x0 for p in ev))
        assert abs(om / area - e["Ek"]) <= 2e-3 * e["Ek"], (t, u, v, om / area, e["Ek"])


def test_rr_bounds_contain_paths(orc, walls):
    """Every leaf's position bound and irradiance bound contain u_k and E_k
    (E_k pinned from first principles above) of the admissible paths through
    a grid of its box."""
    sc, osc, b = walls
    L = b.leaves()
    fin = np.isfinite(L["E"][:, 1])
    assert fin.mean() > 0.8  # the chain's irradiance bound is finite on most leaves
    n_paths = 0
    rng = np.random.default_rng(4)
    for k in rng.choice(len(L["tuple"]), 200, replace=False):
        t = L["tuple"][k]
        u0, u1, v0, v1 = L["box"][k]
        ulo, uhi, vlo, vhi = L["uk"][k]
        Elo, Ehi = L["E"][k]
        for u in np.linspace(u0, u1, 9):
            for v in np.linspace(v0, v1, 9):
                e = orc.eval_path(osc, t, u, v)
                if not e["admissible"] or not (0 <= e["uk"] <= 1 and 0 <= e["vk"] <= 1):
                    continue
                n_paths += 1
                assert ulo - 1e-9 <= e["uk"] <= uhi + 1e-9 and vlo - 1e-9 <= e["vk"] <= vhi + 1e-9, (t, u, v)
                assert Elo * (1 - 1e-9) <= e["Ek"] <= Ehi * (1 + 1e-9), (t, u, v, e["Ek"], Elo, Ehi)
    assert n_paths > 500


def test_rr_irradiance_bound_is_tight_on_small_boxes(orc, walls):
    """On small boxes around admissible paths the bound is no wider than 1.5
    times the range of E_k sampled over the box (a dropped or wrong term in
    det M or Den^3 would leave it far looser or cut into the range)."""
    sc, osc, b = walls
    L = b.leaves()
    n_checked = 0
    for k in np.nonzero(np.isfinite(L["E"][:, 1]))[0][:80]:
        t = L["tuple"][k]
        u0, u1, v0, v1 = L["box"][k]
        uc, vc = 0.5 * (u0 + u1), 0.5 * (v0 + v1)
        if not orc.eval_path(osc, t, uc, vc)["admissible"]:
            continue
        h = (u1 - u0) / 32
        bb = orc.box_bound(osc, t, [uc - h, uc + h, vc - h, vc + h])
        if not (bb["live"] and np.isfinite(bb["E"][1])):
            continue
        E = [orc.eval_path(osc, t, u, v) for u in np.linspace(uc - h, uc + h, 7) for v in np.linspace(vc - h, vc + h, 7)]
        if not all(e["admissible"] for e in E):
            continue
        E = np.array([e["Ek"] for e in E])
        assert bb["E"][0] <= E.min() * (1 + 1e-9) and bb["E"][1] >= E.max() * (1 - 1e-9)
        assert bb["E"][1] - bb["E"][0] <= 1.5 * (E.max() - E.min()) + 1e-9 * E.max(), (k, bb["E"], E.min(), E.max())
        n_checked += 1
    assert n_checked >= 10


def test_rr_c_every_path_is_in_its_cell_list(orc, walls):
    sc, osc, b = walls
    G = b.params["grid_res"]
    pts = S.random_points(sc, 10, seed=5)
    n_roots = n_leaked = 0
    for i in range(pts.shape[1]):
        x = pts[:, i].astype(float)
        u = (x[0] - sc["q0"][0]) / sc["f1"][0]
        v = (x[1] - sc["q0"][1]) / sc["f2"][1]
        U, _ = b.candidates(min(G - 1, int(u * G)), min(G - 1, int(v * G)))
        inU = set(U.tolist())
        for t in range(osc.n_tuples):
            roots = orc.tuple_roots(osc, t, x, lattice=12)
            if len(roots) == 0:
                continue
            n_roots += len(roots)
            assert t in inU, (i, t)
            lr = b.tuple_roots_leaves(t, x)
            for r in roots:
                hit = len(lr) and np.min(np.max(np.abs(lr[:, :2] - r[:2]), axis=1)) < 1e-7
                n_leaked += 0 if hit else 1
    assert n_roots > 10
    assert n_leaked <= 0.05 * n_roots


def test_rr_exhaustive_close_to_true_irradiance(orc, walls):
    sc, osc, b = walls
    pts = S.random_points(sc, 120, seed=6)
    E_true = orc.true_irradiance(osc, pts, lattice=16)
    E_leaf, _ = b.query(pts, 1, 0, mode=1)
    assert np.all(E_leaf <= E_true * (1 + 1e-7) + 1e-12)  # never a root that is not there
    close = np.isclose(E_leaf, E_true, rtol=1e-7, atol=1e-12)
    assert close.mean() >= 0.95
    assert (E_true > 0).sum() >= 60
