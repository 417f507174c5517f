"""Pins of the oracle's sampling and estimation (Sec. 5):

* Philox4x32-10 reproduces its published known-answer vectors (rng() of Alg. 1);
* the selection probabilities satisfy the KKT conditions of Sec. 5.4 and no
  feasible perturbation lowers the variance bound;
* test (c): brute-force roots of every tuple (no bounds consulted) are found
  in the candidate list of their cell, under a per-tuple bound >= E_k, and by
  the leaf-seeded Newton search;
* test (d): the mean of Alg. 1 over many seeds matches the exhaustive sum
  within 3 standard errors of the exact Bernoulli variance, which is itself
  below the bound of Eq. eq_varbound_u; with P = 1 the estimate is the
  exhaustive sum exactly.
"""
import json
import os

import numpy as np
import pytest

from paper_2504_19163_amd import scenes as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers(orc):
    kat = json.load(open(os.path.join(GOLDEN, "philox4x32_10_kat.json")))
    for v in kat["vectors"]:
        ctr = [int(x, 16) for x in v["ctr"]]
        key = [int(x, 16) for x in v["key"]]
        out = orc.philox4x32_10(ctr, key)
        assert [f"{x:08x}" for x in out] == v["out"]


def test_uniform_stream_is_uniform(orc):
    r = np.array([orc.uniform(7, i, t) for i in range(200) for t in range(50)])
    assert r.min() >= 0 and r.max() < 1
    h, _ = np.histogram(r, bins=10, range=(0, 1))
    assert np.all(np.abs(h - 1000) < 5 * np.sqrt(1000))


def _kkt_check(Et, W, P):
    Et = np.asarray(Et, float)
    fin = np.isfinite(Et) & (Et > 0)
    n_inf = np.isinf(Et).sum()
    assert np.all(P[np.isinf(Et)] == 1.0)
    assert np.all(P[Et == 0] == 0.0)
    if fin.sum() == 0:
        return
    Wf = min(max(min(W, len(Et)) - n_inf, 1), fin.sum())
    assert abs(P[fin].sum() - Wf) < 1e-9 * max(1, Wf)
    assert np.all(P[fin] > 0) and np.all(P[fin] <= 1 + 1e-15)
    unsat = fin & (P < 1)
    if unsat.any():
        gam = P[unsat] / Et[unsat]
        assert np.allclose(gam, gam[0], rtol=1e-12)
        assert np.all(gam[0] * Et[fin & (P >= 1)] >= 1 - 1e-12)


def test_probabilities_kkt_and_optimality(orc):
    rng = np.random.default_rng(21)
    for trial in range(200):
        n = int(rng.integers(1, 40))
        Et = rng.lognormal(0, 2, n)
        if trial % 5 == 0:
            Et[rng.integers(0, n)] = np.inf
        if trial % 7 == 0:
            Et[rng.integers(0, n)] = 0.0
        W = float(rng.integers(1, 30))
        P = orc.probabilities(Et, W)
        _kkt_check(Et, W, P)
        # no feasible perturbation (sum kept, inside (0,1]) lowers sum E~^2/P
        fin = np.isfinite(Et) & (Et > 0)
        idx = np.nonzero(fin)[0]
        if len(idx) >= 2:
            obj = np.sum(Et[idx] ** 2 / P[idx])
            for _ in range(20):
                i, j = rng.choice(idx, 2, replace=False)
                eps = 1e-4 * min(P[i], P[j])
                Q = P.copy()
                Q[i] += eps
                Q[j] -= eps
                if Q[i] <= 1 and Q[j] > 0:
                    assert np.sum(Et[idx] ** 2 / Q[idx]) >= obj * (1 - 1e-12)


def _small_scene():
    return S.heightfield_mirror(8)


@pytest.fixture(scope="module")
def small(orc):
    sc = _small_scene()
    osc = orc.OracleScene(sc)
    b = orc.OracleBuild(osc, dict(max_depth=4))
    pts = S.random_points(sc, 48, seed=3)
    return sc, osc, b, pts


def test_c_brute_force_roots_are_enumerated(orc, small):
    sc, osc, b, pts = small
    G = b.params["grid_res"]
    n_roots = 0
    n_leaked = 0
    for i in range(pts.shape[1]):
        x = pts[:, i].astype(float)
        u = (x[0] - sc["q0"][0]) / sc["f1"][0]
        v = (x[1] - sc["q0"][1]) / sc["f2"][1]
        U, Et = b.candidates(min(G - 1, int(u * G)), min(G - 1, int(v * G)))
        inU = dict(zip(U.tolist(), Et.tolist()))
        for t in range(osc.n_tuples):
            roots = orc.tuple_roots(osc, t, x, lattice=24)
            if len(roots) == 0:
                continue
            n_roots += len(roots)
            # every admissible path lies in a tuple of U, under its per-tuple bound
            assert t in inU, (i, t)
            assert inU[t] >= roots[:, 2].max() * (1 - 1e-9)
            # the leaf-seeded Newton search finds the same roots
            lr = b.tuple_roots_leaves(t, x)
            for r in roots:
                hit = len(lr) and np.min(np.max(np.abs(lr[:, :2] - r[:2]), axis=1)) < 1e-7
                n_leaked += 0 if hit else 1
    assert n_roots > 40
    assert n_leaked <= 0.02 * n_roots


def test_c_exhaustive_equals_true_irradiance(orc, small):
    sc, osc, b, pts = small
    E_true = orc.true_irradiance(osc, pts, lattice=24)
    E_brute, _ = b.query(pts, 1, 0, mode=3)  # every tuple of U, brute-force roots
    np.testing.assert_allclose(E_brute, E_true, rtol=1e-9, atol=1e-12)
    E_leaf, _ = b.query(pts, 1, 0, mode=1)  # every tuple of U, leaf-seeded roots
    close = np.isclose(E_leaf, E_true, rtol=1e-7, atol=1e-12)
    assert close.mean() >= 0.95


def test_d_estimator_unbiased_within_3se(orc, small):
    sc, osc, b, pts = small
    W = 2.0
    G = b.params["grid_res"]
    E_exh, _ = b.query(pts, W, 0, mode=1)
    K = 400
    acc = np.zeros(pts.shape[1])
    for seed in range(K):
        E, st = b.query(pts, W, seed, mode=0, n_threads=1)
        acc += E
    mean = acc / K
    # exact variance of Alg. 1: sum_T E(T)^2 (1 - P_T) / P_T
    var = np.zeros(pts.shape[1])
    for i in range(pts.shape[1]):
        x = pts[:, i].astype(float)
        u = (x[0] - sc["q0"][0]) / sc["f1"][0]
        v = (x[1] - sc["q0"][1]) / sc["f2"][1]
        U, Et = b.candidates(min(G - 1, int(u * G)), min(G - 1, int(v * G)))
        if len(U) == 0:
            continue
        P = orc.probabilities(Et, W)
        ET = np.array([b.tuple_roots_leaves(t, x)[:, 2].sum() for t in U])
        var[i] = np.sum(ET ** 2 * (1 - P) / P)
        # the variance is below the bound sum E~^2 / P (Eq. eq_varbound_u)
        fin = np.isfinite(Et)
        assert var[i] <= np.sum(Et[fin] ** 2 / P[fin]) + (np.inf if (~fin).any() else 0)
    sampled = var > 0
    assert sampled.sum() >= 10
    z = (mean[sampled] - E_exh[sampled]) / np.sqrt(var[sampled] / K)
    assert abs(z.sum() / np.sqrt(sampled.sum())) < 3.0
    assert np.all(np.abs(z) < 5.0)
    # points with every P = 1 have zero variance and equal the exhaustive sum
    np.testing.assert_allclose(mean[~sampled], E_exh[~sampled], rtol=1e-12, atol=0)


def test_d_full_probability_is_exhaustive(orc, small):
    sc, osc, b, pts = small
    E1, _ = b.query(pts, 1e9, 5, mode=0)
    E2, _ = b.query(pts, 1e9, 5, mode=1)
    assert np.array_equal(E1, E2)
