"""Pins of the oracle's alternative samplers (Sec. 5.2-5.3 and the figure
comparing sampling schemes): uniform P, the one-sample estimator with
P1 = E~ / sum E~ repeated W times, and the bin-packed multi-sample estimator
(bound-optimal P, one importance sample per bin of total P <= 1).

What fixes them independently of the code: selection frequencies equal the
stated probabilities (uniform: W'/|U|; one-sample draws: E~ / sum E~; bins:
the bound-optimal P_T of every candidate); worked cases whose bins follow
from the definition by hand (a list with sum P = 1 fits one bin, so exactly
one candidate is selected per draw); and unbiasedness of each estimator on a
scene, within 3 standard errors of its exact variance (uniform, one-sample)
or of the variance bound sum E^2 / P (bins)."""
import numpy as np
import pytest

from paper_2504_19163_amd import scenes as S


def _freq(orc, Et, W, sampler, trials, seed=3):
    n = len(Et)
    hits = np.zeros(n)
    weights = {}
    for pt in range(trials):
        k, P = orc.sample(Et, W, seed, pt, sampler)
        hits[k] += 1
        for kk, pp in zip(k, P):
            weights.setdefault(int(kk), set()).add(float(pp))
    return hits / trials, weights


def test_uniform_selects_every_candidate_with_w_over_u(orc):
    Et = np.array([0.0, 1.0, 5.0, np.inf, 2.0, 0.5, 9.0, 3.0] * 3)
    W = 6.0
    T = 4000
    f, w = _freq(orc, Et, W, orc.SAMPLER_UNIFORM, T)
    p = W / len(Et)
    assert np.all(np.abs(f - p) < 4.5 * np.sqrt(p * (1 - p) / T))
    assert all(ws == {p} for ws in w.values())  # the weight is exactly W'/|U| (FP64)


def test_bins_keep_the_bound_optimal_marginals(orc):
    rng = np.random.default_rng(5)
    for trial in range(6):
        n = int(rng.integers(5, 30))
        Et = rng.lognormal(0, 1.5, n)
        Et[rng.integers(0, n)] = 0.0
        if trial % 2:
            Et[rng.integers(0, n)] = np.inf
        W = float(rng.integers(1, n))
        P = orc.probabilities(Et, W)
        T = 3000
        f, w = _freq(orc, Et, W, orc.SAMPLER_BINS, T, seed=trial)
        sd = np.sqrt(np.maximum(P * (1 - P), 1e-12) / T)
        assert np.all(np.abs(f - P) < 4.5 * sd + 1e-12), trial
        assert f[P == 0].sum() == 0
        for k, ws in w.items():  # weight of a selected candidate is its own P (a bin's end cut at 1)
            assert all(abs(x - P[k]) <= 2.0 ** -40 for x in ws)


def test_bins_one_bin_gives_exactly_one_sample(orc):
    # E~ = (3, 3, 4) with W = 1: gamma = 1/10, P = (0.3, 0.3, 0.4), sum 1, so
    # the three share one bin and every draw selects exactly one of them
    Et = np.array([3.0, 3.0, 4.0])
    P = orc.probabilities(Et, 1.0)
    np.testing.assert_allclose(P, [0.3, 0.3, 0.4], rtol=1e-12)
    T = 4000
    counts = np.zeros(3)
    for pt in range(T):
        k, _ = orc.sample(Et, 1.0, 11, pt, orc.SAMPLER_BINS)
        assert len(k) == 1
        counts[k] += 1
    assert np.all(np.abs(counts / T - P) < 4.5 * np.sqrt(P * (1 - P) / T))
    # with W = 2, P = (0.6, 0.6, 0.8): no two fit together, three bins, and
    # the selections are independent: all three with probability 0.288
    P2 = orc.probabilities(Et, 2.0)
    np.testing.assert_allclose(P2, [0.6, 0.6, 0.8], rtol=1e-12)
    three = sum(len(orc.sample(Et, 2.0, 12, pt, orc.SAMPLER_BINS)[0]) == 3 for pt in range(T)) / T
    assert abs(three - 0.288) < 4.5 * np.sqrt(0.288 * 0.712 / T)


def test_one_sample_draws_proportional_to_the_bound(orc):
    Et = np.array([1.0, 3.0, 0.0, np.inf, 4.0])
    W = 8
    T = 2000
    draws = np.zeros(len(Et))
    for pt in range(T):
        k, P = orc.sample(Et, W, 9, pt, orc.SAMPLER_ONE)
        assert 3 in k and P[list(k).index(3)] == 1.0  # the unbounded candidate, once with P = 1
        fin = k != 3
        # a candidate drawn c times has weight W P1 / c, so the counts add to W
        p1 = Et[k[fin]] / 8.0
        c = np.rint(W * p1 / P[fin]).astype(int)
        np.testing.assert_allclose(W * p1 / c, P[fin], rtol=1e-14)
        assert c.sum() == W
        draws[k[fin]] += c
    p = np.array([1, 3, 0, 0, 4]) / 8.0
    f = draws / (W * T)
    assert np.all(np.abs(f - p) < 4.5 * np.sqrt(p * (1 - p) / (W * T)) + 1e-12)
    # a single bounded candidate is drawn every time: weight exactly 1
    k, P = orc.sample([5.0], 4, 1, 0, orc.SAMPLER_ONE)
    assert list(k) == [0] and P[0] == 1.0


@pytest.fixture(scope="module")
def small(orc):
    sc = S.heightfield_mirror(8)
    osc = orc.OracleScene(sc)
    b = orc.OracleBuild(osc, dict(max_depth=4))
    pts = S.random_points(sc, 40, seed=4)
    return sc, osc, b, pts


def _per_point_lists(orc, sc, b, pts):
    G = b.params["grid_res"]
    out = []
    for i in range(pts.shape[1]):
        x = pts[:, i].astype(float)
        u = (x[0] - sc["q0"][0]) / sc["f1"][0]
        v = (x[1] - sc["q0"][1]) / sc["f2"][1]
        U, Et = b.candidates(min(G - 1, int(u * G)), min(G - 1, int(v * G)))
        ET = np.array([b.tuple_roots_leaves(t, x)[:, 2].sum() for t in U]) if len(U) else np.zeros(0)
        out.append((U, Et, ET))
    return out


@pytest.mark.parametrize("mode", [4, 8, 12])
def test_samplers_are_unbiased_within_3se(orc, small, mode):
    sc, osc, b, pts = small
    W = 3.0
    E_exh, _ = b.query(pts, W, 0, mode=1)
    K = 300
    acc = np.zeros(pts.shape[1])
    for seed in range(K):
        E, _ = b.query(pts, W, seed, mode=mode, n_threads=1)
        acc += E
    mean = acc / K
    var = np.zeros(pts.shape[1])
    for i, (U, Et, ET) in enumerate(_per_point_lists(orc, sc, b, pts)):
        if len(U) == 0:
            continue
        if mode == 4:  # independent selections with P = W'/|U|
            p = min(W, len(U)) / len(U)
            var[i] = np.sum(ET ** 2 * (1 - p) / p)
        elif mode == 8:  # W independent draws of E(T)/P1(T) among the bounded candidates
            fin = np.isfinite(Et) & (Et > 0)
            if fin.sum() > 1:
                p1 = Et[fin] / Et[fin].sum()
                var[i] = (np.sum(ET[fin] ** 2 / p1) - ET[fin].sum() ** 2) / W
        else:  # bins: at most the moment bound sum E(T)^2 / P
            P = orc.probabilities(Et, W)
            pos = P > 0
            var[i] = np.sum(ET[pos] ** 2 / P[pos]) - np.sum(ET[pos] ** 2)
    sampled = var > 1e-30
    assert sampled.sum() >= 5
    z = (mean[sampled] - E_exh[sampled]) / np.sqrt(var[sampled] / K)
    assert abs(z.sum() / np.sqrt(sampled.sum())) < 3.0
    assert np.all(np.abs(z) < 5.0)
    np.testing.assert_allclose(mean[~sampled], E_exh[~sampled], rtol=1e-6, atol=1e-12)
