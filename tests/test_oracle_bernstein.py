"""Pins of the oracle's Bernstein toolkit (Sec. 4.1) against what the paper and
the mathematics fix: the footnote's worked example, partition of unity, the
invariance of a polynomial under degree elevation and de Casteljau
subdivision, products and derivatives evaluated pointwise, the monomial
basis conversion, and containment / sign rules of the rational range bound."""
import json
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_poly(rng, deg):
    n = int(np.prod(np.asarray(deg) + 1))
    return rng.normal(size=n)


def test_footnote_example(orc):
    g = json.load(open(os.path.join(GOLDEN, "footnote_bernstein.json")))
    d, f = orc.bern_mul([1], g["g_coeffs_deg1"], [1], g["h_coeffs_deg1"])
    assert list(d[:1]) == [2]
    np.testing.assert_allclose(f, g["f_coeffs_deg2"], atol=1e-15)
    kind, lo, hi = orc.ratio_bound([2], f, [0], [1.0])
    assert kind == 0
    assert (lo, hi) == tuple(g["bernstein_bound"])
    # interval arithmetic treats the two factors as independent: [0,1] x [3,4]
    ia = [min(a * b for a in (0, 1) for b in (3, 4)), max(a * b for a in (0, 1) for b in (3, 4))]
    assert ia == g["interval_arithmetic_bound"]
    assert hi - lo < ia[1] - ia[0]


@pytest.mark.parametrize("deg", [(0, 0), (1, 0), (3, 2), (5, 5), (10, 10), (4, 3, 2, 1)])
def test_partition_of_unity(orc, deg):
    rng = np.random.default_rng(1)
    ones = np.ones(int(np.prod(np.asarray(deg) + 1)))
    for _ in range(50):
        x = rng.uniform(0, 1, 4)
        assert abs(orc.bern_eval(deg, ones, x) - 1.0) < 1e-13


def test_eval_matches_monomial_conversion(orc):
    # x^k on [0,1] has Bernstein coefficients b_i = C(i,k)/C(n,k) (zero for i < k)
    rng = np.random.default_rng(2)
    for n in (1, 3, 7, 12):
        for k in range(n + 1):
            b = np.array([math.comb(i, k) / math.comb(n, k) for i in range(n + 1)])
            for x in rng.uniform(0, 1, 10):
                assert abs(orc.bern_eval([n], b, [x]) - x ** k) < 1e-13


@pytest.mark.parametrize("deg,to", [((2, 3), (5, 3)), ((1, 1), (4, 6)), ((3, 3, 1, 1), (4, 5, 2, 1))])
def test_elevation_invariance(orc, deg, to):
    rng = np.random.default_rng(3)
    a = _rand_poly(rng, deg)
    _, b = orc.bern_elevate(deg, a, to)
    for _ in range(200):
        x = rng.uniform(0, 1, 4)
        assert abs(orc.bern_eval(to, b, x) - orc.bern_eval(deg, a, x)) < 1e-13


@pytest.mark.parametrize("deg,axis,t", [((4, 4), 0, 0.5), ((4, 4), 1, 0.5), ((10, 3), 0, 0.3), ((2, 2, 3, 1), 2, 0.7)])
def test_split_invariance(orc, deg, axis, t):
    rng = np.random.default_rng(4)
    a = _rand_poly(rng, deg)
    left, right = orc.bern_split(deg, a, axis, t)
    for _ in range(200):
        x = rng.uniform(0, 1, 4)
        ref = orc.bern_eval(deg, a, x)
        if x[axis] <= t:
            y = x.copy()
            y[axis] = x[axis] / t
            got = orc.bern_eval(deg, left, y)
        else:
            y = x.copy()
            y[axis] = (x[axis] - t) / (1 - t)
            got = orc.bern_eval(deg, right, y)
        assert abs(got - ref) < 1e-12 * max(1.0, abs(ref))


def test_product_pointwise(orc):
    rng = np.random.default_rng(5)
    for da, db in [((1, 1), (1, 1)), ((3, 4), (4, 3)), ((2, 0, 1, 0), (1, 2, 0, 1))]:
        a = _rand_poly(rng, da)
        b = _rand_poly(rng, db)
        dc, c = orc.bern_mul(da, a, db, b)
        for _ in range(100):
            x = rng.uniform(0, 1, 4)
            ref = orc.bern_eval(da, a, x) * orc.bern_eval(db, b, x)
            assert abs(orc.bern_eval(dc, c, x) - ref) < 1e-12 * max(1.0, abs(ref))


def test_derivative_matches_finite_difference(orc):
    rng = np.random.default_rng(6)
    deg = (5, 4)
    a = _rand_poly(rng, deg)
    for axis in (0, 1):
        dd, d = orc.bern_deriv(deg, a, axis)
        for _ in range(50):
            x = rng.uniform(0.05, 0.95, 4)
            h = 1e-5
            xp, xm = x.copy(), x.copy()
            xp[axis] += h
            xm[axis] -= h
            fd = (orc.bern_eval(deg, a, xp) - orc.bern_eval(deg, a, xm)) / (2 * h)
            assert abs(orc.bern_eval(dd, d, x) - fd) < 1e-6 * max(1.0, abs(fd))


def _grid_ratio(orc, dp, p, dq, q, n=41):
    xs = np.linspace(0, 1, n)
    vals = []
    for x in xs:
        for y in xs:
            qq = orc.bern_eval(dq, q, [x, y])
            if qq != 0:
                vals.append(orc.bern_eval(dp, p, [x, y]) / qq)
    return np.array(vals)


def test_ratio_bound_contains_range(orc):
    rng = np.random.default_rng(7)
    for _ in range(10):
        p = rng.normal(size=16)
        q = rng.uniform(0.5, 2.0, 9)  # strictly positive denominator
        kind, lo, hi = orc.ratio_bound([3, 3], p, [2, 2], q)
        assert kind == 0
        v = _grid_ratio(orc, [3, 3], p, [2, 2], q)
        assert v.min() >= lo - 1e-12 and v.max() <= hi + 1e-12


def test_ratio_bound_sign_failure_rules(orc):
    # q changes sign but p does not: the reciprocal rule gives two half-lines
    p = np.array([1.0, 2.0, 1.5, 3.0])
    q = np.array([-1.0, 0.5, 1.0, 2.0])
    kind, lo, hi = orc.ratio_bound([1, 1], p, [1, 1], q)
    assert kind == 1
    v = _grid_ratio(orc, [1, 1], p, [1, 1], q, n=101)
    assert np.all((v <= lo + 1e-12) | (v >= hi - 1e-12))
    # both change sign: no bound
    kind, _, _ = orc.ratio_bound([1, 1], np.array([-1.0, 1, 1, 1]), [1, 1], q)
    assert kind == 2
    # a zero coefficient is not a strict sign
    kind, _, _ = orc.ratio_bound([1, 1], p, [1, 1], np.array([0.0, 1, 1, 1]))
    assert kind == 0 and True  # reciprocal rule applies (p strictly positive): q/p in [0, ...]


def _sub_box(orc, deg, a, lo, hi):
    """Coefficients of the same polynomial on the sub-box [lo0,hi0] x [lo1,hi1]."""
    sub = a
    for axis in (0, 1):
        _, right = orc.bern_split(deg, sub, axis, lo[axis])
        left, _ = orc.bern_split(deg, right, axis, (hi[axis] - lo[axis]) / (1 - lo[axis]))
        sub = left
    return sub


def test_bernstein_bound_converges_quadratically(orc):
    # Sec. 4.1: the Bernstein bound's excess over the true range shrinks with the
    # square of the box width.  Boxes centred on an interior minimum of a
    # polynomial (x-0.3)^2 + (y-0.6)^2, where the true range is O(w^2)
    # too and corner values do not give the range.
    deg = (4, 4)
    mono = {(2, 0): 1.0, (1, 0): -0.6, (0, 2): 1.0, (0, 1): -1.2, (0, 0): 0.45}
    a = np.zeros(25)
    for i in range(5):
        for j in range(5):
            a[i * 5 + j] = sum(c * math.comb(i, p) / math.comb(4, p) * math.comb(j, q) / math.comb(4, q)
                               for (p, q), c in mono.items() if p <= i and q <= j)
    cx, cy = 0.3, 0.6
    widths, excess = [], []
    for k in range(2, 8):
        w = 0.5 ** k
        sub = _sub_box(orc, deg, a, (cx - w / 3, cy - w / 2), (cx + 2 * w / 3, cy + w / 2))
        xs = np.linspace(0, 1, 61)
        vals = [orc.bern_eval(deg, sub, [x, y]) for x in xs for y in xs]
        excess.append((sub.max() - sub.min()) - (max(vals) - min(vals)))
        widths.append(w)
    slope = np.polyfit(np.log(widths), np.log(excess), 1)[0]
    assert 1.7 < slope < 2.3, (slope, excess)
