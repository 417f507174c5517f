"""Pins of the oracle's degree reduction (Sec. 6.1, "Degree reduction": a
least-squares approximant of lower degree fitted through the singular-value
decomposition, plus a remainder variable that keeps the bound valid) and of
its use in the two-reflection irradiance bound (oracle flag 8).

The reduced coefficients X minimise |A - E X| over the coefficients at A's
degree (E the degree-elevation matrix, E_ij = C(n-m, i-j) C(m, j) / C(n, i)),
and the remainder r = max |A - E X| bounds |A(x) - X(x)| on the whole box
(partition of unity).  The checks below rebuild E from that closed form and
solve the least-squares problem with numpy's own routine, evaluate the
polynomials with the power-form Bernstein basis, and never call the oracle's
elevation or evaluation."""
import math

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2504_19163_amd import scenes as S

REDUCE_FLAG = 8


def elevation_matrix(m, n):
    E = np.zeros((n + 1, m + 1))
    for i in range(n + 1):
        for j in range(m + 1):
            if 0 <= i - j <= n - m:
                E[i, j] = math.comb(n - m, i - j) * math.comb(m, j) / math.comb(n, i)
    return E


def basis(n, x):
    return np.array([math.comb(n, i) * x**i * (1 - x) ** (n - i) for i in range(n + 1)])


def eval2(c, x, y):
    n1, n2 = c.shape[0] - 1, c.shape[1] - 1
    return basis(n1, x) @ c @ basis(n2, y)


def test_elevation_matrix_small_case():
    # degree 1 -> 2: the line's coefficients (a, b) become (a, (a + b) / 2, b)
    np.testing.assert_array_equal(elevation_matrix(1, 2), [[1, 0], [0.5, 0.5], [0, 1]])
    # reducing the elevated line returns it with no remainder
    d, X, r = orc.bern_reduce([2], [3.0, 2.0, 1.0], [1])
    np.testing.assert_allclose(X, [3.0, 1.0], atol=1e-14)
    assert r <= 1e-14


@pytest.mark.parametrize("m,n", [(3, 9), (12, 46), (16, 46)])
def test_reduction_recovers_an_elevated_polynomial(m, n):
    rng = np.random.default_rng(m * 100 + n)
    X0 = rng.normal(size=(m + 1, m + 1))
    A = elevation_matrix(m, n) @ X0 @ elevation_matrix(m, n).T
    d, X, r = orc.bern_reduce([n, n], A.ravel(), [m, m])
    assert list(d[:2]) == [m, m]
    np.testing.assert_allclose(X.reshape(m + 1, m + 1), X0, atol=1e-9 * np.abs(X0).max())
    assert r <= 1e-10 * np.abs(A).max()


def test_reduction_is_the_least_squares_fit():
    rng = np.random.default_rng(7)
    # one axis
    a = rng.normal(size=21)
    E = elevation_matrix(6, 20)
    d, X, r = orc.bern_reduce([20], a, [6])
    ref = np.linalg.lstsq(E, a, rcond=None)[0]
    np.testing.assert_allclose(X, ref, atol=1e-10)
    assert r == pytest.approx(np.abs(a - E @ ref).max(), rel=1e-9)
    # two axes: the fit over the Kronecker product of the per-axis elevations
    A = rng.normal(size=(11, 10))
    E1, E2 = elevation_matrix(4, 10), elevation_matrix(3, 9)
    d, X, r = orc.bern_reduce([10, 9], A.ravel(), [4, 3])
    ref = np.linalg.lstsq(np.kron(E1, E2), A.ravel(), rcond=None)[0]
    np.testing.assert_allclose(X, ref, atol=1e-10)
    assert r == pytest.approx(np.abs(A.ravel() - np.kron(E1, E2) @ ref).max(), rel=1e-9)


def test_remainder_bounds_the_difference_everywhere():
    rng = np.random.default_rng(11)
    # a smooth polynomial of degree (30, 30): products of low-degree factors
    # with a little high-degree noise
    n, m = 30, 8
    A = elevation_matrix(4, n) @ rng.normal(size=(5, 5)) @ elevation_matrix(4, n).T
    A += 1e-3 * rng.normal(size=(n + 1, n + 1))
    d, X, r = orc.bern_reduce([n, n], A.ravel(), [m, m])
    X = X.reshape(m + 1, m + 1)
    worst = 0.0
    for x, y in rng.random((400, 2)):
        worst = max(worst, abs(eval2(A, x, y) - eval2(X, x, y)))
    assert worst <= r * (1 + 1e-9)
    assert r > 0 and worst > 0.05 * r  # the remainder is not vacuous


def test_reduction_rejects_a_higher_target():
    d = np.array([3, 0, 0, 0], np.int32)
    out = np.zeros(5)
    rem = np.zeros(1)
    a = np.zeros(4)
    assert orc.lib().orc_bern_reduce(d.ctypes.data, a.ctypes.data, np.array([4, 0, 0, 0], np.int32).ctypes.data,
                                     out.ctypes.data, rem.ctypes.data) == -1


@pytest.fixture(scope="module")
def walls():
    sc = S.facing_walls(4)
    osc = orc.OracleScene(sc)
    Ob = orc.OracleBuild(osc, dict(max_depth=5, alpha=10.0))
    return osc, Ob.leaves()


def test_reduced_rr_bound_contains_the_full_degree_bound(walls):
    """det M (46, 46) and Q^3 (45, 45) exceed the threshold: with the flag both
    are reduced to degree 16 plus a remainder each, and the bound of Q^3/det M
    contains the full-degree one on every leaf.  Its excess is the remainder's
    cost: below 1e-6 on nine leaves in ten (the fit is exact to rounding on
    small boxes), at most a few per cent on the largest leaves."""
    osc, L = walls
    excess = []
    for k in np.random.default_rng(5).choice(len(L["tuple"]), 400, replace=False):
        t, b = int(L["tuple"][k]), L["box"][k].astype(np.float64)
        E0 = orc.box_bound(osc, t, b)["E"]
        E1 = orc.box_bound(osc, t, b, flags=REDUCE_FLAG)["E"]
        assert E1[0] <= E0[0] * (1 + 1e-12)
        assert E1[1] >= E0[1] * (1 - 1e-12)
        if np.isfinite(E0[1]) and E0[0] > 0:
            assert np.isfinite(E1[1])
            excess.append(max(E1[1] / E0[1] - 1, 1 - E1[0] / E0[0]))
    excess = np.array(excess)
    assert len(excess) > 250
    assert np.percentile(excess, 90) <= 1e-6
    assert 1e-9 < excess.max() <= 0.1  # the reduction is in effect


def test_reduced_bound_tightens_under_subdivision(walls):
    """The remainder of a fixed-degree fit shrinks with the box: along a chain
    of nested boxes the reduced bound's excess over the full-degree bound
    falls to the rounding level."""
    osc, L = walls
    n_chains = 0
    for k in range(0, len(L["tuple"]), 7):
        t, leaf = int(L["tuple"][k]), L["box"][k].astype(np.float64)
        cu, cv = (leaf[0] + leaf[1]) / 2, (leaf[2] + leaf[3]) / 2
        excess = []
        for w in (0.25, 0.125, 0.0625, 0.03125, 0.015625):
            b = np.array([cu - w / 2, cu + w / 2, cv - w / 2, cv + w / 2])
            E0 = orc.box_bound(osc, t, b)
            if not (E0["live"] and np.isfinite(E0["E"][1]) and E0["E"][0] > 0):
                break
            E1 = orc.box_bound(osc, t, b, flags=REDUCE_FLAG)["E"]
            excess.append(max(E1[1] / E0["E"][1] - 1, 1 - E1[0] / E0["E"][0]))
        if len(excess) < 5:
            continue
        n_chains += 1
        assert excess[-1] <= 1e-6, excess
        assert all(b <= a * 1.01 + 1e-9 for a, b in zip(excess, excess[1:])), excess
        if n_chains == 8:
            break
    assert n_chains >= 3


def test_reduction_leaves_low_degree_chains_alone():
    """Single-reflection det M (degree (10, 10)) stays below the threshold:
    the flag changes nothing."""
    sc = S.heightfield_mirror(4)
    osc = orc.OracleScene(sc)
    for t in range(4):
        b = np.array([0.0, 0.25, 0.0, 0.25])
        assert orc.box_bound(osc, t, b)["E"].tolist() == orc.box_bound(osc, t, b, flags=REDUCE_FLAG)["E"].tolist()
