"""Comparisons of GPU bound hierarchies with the FP64 oracle, shared by the
GPU parity tests."""
import numpy as np

BOUND_TOL = 1e-5


def keyset(L):
    return set(zip(np.asarray(L["tuple"]).tolist(), map(tuple, np.asarray(L["code"]).tolist())))


def check_leaf_bounds(orc, osc, L, idx, tol=BOUND_TOL, e_face_value=False, flags=0, uk_face_value=False,
                      e_tail=None, e_abs=0.0):
    """GPU leaves against the oracle's bound of the very same box: the GPU
    bound contains the oracle's and exceeds it by at most `tol`.  With
    e_face_value the irradiance bound is one taken at face value on both
    sides (no rounding control), so it only agrees to within `tol`.  With
    e_tail = (frac, tol2) at most a fraction `frac` of the leaves may exceed
    `tol` on the irradiance bound, and none `tol2`: a rounding-controlled
    bound exceeds the exact one by its rounding slack, theta times the
    magnitude-to-value ratio of its extremal coefficients, which is large
    only where the polynomial's terms cancel (next to a caustic or to total
    internal reflection).  With e_abs a face-value E_lo may also differ by
    e_abs times E_hi: a lower bound formed as a difference that nearly cancels
    (a fitted coefficient minus its remainder) is accurate to the rounding of
    its terms, not of itself."""
    n_tail, n = 0, 0
    for k in idx:
        n += 1
        ob = orc.box_bound(osc, int(L["tuple"][k]), L["box"][k].astype(np.float64), flags=flags)
        assert ob["live"], k
        gu = L["uk"][k].astype(np.float64)
        ou = ob["uk"]
        if not uk_face_value:  # a rigorous position bound contains the oracle's
            assert gu[0] <= ou[0] + 1e-12 and gu[2] <= ou[2] + 1e-12, (k, gu, ou)
            assert gu[1] >= ou[1] - 1e-12 and gu[3] >= ou[3] - 1e-12, (k, gu, ou)
        assert np.max(np.abs(gu - ou)) <= tol, (k, gu, ou)
        gE = L["E"][k].astype(np.float64)
        oE = ob["E"]
        assert np.isinf(gE[1]) == np.isinf(oE[1]), (k, gE, oE)
        if e_face_value:
            if np.isfinite(oE[1]):
                assert abs(gE[1] - oE[1]) <= tol * oE[1], (k, gE, oE)
            slack = e_abs * oE[1] if np.isfinite(oE[1]) else 0.0
            assert abs(gE[0] - oE[0]) <= tol * oE[0] + slack, (k, gE, oE)
            continue
        if np.isfinite(oE[1]):
            assert gE[1] >= oE[1] * (1 - 1e-12), (k, gE, oE)
        assert gE[0] <= oE[0] * (1 + 1e-12), (k, gE, oE)
        ex = max(gE[1] / oE[1] - 1 if np.isfinite(oE[1]) else 0.0, 1 - gE[0] / oE[0] if oE[0] > 0 else 0.0)
        if ex > tol:
            assert e_tail is not None and ex <= e_tail[1], (k, gE, oE)
            n_tail += 1
    if e_tail is not None:
        assert n_tail <= e_tail[0] * n, (n_tail, n)


def check_cover_list(off, gt, ge, Ob, G, tol=BOUND_TOL):
    """The GPU grid's last slice (the cover-all list) against the oracle's:
    the same tuples in the same order, and the same largest E_hi up to the
    FP32 rounding of the outputs (both are maxima of the leaves' E_hi)."""
    assert len(off) == G * G + 2 and off[-1] == len(gt)
    ot, oe = Ob.cover_list()
    a, b = off[G * G], off[G * G + 1]
    assert np.array_equal(gt[a:b].astype(np.int64), ot)
    e = ge[a:b].astype(np.float64)
    fin = np.isfinite(oe)
    assert np.array_equal(np.isfinite(e), fin)
    assert np.all(np.abs(e[fin] - oe[fin]) <= tol * np.abs(oe[fin]))
