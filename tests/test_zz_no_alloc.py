"""bbc_query_irradiance_noalloc (the staged query over the library's own
device work space) against bbc_query_irradiance_ex in the staged form: the
same kernels on the same inputs, so estimates and per-point statistics must be
bit-identical.  Two calls in a row, the second with fewer points, so the
second runs over what the first left in the shared work space; the first is
large enough to run in several slices of that space."""
import ctypes as C

import numpy as np
import pytest

from paper_2504_19163_amd import scenes as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bbc():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2504_19163_amd import bbc as B
    B.lib()
    return B


def _both(bbc, B, pts, spp, seed, base, mode):
    E0, st0 = B.query(pts, spp, seed, mode=mode, stats=True, point_index_base=base)
    E1, st1 = B.query_noalloc(pts, spp, seed, mode=mode, stats=True, point_index_base=base)
    torch.cuda.synchronize()
    return E0.cpu().numpy(), st0.cpu().numpy(), E1.cpu().numpy(), st1.cpu().numpy()


@pytest.mark.parametrize("mode_name", ["sampled", "exhaustive", "bins"])
def test_noalloc_query_matches_staged_query(bbc, mode_name):
    mode = bbc.QUERY_STAGED | {"sampled": 0, "exhaustive": bbc.QUERY_EXHAUSTIVE, "bins": bbc.QUERY_BINS}[mode_name]
    sc = S.displaced_sphere(5)  # 8192 triangles
    B = bbc.Bounds(bbc.DeviceScene(sc), dict(max_depth=6))
    big = torch.as_tensor(S.receiver_points(sc, 512), device="cuda")  # 262 144 points
    small = torch.as_tensor(S.receiver_points(sc, 40), device="cuda")
    off, _, _ = B.grid()
    max_cell = int(np.diff(off.astype(np.int64)).max())
    # the worst-case pair space of the large call alone (21 bytes per pair)
    # exceeds the 64 MiB work space, so that call runs in several slices
    assert big.shape[1] * max_cell * 21 > 64 << 20, max_cell
    for pts, spp, seed, base in ((big, 64, 5, 0), (small, 16, 6, 1000)):
        print(mode_name, "points", pts.shape[1], "spp", spp, flush=True)
        E0, st0, E1, st1 = _both(bbc, B, pts, spp, seed, base, mode)
        assert st0[:, 0].sum() > 0 and np.count_nonzero(E0) > 0
        assert np.array_equal(E0.view(np.uint32), E1.view(np.uint32)), (mode_name, pts.shape[1])
        assert np.array_equal(st0.view(np.uint32), st1.view(np.uint32)), (mode_name, pts.shape[1])
    B.free()


def test_noalloc_query_rejects_other_forms(bbc):
    sc = S.heightfield_mirror(8)
    B = bbc.Bounds(bbc.DeviceScene(sc), dict(max_depth=3))
    pts = torch.as_tensor(S.receiver_points(sc, 8), device="cuda")
    out = torch.empty(pts.shape[1], dtype=torch.float32, device="cuda")
    L = bbc.lib()
    for mode in (bbc.QUERY_FUSED, bbc.QUERY_STAGED | bbc.QUERY_EXHAUSTIVE | bbc.QUERY_BINS, 1 << 12):
        st = L.bbc_query_irradiance_noalloc(B.h, pts.data_ptr(), pts.shape[1], 4, 1, 0, mode, out.data_ptr(), None,
                                            None)
        assert st == bbc.EINVAL, mode
    assert L.bbc_query_irradiance_noalloc(B.h, pts.data_ptr(), pts.shape[1], 0, 1, 0, bbc.QUERY_STAGED,
                                          out.data_ptr(), None, None) == bbc.EINVAL
    assert L.bbc_query_irradiance_noalloc(B.h, pts.data_ptr(), 0, 4, 1, 0, bbc.QUERY_STAGED, out.data_ptr(), None,
                                          None) == bbc.OK
    B.free()
