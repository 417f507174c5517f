"""Bound files on the GPU: a hierarchy saved with bbc_bounds_save and read
back with bbc_bounds_load answers exactly like the handle that wrote it
(same statistics, leaves, receiver grid, and bit-identical estimates in the
fused and staged query forms), for every chain and for area lights; a loaded
handle can be rebuilt like any other."""
import numpy as np
import pytest

from paper_2504_19163_amd import scenes as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = {
    "R": (lambda: S.heightfield_mirror(8), dict(max_depth=5)),
    "R_grid128": (lambda: S.curved_triangles(4, seed=7), dict(max_depth=4, grid_res=128)),
    "T": (lambda: S.curved_triangles(4, seed=7, chain="T", eta=1.0 / 1.5), dict(max_depth=4)),
    "RR": (lambda: S.double_mirror(), dict(max_depth=4)),
    # many leaves per tuple: the query's run bounds are rebuilt on load
    "RR_walls": (lambda: S.facing_walls(4), dict(max_depth=4)),
    "R_area": (lambda: S.area_light(S.flat_mirror(), [0.5, 0.0, 0.0], [0.0, 0.3, 0.0]), dict(max_depth=3)),
}


@pytest.fixture(scope="module")
def bbc():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2504_19163_amd import bbc as B
    B.lib()
    return B


def _same_export(A, B):
    ia, ib = A.info(), B.info()
    for k in ia:
        if k != "device_bytes":
            assert ia[k] == ib[k], k
    la, lb = A.leaves(), B.leaves()
    for k in la:
        assert np.array_equal(la[k], lb[k], equal_nan=True), k
    for x, y in zip(A.grid(), B.grid()):
        assert np.array_equal(x, y, equal_nan=True)


@pytest.mark.parametrize("case", list(CASES))
def test_saved_bounds_load_identically(bbc, tmp_path, case):
    make, params = CASES[case]
    sc = make()
    ds = bbc.DeviceScene(sc)
    A = bbc.Bounds(ds, params)
    path = tmp_path / f"{case}.bbc"
    A.save(path)
    print(case, "file bytes", path.stat().st_size, "leaves", A.info()["n_leaves"], flush=True)
    B = bbc.Bounds.load(path)
    _same_export(A, B)
    G = A.info()["grid_res"]
    pts = torch.as_tensor(S.random_points(sc, 3000, seed=5, grid_res=G), device="cuda")
    for mode in (bbc.QUERY_FUSED, bbc.QUERY_STAGED, bbc.QUERY_STAGED | bbc.QUERY_EXHAUSTIVE):
        Ea, sa = A.query(pts, 4, 99, mode=mode, stats=True)
        Eb, sb = B.query(pts, 4, 99, mode=mode, stats=True)
        torch.cuda.synchronize()
        assert torch.equal(Ea, Eb), mode
        assert torch.equal(sa, sb), mode
    # the loaded handle is an ordinary handle: a rebuild from the scene gives the same hierarchy
    B.dscene, B.params = ds, dict(bbc.default_params(), **params)
    B._p = bbc.SubdivParams(**B.params)
    B.rebuild()
    _same_export(A, B)
    # and saving the loaded handle writes the same bytes
    path2 = tmp_path / f"{case}_2.bbc"
    bbc.Bounds.load(path).save(path2)
    assert path.read_bytes() == path2.read_bytes()
    A.free()
    B.free()


def test_rebuilt_handle_saves_its_new_hierarchy(bbc, tmp_path):
    """Saving after a rebuild with other parameters writes the new hierarchy,
    not the buffers' larger capacities or the old counts."""
    sc = S.heightfield_mirror(8)
    ds = bbc.DeviceScene(sc)
    A = bbc.Bounds(ds, dict(max_depth=6))
    A.params = dict(bbc.default_params(), max_depth=2, grid_res=64)
    A._p = bbc.SubdivParams(**A.params)
    A.rebuild()
    A.save(tmp_path / "small.bbc")
    B = bbc.Bounds.load(tmp_path / "small.bbc")
    _same_export(A, B)
    C = bbc.Bounds(ds, dict(max_depth=2, grid_res=64))
    _same_export(C, B)


def test_loaded_bounds_serve_like_the_original(bbc, tmp_path):
    """A server over a loaded handle returns what the staged query of the
    handle that wrote the file returns, bit for bit."""
    sc = S.heightfield_mirror(8)
    A = bbc.Bounds(bbc.DeviceScene(sc), dict(max_depth=5))
    A.save(tmp_path / "serve.bbc")
    B = bbc.Bounds.load(tmp_path / "serve.bbc")
    pts = S.random_points(sc, 2000, seed=9)
    Ea, _ = A.query(torch.as_tensor(pts, device="cuda"), 16, 7, mode=bbc.QUERY_STAGED, point_index_base=100)
    torch.cuda.synchronize()
    srv = bbc.Server([B], hbm_budget_bytes=1 << 28, max_inflight=2)
    try:
        out, _ = srv.wait(srv.submit(0, pts, 16, 7, point_index_base=100))
    finally:
        srv.close()
    assert np.array_equal(out, Ea.cpu().numpy())
