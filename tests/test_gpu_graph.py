"""The staged query replayed as a HIP graph (BBC_TUNE_GRAPH) and served
batches replayed as graphs (BBC_SERVER_GRAPH): the same kernels with the same
arguments, so every result must be bit-identical to the direct launches, call
after call (the executable graph is updated in place with each call's
arguments, or re-instantiated when the launch sequence changes: other point
counts, sampler modes, sliced queries), with eager work and synchronisations
between the replays."""
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


CALLS = [  # (points seed, n, spp, seed, base, mode bits)
    (1, 3000, 16, 5, 0, 0), (2, 3000, 16, 6, 0, 0), (3, 777, 4, 7, 100, 0), (4, 5000, 64, 8, 0, 16),
    (5, 2000, 16, 9, 0, 96), (6, 2000, 8, 10, 0, 64), (7, 3000, 16, 11, 7, 32), (8, 64, 1, 12, 0, 0),
]


@pytest.mark.parametrize("scene", ["heightfield", "water"])
def test_graph_replay_equals_direct(bbc, scene):
    if scene == "heightfield":
        sc, params = S.heightfield_mirror(16), dict(max_depth=4)
    else:
        sc, params = S.water_surface(m=8, amp_scale=0.04), dict(max_depth=4)
    B = bbc.Bounds(bbc.DeviceScene(sc), params)
    for sliced in (False, True):
        if sliced:  # several slices per query: a longer launch sequence
            off = B.grid()[0].astype(np.int64)
            B.set_tuning(bbc.TUNE_STAGED_PAIRS, max(1, int(np.diff(off).max())) * 300)
        for ps, n, spp, seed, base, bits in CALLS:
            pts = torch.as_tensor(S.random_points(sc, n, seed=ps), device="cuda")
            mode = bbc.QUERY_STAGED | bits
            B.set_tuning(bbc.TUNE_GRAPH, 0)
            ref, rst = B.query(pts, spp, seed, mode=mode, stats=True, point_index_base=base)
            torch.cuda.synchronize()
            B.set_tuning(bbc.TUNE_GRAPH, 1)
            for rep in range(3):
                got, gst = B.query(pts, spp, seed, mode=mode, stats=True, point_index_base=base)
                torch.ones(1024, device="cuda").mul_(2.0)  # eager work between replays
                torch.cuda.synchronize()
                assert torch.equal(got, ref), (scene, sliced, n, bits, rep)
                assert torch.equal(gst, rst), (scene, sliced, n, bits, rep)
    B.set_tuning(bbc.TUNE_GRAPH, 0)
    B.free()


def test_served_graph_batches_equal_alone(bbc):
    sc = S.heightfield_mirror(16)
    B = bbc.Bounds(bbc.DeviceScene(sc), dict(max_depth=4))
    rng = np.random.default_rng(3)
    reqs = []
    for k in range(30):
        n = int(rng.integers(1, 3000))
        reqs.append((S.random_points(sc, n, seed=200 + k), int(rng.choice([1, 4, 16])), int(rng.integers(0, 2**62)),
                     int(rng.integers(0, 1000))))
    ref = []
    for pts, spp, seed, base in reqs:
        E, _ = B.query(torch.as_tensor(pts, device="cuda"), spp, seed, mode=bbc.QUERY_STAGED, point_index_base=base)
        ref.append(E.cpu().numpy())
    for paused in (True, False):
        srv = bbc.Server([B], hbm_budget_bytes=1 << 28, max_inflight=3, max_batch_points=8192, max_batch_requests=8,
                         paused=paused, graph=True)
        try:
            ts = [srv.submit(0, pts, spp, seed, point_index_base=base) for pts, spp, seed, base in reqs]
            if paused:
                srv.resume()
            for t, e in zip(ts, ref):
                got = srv.wait(t)[0]
                assert np.array_equal(got.view(np.uint32), e.view(np.uint32))
        finally:
            srv.close()
    B.free()


@pytest.mark.parametrize("case", ["heightfield", "water", "walls", "area"])
def test_build_graph_replay_equals_direct(bbc, case):
    """BBC_TUNE_BUILD_GRAPH: the build's launch sequence captured and replayed
    gives the directly launched build's leaves and grid, bit for bit, on the
    first capture and on rebuilds that update the executable graph, with
    eager work between them."""
    if case == "heightfield":
        sc, params = S.heightfield_mirror(16), dict(max_depth=4)
    elif case == "water":
        sc, params = S.water_surface(m=8, amp_scale=0.04), dict(max_depth=4)
    elif case == "walls":
        sc, params = S.facing_walls(4), dict(max_depth=4, alpha=10.0)
    else:
        sc, params = S.area_light(S.heightfield_mirror(8), [0.6, 0.0, 0.0], [0.0, 0.4, 0.0]), dict(max_depth=3)
    B0 = bbc.Bounds(bbc.DeviceScene(sc), params)
    L0, g0 = B0.leaves(), B0.grid()
    B = bbc.Bounds(bbc.DeviceScene(sc), params)
    B.set_tuning(bbc.TUNE_BUILD_GRAPH, 1)
    for rep in range(3):
        B.rebuild()
        torch.ones(1024, device="cuda").mul_(2.0)
        torch.cuda.synchronize()
        L, g = B.leaves(), B.grid()
        for k in ("tuple", "code", "uk", "E"):
            assert np.array_equal(np.asarray(L[k]), np.asarray(L0[k])), (case, rep, k)
        for a, b in zip(g, g0):
            assert np.array_equal(np.asarray(a).view(np.uint8), np.asarray(b).view(np.uint8)), (case, rep)
    assert B.info()["n_boxes"] == B0.info()["n_boxes"]
    B.free()
    B0.free()
