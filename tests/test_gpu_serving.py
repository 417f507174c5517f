"""Continuous-batching server on the GPU (bbc_server_*): every request's
result is bit-identical to the same request run alone through
bbc_query_irradiance_ex, whatever batch it lands in; a sample of requests
matches the FP64 oracle; admission by memory budget, the queue limit and the
never-fits rejection behave as declared."""
import threading
import time

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


@pytest.fixture(scope="module")
def two_scenes(bbc):
    a = S.heightfield_mirror(16)
    b = S.curved_triangles(40, seed=3)
    out = []
    for sc, depth in ((a, 4), (b, 5)):
        ds = bbc.DeviceScene(sc)
        out.append((sc, ds, bbc.Bounds(ds, dict(max_depth=depth))))
    return out


def _requests(scenes, n_req, seed, max_n=3000):
    rng = np.random.default_rng(seed)
    reqs = []
    for k in range(n_req):
        s = int(rng.integers(0, len(scenes)))
        n = int(rng.integers(0, max_n)) if k % 7 else 0 if k == 7 else int(rng.integers(1, 64))
        pts = S.random_points(scenes[s][0], n, seed=1000 + k) if n else np.zeros((3, 0), np.float32)
        reqs.append(dict(scene=s, pts=np.ascontiguousarray(pts, np.float32), spp=int(rng.choice([1, 4, 16, 64])),
                         seed=int(rng.integers(0, 2**63)), base=int(rng.integers(0, 5000)), device=bool(k % 3 == 0)))
    return reqs


def _alone(bbc, scenes, r):
    B = scenes[r["scene"]][2]
    if r["pts"].shape[1] == 0:
        return np.zeros(0, np.float32)
    E, _ = B.query(torch.as_tensor(r["pts"], device="cuda"), r["spp"], r["seed"], mode=bbc.QUERY_STAGED,
                   point_index_base=r["base"])
    return E.cpu().numpy()


def _submit(srv, r):
    pts = torch.as_tensor(r["pts"], device="cuda") if r["device"] else r["pts"]
    return srv.submit(r["scene"], pts, r["spp"], r["seed"], point_index_base=r["base"])


def _host(out):
    return out.cpu().numpy() if hasattr(out, "cpu") else out


def test_mix_equals_alone_bitwise(bbc, two_scenes):
    reqs = _requests(two_scenes, 48, seed=1)
    ref = [_alone(bbc, two_scenes, r) for r in reqs]
    srv = bbc.Server([b for _, _, b in two_scenes], hbm_budget_bytes=1 << 30, max_inflight=4,
                     max_batch_points=16384, max_batch_requests=64, paused=True)
    try:
        tickets = [_submit(srv, r) for r in reqs]
        srv.resume()
        for t, r, e in zip(tickets, reqs, ref):
            out, lat = srv.wait(t)
            got = _host(out)
            assert got.shape == e.shape
            assert np.array_equal(got.view(np.uint32), e.view(np.uint32)), (r["scene"], r["pts"].shape, r["spp"])
            assert lat >= 0.0
        st = srv.stats()
        assert st["completed"] == st["submitted"] == len(reqs)
        assert st["batches"] < len(reqs)  # requests were batched together
        assert st["points"] == sum(r["pts"].shape[1] for r in reqs)
        assert 0 < st["arena_peak_bytes"] <= st["arena_bytes"]
        assert st["latency_p50_ms"] <= st["latency_p99_ms"] <= st["latency_max_ms"]
    finally:
        srv.close()


def test_continuous_arrivals_from_threads(bbc, two_scenes):
    """Requests arrive from two host threads while batches run; results still
    equal the alone runs."""
    reqs = _requests(two_scenes, 40, seed=2, max_n=6000)
    ref = [_alone(bbc, two_scenes, r) for r in reqs]
    for r in reqs:
        r["device"] = False  # host requests only: submitted from plain threads
    srv = bbc.Server([b for _, _, b in two_scenes], hbm_budget_bytes=1 << 30, max_inflight=3,
                     max_batch_points=8192, max_batch_requests=16)
    results = [None] * len(reqs)
    try:
        def client(idx):
            rng = np.random.default_rng(idx[0])
            for k in idx:
                time.sleep(float(rng.exponential(0.002)))
                t = _submit(srv, reqs[k])
                results[k] = srv.wait(t)[0]

        th = [threading.Thread(target=client, args=(list(range(j, len(reqs), 2)),)) for j in range(2)]
        for t in th:
            t.start()
        for t in th:
            t.join(timeout=120)
        for got, e in zip(results, ref):
            assert got is not None
            assert np.array_equal(got.view(np.uint32), e.view(np.uint32))
    finally:
        srv.close()


def test_served_requests_match_oracle(bbc, orc, two_scenes):
    """Two served requests against the FP64 oracle: the oracle's point index
    is the position in its input, so the request's points are placed after
    `base` points off the receiver."""
    sc, ds, B = two_scenes[0]
    osc = orc.OracleScene(sc)
    Ob = orc.OracleBuild(osc, dict(max_depth=4))
    srv = bbc.Server([B], hbm_budget_bytes=256 << 20, max_inflight=2, max_batch_points=4096)
    try:
        for base, n, spp, seed in ((0, 700, 16, 5), (1234, 333, 4, 77)):
            pts = S.random_points(sc, n, seed=50 + base)
            out, _ = srv.wait(srv.submit(0, pts, spp, seed, point_index_base=base))
            off = np.full((3, base), 100.0)
            full = np.concatenate([off, pts.astype(np.float64)], 1)
            OE, _ = Ob.query(full, spp, seed, mode=0)
            np.testing.assert_allclose(out.astype(np.float64), OE[base:], rtol=1e-5, atol=1e-12)
    finally:
        srv.close()


def test_budget_admission_and_rejections(bbc, two_scenes):
    sc, ds, B = two_scenes[0]
    # never fits: more points than a batch holds, or more work space than the whole budget
    srv = bbc.Server([B], hbm_budget_bytes=1 << 20, max_inflight=2, max_batch_points=1 << 20)
    try:
        big = S.random_points(sc, 200000, seed=1)
        with pytest.raises(bbc.BBCError) as ei:
            srv.submit(0, big, 4, 1)
        assert ei.value.status == bbc.EBUDGET
        small = S.random_points(sc, 64, seed=2)
        out, _ = srv.wait(srv.submit(0, small, 4, 1))
        assert np.array_equal(out, _alone(bbc, two_scenes, dict(scene=0, pts=small, spp=4, seed=1, base=0)))
        assert srv.stats()["rejected"] == 1
    finally:
        srv.close()
    srv = bbc.Server([B], hbm_budget_bytes=1 << 24, max_inflight=2, max_batch_points=1000)
    try:
        with pytest.raises(bbc.BBCError) as ei:
            srv.submit(0, S.random_points(sc, 1001, seed=1), 4, 1)
        assert ei.value.status == bbc.EBUDGET
    finally:
        srv.close()
    # queue limit: a paused server with room for two waiting requests
    srv = bbc.Server([B], hbm_budget_bytes=1 << 24, max_inflight=2, max_batch_points=4096, queue_capacity=2,
                     paused=True)
    try:
        p = S.random_points(sc, 100, seed=3)
        t1, t2 = srv.submit(0, p, 4, 1), srv.submit(0, p, 4, 2)
        with pytest.raises(bbc.BBCError) as ei:
            srv.submit(0, p, 4, 3)
        assert ei.value.status == bbc.EQUEUE
        done, _ = srv.poll(t1)
        assert not done
        srv.resume()
        srv.wait(t1)
        srv.wait(t2)
        with pytest.raises(bbc.BBCError):
            srv.poll(t1)  # retired
    finally:
        srv.close()


def test_budget_limits_concurrency(bbc, two_scenes):
    """A budget that holds one batch at a time: batches queue for memory, the
    arena never exceeds the budget, results are unchanged."""
    reqs = [r for r in _requests(two_scenes, 12, seed=5, max_n=2000) if r["scene"] == 0]
    for r in reqs:
        r["device"] = False
    ref = [_alone(bbc, two_scenes, r) for r in reqs]
    B = two_scenes[0][2]
    # work space of one request of 2000 points, with room for one at a time
    probe = bbc.Server([B], hbm_budget_bytes=1 << 30, max_inflight=1, max_batch_points=2000, max_batch_requests=1)
    try:
        probe.wait(probe.submit(0, S.random_points(two_scenes[0][0], 2000, seed=9), 4, 1))
        one = probe.stats()["arena_peak_bytes"]
    finally:
        probe.close()
    srv = bbc.Server([B], hbm_budget_bytes=max(int(one * 1.5), 1 << 20), max_inflight=4, max_batch_points=2000,
                     max_batch_requests=1)
    try:
        ts = [_submit(srv, r) for r in reqs]
        for t, e in zip(ts, ref):
            assert np.array_equal(srv.wait(t)[0], e)
        st = srv.stats()
        assert st["arena_peak_bytes"] <= st["arena_bytes"]
        assert st["batches"] == len(reqs)
    finally:
        srv.close()


def test_sliced_batches_equal_whole(bbc, two_scenes):
    """A small BBC_TUNE_STAGED_PAIRS makes the staged query and every served
    batch run as consecutive launches over slices of their points (the path a
    scene with very full grid cells takes at full size); each point keeps its
    request's random stream, so results equal the whole-launch ones bit for
    bit."""
    reqs = [r for r in _requests(two_scenes, 24, seed=8, max_n=2500)]
    ref = [_alone(bbc, two_scenes, r) for r in reqs]
    bounds = [b for _, _, b in two_scenes]
    old = [b.get_tuning(bbc.TUNE_STAGED_PAIRS) for b in bounds]
    try:
        for b in bounds:
            off = b.grid()[0].astype(np.int64)
            # slices of about 100 points at the worst case
            b.set_tuning(bbc.TUNE_STAGED_PAIRS, max(1, int(np.diff(off).max())) * 100)
        sliced = [_alone(bbc, two_scenes, r) for r in reqs]
        for e, g in zip(ref, sliced):
            assert np.array_equal(e.view(np.uint32), g.view(np.uint32))
        srv = bbc.Server(bounds, hbm_budget_bytes=1 << 28, max_inflight=3, max_batch_points=16384,
                         max_batch_requests=64, paused=True)
        try:
            tickets = [_submit(srv, r) for r in reqs]
            srv.resume()
            for t, e in zip(tickets, ref):
                got = _host(srv.wait(t)[0])
                assert np.array_equal(got.view(np.uint32), e.view(np.uint32))
            assert srv.stats()["batches"] < len(reqs)
        finally:
            srv.close()
    finally:
        for b, v in zip(bounds, old):
            b.set_tuning(bbc.TUNE_STAGED_PAIRS, v)
