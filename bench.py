#!/usr/bin/env python3
"""Benchmark of the bound-driven caustic estimator on one MI355X.

Headline workload (the serving stream): the bound hierarchies of three scenes
are built once and stay resident in device memory --

  * single reflection off a displaced sphere (131072 triangles, point light at
    distance 3, depth cap 8),
  * single refraction through a water surface (524288 triangles x 4 point
    lights, wave amplitudes scaled by 0.04, depth cap 6),
  * two reflections between two facing rippled walls (8192 + 8192 triangles,
    67.1 M candidate pairs, depth cap 6, alpha 10) --

and a stream of shading-point query requests is answered over them: request
sizes floor(exp U[ln 256, ln 65536]) points uniform on the chosen receiver,
W (expected tuple samples per point) uniform over {16, 32, 64, 128, 256}, the
scene uniform over the three.  A step is one chunk of consecutive requests of
the stream; each query runs gather, bound-optimal probabilities, Bernoulli
selection, Newton root-finding and the estimate.  The served form is the
library's continuous-batching server (64 GB budget, 4 batch slots); the plain
form answers each request with its own one-launch-per-stage staged query on
one stream.  Both draw identical random numbers, so their estimates (and
errors) are bit-identical; that is checked.  `value` is the served form's
shading-point queries per second over the timed steps, inputs and outputs
resident in device memory.  `latency_ms` is submit-to-ready batch latency of
the served form under Poisson arrivals at the plain form's capacity.

`roofline` is for the stream's dominant kernel (the staged query's pooled
Newton kernel), timed with HIP events on its stream over the plain form's
timed pass.  Sections report each configuration on its own (the sphere's
whole step of build + query, with the roofline of its dominant build kernel),
the sampling schemes, the implicit irradiance bound, area lights, the literal
water spectrum, and the FP64 oracle on the host cores (`cpu_baseline`).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "shading-point caustic queries/s at matched error; p50/p99 batch latency"
WORKLOAD = ("serving stream over device-resident bounds of three scenes: displaced sphere 131072 triangles "
            "(single reflection, depth cap 8), water surface 524288 triangles x 4 lights (single refraction, "
            "amplitudes x 0.04, depth cap 6), facing walls 8192 + 8192 triangles (two reflections, 67.1M candidate "
            "pairs, depth cap 6); requests of floor(exp U[ln 256, ln 65536]) points, W uniform over "
            "{16,32,64,128,256}, scene uniform; 64 GB work-space budget, 4 batch slots")
# MI355X published vector peaks (TFLOP/s).  FP32 157.3 counts packed FP32
# (two lanes per instruction); this library compiles without packed FP32, so
# its FP32 and FP64 code both issue at 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA)
# x 2.4 GHz = 78.6 TFLOP/s.
PEAK_FP32 = 157.3
PEAK_FP64 = 78.6
PEAK_UNPACKED = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# Algorithmic work (counted on the method, not on the code).  Newton: ~150 flop
# per iteration (value and Jacobian of the rational map, the 2x2 solve).  One
# subdivision box of the single reflection: the midpoint quad split of the
# position tensors (three of degree (4,4): 900 flop) and of the irradiance
# tensors (two of degree (10,10): 3630 flop), and 3 flop per coefficient pair
# of its ratio bounds (Pu/Q and Pv/Q at 25 pairs, t at 16, |Q^3/det M| at 121).
FLOP_NEWTON_ITER = 150
# The same counted per chain on the code's path evaluation (value and
# Jacobian by forward differentiation, the 2x2 step; FMA = 2, a division,
# reciprocal or square root = 1): single reflection ~256, refraction ~330,
# two reflections ~670 (two reflected directions with dual-number derivatives
# and six rational divisions).
FLOP_ITER_COUNTED = {"sphere131072": 256, "water512x512": 330, "walls64x64": 670}
FLOP_SUBDIV_BOX = 900 + 3630 + 3 * (25 + 25 + 16 + 121)
# HBM bytes of one launch of a kernel from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE (KiB per dispatch), each scaled by what the counter reads for a
# 256 MiB device copy; valid only while the kernel sources hash to the digest
# they were measured with (null afterwards).
COUNTERS = {
    # the subdivision, per build of the sphere (k_subdiv_split at depth 0 and
    # k_subdiv_rec below: 9 launches, 39,961 boxes; builds 2 and 3 of
    # profiles/subdiv_sphere131072_hbm_sq_counters.md averaged)
    "k_subdiv": dict(
        sources=['paper_2504_19163_amd/csrc/build.hip', 'paper_2504_19163_amd/csrc/box_r.hpp', 'paper_2504_19163_amd/csrc/bern_dev.hpp', 'paper_2504_19163_amd/csrc/dev_common.hpp', 'paper_2504_19163_amd/csrc/geom_dev.hpp'],
        sha256="43fa6aa2f1af37c4b7bee41c7be93125528047cd0c57e94723b898cb2dc79ec6",
        fetch_kib=71004.8, write_kib=149273.8, fetch_scale=262144.0 / 131088.625, write_scale=1.0),
    # the pooled Newton kernels of the serving stream, mean per launch over the
    # run's launches of all three chains (394 counted for FETCH_SIZE and for
    # WRITE_SIZE)
    # (profiles/serving_stream_three_scenes_newton_hbm_counters.md)
    "newton_stream": dict(
        sources=['paper_2504_19163_amd/csrc/query.hip', 'paper_2504_19163_amd/csrc/path_dev.hpp', 'paper_2504_19163_amd/csrc/geom_dev.hpp', 'paper_2504_19163_amd/csrc/dev_common.hpp', 'paper_2504_19163_amd/csrc/internal.hpp'],
        sha256="eecbcd64d127a02780a320f12d58cca114571f7c3bfa99498cce820dcaa700ce",
        fetch_kib=135773.6, write_kib=89223.6, fetch_scale=262144.0 / 131088.9375, write_scale=1.0),
}


def traffic_bytes(name):
    import hashlib
    c = COUNTERS.get(name)
    if c is None:
        return None
    h = hashlib.sha256()
    for f in c["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != c["sha256"]:
        return None
    return int(round((c["fetch_kib"] * c["fetch_scale"] + c["write_kib"] * c["write_scale"]) * 1024))


def cpu_info():
    try:
        n_aff = len(os.sched_getaffinity(0))
    except AttributeError:
        n_aff = os.cpu_count() or 1
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return n_aff, os.cpu_count() or n_aff, model


def relmse(est, ref):
    """RelMSE = mean((est - ref)^2 / (ref^2 + 0.01)) over the points (the
    paper's relative MSE with a 0.01 floor in the denominator)."""
    return float(np.mean((est - ref) ** 2 / (ref ** 2 + 1e-2)))


def make_trace(n_req, n_scenes, seed):
    """Requests of the serving stream: sizes floor(exp U[ln 256, ln 65536])
    points, W uniform over {16, 32, 64, 128, 256}, scene uniform."""
    rng = np.random.default_rng(seed)
    sizes = np.floor(np.exp(rng.uniform(np.log(256), np.log(65536), n_req))).astype(np.int64)
    spp = rng.choice([16, 32, 64, 128, 256], n_req)
    scene = rng.integers(0, n_scenes, n_req)
    seeds = rng.integers(0, 2**62, n_req)
    offs = rng.integers(0, 65536, n_req)
    return [dict(n=int(sizes[k]), spp=int(spp[k]), scene=int(scene[k]), seed=int(seeds[k]),
                 off=int(min(offs[k], 65536 - sizes[k]))) for k in range(n_req)]


def _wait_until(t0, t):
    while True:
        dt = t - (time.perf_counter() - t0)
        if dt <= 0:
            return
        if dt > 5e-4:
            time.sleep(dt - 3e-4)


def run_plain(bbc, torch, bounds, reqs, trace, outs, arrivals=None, kern=None):
    """One staged query per request on one stream, in arrival order; returns
    (makespan s, latencies ms).  kern (list): Newton kernel ms per request."""
    lat = []
    t0 = time.perf_counter()
    for k, r in enumerate(trace):
        if arrivals is not None:
            _wait_until(t0, arrivals[k])
        B = bounds[r["scene"]]
        B.query(reqs[k], r["spp"], r["seed"], mode=bbc.QUERY_STAGED, out=outs[k])
        if kern is not None:
            kern.append(B.kernel_ms())
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        lat.append(1e3 * (t - (arrivals[k] if arrivals is not None else 0.0)))
    return time.perf_counter() - t0, lat


def run_served(bbc, srv, reqs, trace, arrivals=None, outs=None):
    """Submit the requests to the server (at the arrival times, or all at
    once) and wait for all of them; returns (makespan s, latencies ms,
    outputs)."""
    import threading
    tickets = [None] * len(trace)
    res = [None] * len(trace)
    ready = threading.Semaphore(0)

    def waiter():
        for k in range(len(trace)):
            ready.acquire()
            res[k] = srv.wait(tickets[k])

    th = threading.Thread(target=waiter)
    th.start()
    t0 = time.perf_counter()
    for k, r in enumerate(trace):
        if arrivals is not None:
            _wait_until(t0, arrivals[k])
        tickets[k] = srv.submit(r["scene"], reqs[k], r["spp"], r["seed"], sync_inputs=False)
        ready.release()
    th.join()
    t1 = time.perf_counter()
    return t1 - t0, [x[1] for x in res], [x[0] for x in res]


SCENES = [
    ("sphere131072", "single reflection, displaced sphere 131072 triangles, depth cap 8",
     lambda S: S.displaced_sphere(7), dict(max_depth=8, sigma=1e-4, alpha=2.0, grid_res=512)),
    ("water512x512", "single refraction, water surface 524288 triangles x 4 lights (amplitudes x 0.04), depth cap 6",
     lambda S: S.water_surface(m=512, amp_scale=0.04), dict(max_depth=6, sigma=1e-4, alpha=2.0, grid_res=512)),
    ("walls64x64", "two reflections, facing walls 8192 + 8192 triangles (67.1M candidate pairs), depth cap 6",
     lambda S: S.facing_walls(64), dict(max_depth=6, sigma=1e-4, alpha=10.0, grid_res=512)),
]


def progress(msg):
    """One line per finished part of the run, on stderr (the JSON line is
    the only stdout output)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def build_resident(bbc, S, torch):
    out = []
    for key, desc, make, params in SCENES:
        sc = make(S)
        t0 = time.perf_counter()
        B = bbc.Bounds(bbc.DeviceScene(sc), params)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        bbc.apply_tuning(B, key)
        B.set_tuning(bbc.TUNE_TIMING, 1)
        out.append(dict(key=key, desc=desc, scene=sc, params=params, B=B, first_build_ms=1e3 * tb))
        progress(f"built {key} in {tb:.2f} s")
    return out


def serving_headline(bbc, torch, res, steps, warmup, chunk, seed=5, sweep=(0.5, 1.0, 2.0)):
    dev = torch.device("cuda:0")
    from paper_2504_19163_amd import scenes as S
    bounds = [r["B"] for r in res]
    pools = [torch.as_tensor(S.random_points(r["scene"], 65536, seed=77 + j), device=dev) for j, r in enumerate(res)]
    n_req = (warmup + steps) * chunk
    trace = make_trace(n_req, len(res), seed)
    reqs = [pools[r["scene"]][:, r["off"]:r["off"] + r["n"]].contiguous() for r in trace]
    outs = [torch.empty(r["n"], dtype=torch.float32, device=dev) for r in trace]
    chunks = [list(range(c * chunk, (c + 1) * chunk)) for c in range(warmup + steps)]
    torch.cuda.synchronize()

    # plain form: one staged query per request, Newton kernel timed per request
    kern = []
    plain_ms = []
    for c, idx in enumerate(chunks):
        k0 = len(kern)
        t, _ = run_plain(bbc, torch, bounds, [reqs[i] for i in idx], [trace[i] for i in idx],
                         [outs[i] for i in idx], kern=kern)
        if c >= warmup:
            plain_ms.append(1e3 * t)
        else:
            del kern[k0:]
    timed = [i for idx in chunks[warmup:] for i in idx]
    plain_out = [outs[i].clone() for i in range(n_req)]
    progress(f"plain form: {sum(plain_ms):.1f} ms over {steps} steps")

    serve_graph = bool(bbc.tuned_value("serving", "graph", 0))
    srv = bbc.Server(bounds, hbm_budget_bytes=64 << 30, max_inflight=4, max_batch_points=1 << 20,
                     max_batch_requests=1024, queue_capacity=1 << 16, graph=serve_graph)
    try:
        served_ms = []
        got = [None] * n_req
        for c, idx in enumerate(chunks):
            if c == warmup:
                srv.stats(reset=True)
                torch.cuda.synchronize()
                t_timed0 = time.perf_counter()
            t, _, o = run_served(bbc, srv, [reqs[i] for i in idx], [trace[i] for i in idx])
            for i, x in zip(idx, o):
                got[i] = x
            if c >= warmup:
                served_ms.append(1e3 * t)
        torch.cuda.synchronize()
        t_timed = time.perf_counter() - t_timed0
        st_cap = srv.stats(reset=True)
        progress(f"served form: {1e3 * t_timed:.1f} ms over {steps} steps")
        identical = all(torch.equal(got[i], plain_out[i]) for i in range(n_req))
        n_pts = sum(trace[i]["n"] for i in timed)
        plain_s = sum(plain_ms) / 1e3
        cap_req = len(timed) / plain_s
        # latency under Poisson arrivals, both forms on the same timed requests
        rng = np.random.default_rng(seed + 1)
        tt = [trace[i] for i in timed]
        tr = [reqs[i] for i in timed]
        to = [outs[i] for i in timed]
        rows = []
        for x in sweep:
            rate = x * cap_req
            arr = np.cumsum(rng.exponential(1.0 / rate, len(timed)))
            tp, lp = run_plain(bbc, torch, bounds, tr, tt, to, arrivals=arr)
            ts, ls, _ = run_served(bbc, srv, tr, tt, arrivals=arr)
            st = srv.stats(reset=True)
            progress(f"Poisson arrivals at {x} x the plain capacity done")
            rows.append({"rate_x_plain_capacity": x, "offered_req_s": round(rate, 1),
                         "plain": {"queries_s": round(n_pts / tp, 1), "p50_ms": round(float(np.percentile(lp, 50)), 3),
                                   "p99_ms": round(float(np.percentile(lp, 99)), 3)},
                         "served": {"queries_s": round(n_pts / ts, 1), "p50_ms": round(float(np.percentile(ls, 50)), 3),
                                    "p99_ms": round(float(np.percentile(ls, 99)), 3),
                                    "mean_batch_requests": round(st["mean_batch_requests"], 2)}})
    finally:
        srv.close()

    # algorithmic work of the plain timed pass: the same requests again with
    # the library's work counters (same seeds, so the same iterations)
    it32 = it64 = pairs = 0
    per_scene = {r["key"]: dict(requests=0, points=0, it32=0, it64=0) for r in res}
    for i in timed:
        r = trace[i]
        _, _, hs = bounds[r["scene"]].query(reqs[i], r["spp"], r["seed"], mode=bbc.QUERY_STAGED, host_stats=True)
        it32 += hs["n_iter_fp32"]
        it64 += hs["n_iter_fp64"]
        pairs += hs["n_pairs"]
        ps = per_scene[res[r["scene"]]["key"]]
        ps["requests"] += 1
        ps["points"] += r["n"]
        ps["it32"] += hs["n_iter_fp32"]
        ps["it64"] += hs["n_iter_fp64"]
    kms = float(np.sum(kern))
    return dict(
        n_points=n_pts, timed_s=t_timed, served_ms=served_ms, plain_ms=plain_ms, identical=identical,
        cap_req=cap_req, sweep=rows, st_cap=st_cap, newton_ms=kms, serve_graph=serve_graph, newton_launch_ms=kms / max(1, len(kern)),
        it32=it32, it64=it64, pairs=pairs, per_scene=per_scene, n_timed=len(timed), trace=trace, reqs=reqs,
        plain_out=plain_out)


MATCHED_SPP = {"sphere131072": 64, "water512x512": 64, "walls64x64": 256}  # each workload's samples per point


def matched_error(bbc, torch, res, n_side=64, seeds=4):
    """RelMSE of the estimate against the exhaustive sum over each point's
    candidate list (every tuple of U evaluated, P = 1) on a fixed 64 x 64
    grid of shading points per scene at the workload's samples per point,
    mean over seeds.  Served and plain estimates are bit-identical, so this is
    the error of both forms."""
    from paper_2504_19163_amd import scenes as S
    out = {}
    for r in res:
        spp = MATCHED_SPP[r["key"]]
        B = r["B"]
        pts = torch.as_tensor(S.receiver_points(r["scene"], n_side), device="cuda:0")
        ex, _ = B.query(pts, 1, 0, mode=bbc.QUERY_STAGED | bbc.QUERY_EXHAUSTIVE)
        ref = ex.double().cpu().numpy()
        errs = []
        for k in range(seeds):
            E, _ = B.query(pts, spp, 900 + k, mode=bbc.QUERY_STAGED)
            errs.append(relmse(E.double().cpu().numpy(), ref))
        out[r["key"]] = {"relmse": float(np.mean(errs)), "points": int(pts.shape[1]), "spp": spp,
                         "seeds": seeds, "lit_points": int(np.count_nonzero(ref))}
    return out


def whole_step_section(bbc, torch, r, steps=5, spp=64, n_side=512):
    """One configuration on its own: a step is a rebuild of its bounds plus the
    staged query of n_side^2 receiver points at W = spp; the subdivision
    kernels are timed with HIP events on the build's stream (roofline of the
    build's dominant kernel)."""
    from paper_2504_19163_amd import scenes as S
    B = r["B"]
    pts = torch.as_tensor(S.receiver_points(r["scene"], n_side), device="cuda:0")
    B.rebuild()
    B.query(pts, spp, 0, mode=bbc.QUERY_STAGED)
    torch.cuda.synchronize()
    tb, tq, sub = [], [], []
    for k in range(steps):
        t = time.perf_counter()
        B.rebuild()
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t)
        sub.append(B.build_kernel_ms())
        t = time.perf_counter()
        B.query(pts, spp, 1 + k, mode=bbc.QUERY_STAGED)
        torch.cuda.synchronize()
        tq.append(time.perf_counter() - t)
    _, _, qs = B.query(pts, spp, 1, mode=bbc.QUERY_STAGED, host_stats=True)
    info = B.info()
    n = pts.shape[1]
    b, q = float(np.median(tb)), float(np.median(tq))
    sub_ms = float(np.median([s[0] for s in sub]))
    out = {"workload": f"{r['desc']}, {n_side}x{n_side} receiver points, {spp} samples/point",
           "queries_s_whole_step": round(n / (b + q), 1), "build_ms": round(1e3 * b, 3),
           "query_ms": round(1e3 * q, 3), "query_only_queries_s": round(n / q, 1),
           "first_build_ms": round(r["first_build_ms"], 1), "subdivision_ms": round(sub_ms, 4),
           "subdivision_launches": sub[0][1],
           "tuples": info["n_tuples"], "live_tuples": info["n_live_tuples"], "boxes": info["n_boxes"],
           "leaves": info["n_leaves"], "inf_leaves": info["n_inf_leaves"], "grid_entries": info["n_grid_entries"],
           "device_bytes": info["device_bytes"], "max_depth_reached": info["max_depth_reached"],
           "pairs": qs["n_pairs"], "roots": qs["n_roots"], "mean_candidates_per_point": round(qs["sum_U"] / n, 2)}
    if r["scene"]["chain"] == "R" and r["scene"].get("eedge") is None:
        flop = info["n_boxes"] * FLOP_SUBDIV_BOX
        ach = flop / (sub_ms * 1e-3) / 1e12
        split = B.get_tuning(bbc.TUNE_SUBDIV_SPLIT) != 0
        kern = ("k_subdiv_split + k_subdiv_rec (adaptive subdivision, FP64: depth 0 from the box corners, "
                "deeper boxes from their parents' split polynomials)" if split else
                "k_subdiv (adaptive subdivision, FP64, every box from its corners)")
        out["roofline_subdivision"] = {
            "bound": "alu", "kernel": kern, "achieved": round(ach, 5),
            "peak": PEAK_FP64, "unit": "TFLOP/s", "frac": round(ach / PEAK_FP64, 6),
            "traffic": traffic_bytes("k_subdiv" if split else None), "traffic_unit": "HBM bytes per build (all launches)",
            "boxes_per_build": info["n_boxes"], "flop_per_box": FLOP_SUBDIV_BOX,
            "kernel_ms_per_build": round(sub_ms, 4), "launches_per_build": sub[0][1]}
    return out


def samplers_section(bbc, torch, B, pts, spps=(4, 16), seeds=4, reps=5):
    """The sampling schemes side by side (the paper's sampling-scheme
    comparison): RelMSE against the exhaustive sum over U at equal expected
    samples per point W, the staged query time, samples and roots per point."""
    ex, _ = B.query(pts, 1, 0, mode=bbc.QUERY_STAGED | bbc.QUERY_EXHAUSTIVE)
    ref = ex.double().cpu().numpy()
    modes = {"bound_optimal": 0, "bins": bbc.QUERY_BINS, "one_sample": bbc.QUERY_ONE_SAMPLE,
             "uniform": bbc.QUERY_UNIFORM}
    n = pts.shape[1]
    out = {"reference": "exhaustive sum over the cell list (enumerate)", "seeds": seeds}
    for spp in spps:
        row = {}
        for name, m in modes.items():
            mode = bbc.QUERY_STAGED | m
            times, errs = [], []
            for k in range(max(seeds, reps)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                E, _ = B.query(pts, spp, 500 + k, mode=mode)
                torch.cuda.synchronize()
                times.append(1e3 * (time.perf_counter() - t0))
                if k < seeds:
                    errs.append(relmse(E.double().cpu().numpy(), ref))
            _, _, qs = B.query(pts, spp, 500, mode=mode, host_stats=True)
            row[name] = {"relmse": float(np.mean(errs)), "query_ms": round(float(np.median(times)), 3),
                         "samples_per_point": round(qs["sum_S"] / n, 3),
                         "roots_per_point": round(qs["n_roots"] / n, 4)}
        out[f"spp{spp}"] = row
    times = []
    for k in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.query(pts, 1, 0, mode=bbc.QUERY_STAGED | bbc.QUERY_EXHAUSTIVE)
        torch.cuda.synchronize()
        times.append(1e3 * (time.perf_counter() - t0))
    _, _, qs = B.query(pts, 1, 0, mode=bbc.QUERY_STAGED | bbc.QUERY_EXHAUSTIVE, host_stats=True)
    out["enumerate"] = {"relmse": 0.0, "query_ms": round(float(np.median(times)), 3),
                        "samples_per_point": round(qs["sum_S"] / n, 3), "roots_per_point": round(qs["n_roots"] / n, 4)}
    return out


def implicit_section(bbc, S, torch, steps=2):
    """The water surface with the irradiance bound by implicit differentiation
    (build and query timed, RelMSE against the exhaustive sum)."""
    dev = torch.device("cuda:0")
    sc = S.water_surface(m=512, amp_scale=0.04)
    params = dict(max_depth=6, sigma=1e-4, alpha=2.0, grid_res=512, flags=bbc.FLAG_IMPLICIT_IRR)
    B = bbc.Bounds(bbc.DeviceScene(sc), params)
    pts = torch.as_tensor(S.receiver_points(sc, 1024), device=dev)
    tb, tq = [], []
    for k in range(steps):
        t = time.perf_counter()
        B.rebuild()
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t)
        t = time.perf_counter()
        B.query(pts, 64, 1 + k, mode=bbc.QUERY_STAGED)
        torch.cuda.synchronize()
        tq.append(time.perf_counter() - t)
    sub = torch.as_tensor(S.receiver_points(sc, 64), device=dev)
    ex, _ = B.query(sub, 1, 0, mode=bbc.QUERY_STAGED | bbc.QUERY_EXHAUSTIVE)
    errs = [relmse(B.query(sub, 64, 900 + k, mode=bbc.QUERY_STAGED)[0].double().cpu().numpy(),
                   ex.double().cpu().numpy()) for k in range(4)]
    info = B.info()
    B.free()
    b, q = float(np.median(tb)), float(np.median(tq))
    return {"workload": "single refraction, water surface 524288 triangles x 4 lights (amplitudes x 0.04), depth cap "
                        "6, irradiance bound by implicit differentiation, 1024x1024 floor points, 64 samples/point",
            "relmse": float(np.mean(errs)), "build_ms": round(1e3 * b, 2), "query_ms": round(1e3 * q, 2),
            "queries_s_whole_step": round(pts.shape[1] / (b + q), 1), "boxes": info["n_boxes"],
            "leaves": info["n_leaves"], "inf_leaves": info["n_inf_leaves"], "grid_entries": info["n_grid_entries"]}


def degree_reduction_section(bbc, S, torch, steps=2, n_side=256, spp=256):
    """The facing walls built with and without the degree reduction of the
    irradiance ratio (Sec. 6.1): build and query time, tree, grid and the
    sampled estimate's RelMSE against the exhaustive sum of the same build."""
    dev = torch.device("cuda:0")
    sc = S.facing_walls(64)
    pts = torch.as_tensor(S.receiver_points(sc, n_side), device=dev)
    sub = torch.as_tensor(S.receiver_points(sc, 64), device=dev)
    out = {"workload": "two reflections, facing walls 8192 + 8192 triangles, depth cap 6, E-ratio 10, "
                       f"{n_side}x{n_side} receiver points, {spp} samples/point; with and without the reduction of "
                       "Den^3 and det M (46, 46) to degree (16, 16) plus remainders"}
    for name, flags in (("full_degree", 0), ("reduced", bbc.FLAG_DEGREE_REDUCTION)):
        B = bbc.Bounds(bbc.DeviceScene(sc), dict(max_depth=6, alpha=10.0, flags=flags))
        tb, tq = [], []
        for k in range(steps):
            t = time.perf_counter()
            B.rebuild()
            torch.cuda.synchronize()
            tb.append(time.perf_counter() - t)
            t = time.perf_counter()
            B.query(pts, spp, 1 + k, mode=bbc.QUERY_STAGED)
            torch.cuda.synchronize()
            tq.append(time.perf_counter() - t)
        ex, _ = B.query(sub, 1, 0, mode=bbc.QUERY_STAGED | bbc.QUERY_EXHAUSTIVE)
        errs = [relmse(B.query(sub, spp, 900 + k, mode=bbc.QUERY_STAGED)[0].double().cpu().numpy(),
                       ex.double().cpu().numpy()) for k in range(4)]
        info = B.info()
        B.free()
        b, q = float(np.median(tb)), float(np.median(tq))
        out[name] = {"build_ms": round(1e3 * b, 2), "query_ms": round(1e3 * q, 2), "relmse": float(np.mean(errs)),
                     "boxes": info["n_boxes"], "leaves": info["n_leaves"], "inf_leaves": info["n_inf_leaves"],
                     "grid_entries": info["n_grid_entries"]}
    return out


def area_light_section(bbc, S, torch, steps=3):
    """Single reflection off a 65 x 65-vertex heightfield (8192 triangles) lit
    by a 0.4 x 0.4 area light, depth cap 3, 512 x 512 receiver points, 64
    samples per point (one light point per selected pair)."""
    dev = torch.device("cuda:0")
    sc = S.area_light(S.heightfield_mirror(64), [0.4, 0.0, 0.0], [0.0, 0.4, 0.0])
    params = dict(max_depth=3, sigma=1e-4, alpha=2.0, grid_res=512)
    B = bbc.Bounds(bbc.DeviceScene(sc), params)
    pts = torch.as_tensor(S.receiver_points(sc, 512), device=dev)
    B.query(pts, 64, 0, mode=bbc.QUERY_STAGED)
    torch.cuda.synchronize()
    tb, tq = [], []
    for k in range(steps):
        t = time.perf_counter()
        B.rebuild()
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t)
        t = time.perf_counter()
        B.query(pts, 64, 1 + k, mode=bbc.QUERY_STAGED)
        torch.cuda.synchronize()
        tq.append(time.perf_counter() - t)
    info = B.info()
    B.free()
    n = pts.shape[1]
    b, q = float(np.median(tb)), float(np.median(tq))
    return {"workload": "single reflection, heightfield 8192 triangles, 0.4 x 0.4 area light, depth cap 3, "
                        "512x512 receiver points, 64 samples/point",
            "queries_s_whole_step": round(n / (b + q), 1), "build_ms": round(1e3 * b, 2),
            "query_ms": round(1e3 * q, 2), "live_tuples": info["n_live_tuples"], "boxes": info["n_boxes"],
            "leaves": info["n_leaves"], "inf_leaves": info["n_inf_leaves"], "grid_entries": info["n_grid_entries"]}


def literal_water_section(bbc, S, torch, ms=(32, 64)):
    """The water spectrum as written (amplitudes U[0.01, 0.05] with
    wavelengths U[0.05, 0.5], slopes up to ~6) on crops of the surface
    tessellation: how the bound hierarchy grows with it."""
    rows = []
    for m in ms:
        sc = S.water_surface(m=m)
        try:
            t = time.perf_counter()
            B = bbc.Bounds(bbc.DeviceScene(sc), dict(max_depth=6, sigma=1e-4, alpha=2.0, grid_res=512))
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            info = B.info()
            pts = torch.as_tensor(S.receiver_points(sc, 256), device="cuda:0")
            _, _, qs = B.query(pts, 64, 1, mode=bbc.QUERY_STAGED, host_stats=True)
            rows.append({"triangles": 2 * m * m, "tuples": info["n_tuples"], "build_ms": round(1e3 * dt, 1),
                         "leaves": info["n_leaves"], "inf_leaves": info["n_inf_leaves"],
                         "grid_entries": info["n_grid_entries"], "device_bytes": info["device_bytes"],
                         "mean_candidates_per_point": round(qs["sum_U"] / pts.shape[1], 1)})
            B.free()
        except Exception as e:  # capacity limits are part of what this section reports
            rows.append({"triangles": 2 * m * m, "error": str(e)[:200]})
    return {"workload": "literal water spectrum (no amplitude scaling), 4 lights, depth cap 6", "crops": rows}


def cpu_baseline_section(bbc, torch, res, trace, reqs, plain_out, budget_s=20.0):
    """The FP64 oracle on the host cores over the sphere's share of the
    stream: its build of the sphere, then the stream's requests addressed to
    the sphere in order, each on all of its points (at their own point
    indices, so with the same random streams), until the oracle's query time
    passes budget_s; all cores, and one core on the first three of those
    requests (on at most 4096 of their points).  The oracle builds of the water surface
    (2.1 M tuples) and of the facing walls (67.1 M candidate pairs) take
    minutes to hours on a host and are not part of the sample.  The GPU's
    estimates for the sampled points are compared with the oracle's."""
    from oracle import oracle as O
    n_aff, n_all, model = cpu_info()
    cores = max(1, n_aff)
    sphere = res[0]
    t = time.perf_counter()
    ob = O.OracleBuild(O.OracleScene(sphere["scene"]), sphere["params"], n_threads=cores)
    t_build = time.perf_counter() - t
    done_pts, t_q, n_done, n_close = 0, 0.0, 0, 0
    single_pts, t_single = 0, 0.0
    for k, r in enumerate(trace):
        if r["scene"] != 0:
            continue
        if t_q > budget_s:
            break
        n = r["n"]
        take = np.arange(n, dtype=np.int64)
        pts = reqs[k].cpu().numpy().astype(np.float64)
        # the oracle's point index is the position in its input: the sampled
        # points sit at their own indices, the others far off the receiver
        full = np.full((3, int(take[-1]) + 1), 1e3)
        full[:, take] = pts[:, take]
        t = time.perf_counter()
        OE, _ = ob.query(full, r["spp"], r["seed"], mode=0, n_threads=cores)
        t_q += time.perf_counter() - t
        done_pts += len(take)
        g = plain_out[k].cpu().numpy().astype(np.float64)[take]
        n_close += int(np.sum(np.abs(g - OE[take]) <= 1e-5 * np.abs(OE[take]) + 1e-12))
        if n_done < 3:
            m = min(n, 4096)
            t = time.perf_counter()
            ob.query(full[:, :m], r["spp"], r["seed"], mode=0, n_threads=1)
            t_single += time.perf_counter() - t
            single_pts += m
        n_done += 1
    del ob
    return {"value": round(done_pts / t_q, 1) if t_q > 0 else None, "unit": "queries/s", "cores": cores,
            "kind": "oracle", "nproc": n_all, "cpu_model": model,
            "single_thread_queries_s": round(single_pts / t_single, 1) if t_single > 0 else None,
            "build_s_all_cores": round(t_build, 2),
            "sample": f"the stream's requests to the sphere scene: first {n_done}, each on all of its points "
                      f"({done_pts} points, {t_q:.1f} s of oracle queries on {cores} threads); the oracle's sphere "
                      f"build ({t_build:.1f} s) is precomputation, outside the rate; the water and walls scenes "
                      f"are not sampled (their oracle builds take minutes to hours)",
            "points_gpu_equal_oracle_1e-5": round(n_close / max(1, done_pts), 5)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--chunk", type=int, default=48, help="requests per step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sections", action="store_true", help="headline only")
    ap.add_argument("--no-sweep", action="store_true", help="skip the Poisson latency sweep")
    ap.add_argument("--sphere-step-only", action="store_true",
                    help="only the sphere's whole step (build + query), for kernel counter runs")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 256 MiB device-to-device tensor copy first (reference kernel for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (DESIGN.md describes how the "
              "method would shard); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2504_19163_amd import bbc, scenes as S

    bbc.lib()  # raises if the HIP library was not built
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.sphere_step_only:
        key, desc, make, params = SCENES[0]
        sc = make(S)
        t0 = time.perf_counter()
        B = bbc.Bounds(bbc.DeviceScene(sc), params)
        torch.cuda.synchronize()
        r = dict(key=key, desc=desc, scene=sc, params=params, B=B, first_build_ms=1e3 * (time.perf_counter() - t0))
        bbc.apply_tuning(B, key)
        B.set_tuning(bbc.TUNE_TIMING, 1)
        print(json.dumps({"sphere_whole_step": whole_step_section(bbc, torch, r, steps=max(1, args.steps))}), flush=True)
        B.free()
        return

    res = build_resident(bbc, S, torch)
    h = serving_headline(bbc, torch, res, args.steps, args.warmup, args.chunk,
                         sweep=() if args.no_sweep else (0.5, 1.0, 2.0))
    value = h["n_points"] / h["timed_s"]
    plain_qs = h["n_points"] / (sum(h["plain_ms"]) / 1e3)
    lat = next((r for r in h["sweep"] if r["rate_x_plain_capacity"] == 1.0), None)
    ach32 = h["it32"] * FLOP_NEWTON_ITER / (h["newton_ms"] * 1e-3) / 1e12
    counted = sum(v["it32"] * FLOP_ITER_COUNTED[k] for k, v in h["per_scene"].items())
    ach_counted = counted / (h["newton_ms"] * 1e-3) / 1e12
    ach64 = h["it64"] * FLOP_NEWTON_ITER / (h["newton_ms"] * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * h["timed_s"] / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32+fp64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "requests_per_step": args.chunk, "timed_requests": h["n_timed"],
                   "timed_points": int(h["n_points"]),
                   "requests_by_scene": {k: {"requests": v["requests"], "points": v["points"]}
                                         for k, v in h["per_scene"].items()},
                   "query_form": "served (continuous batching)", "parallelism": "single GPU"},
        "latency_ms": ({"p50": lat["served"]["p50_ms"], "p99": lat["served"]["p99_ms"],
                        "load": f"Poisson arrivals at the plain form's capacity ({lat['offered_req_s']} requests/s)"}
                       if lat else None),
        "plain": {"queries_s": round(plain_qs, 1), "ms_per_step": round(float(np.mean(h["plain_ms"])), 3),
                  "latency_ms": ({"p50": lat["plain"]["p50_ms"], "p99": lat["plain"]["p99_ms"]} if lat else None),
                  "form": "one staged query (one launch per stage) per request on one stream"},
        "speedup_vs_plain": round(value / plain_qs, 3),
        "results_identical_to_plain": bool(h["identical"]),
        "roofline": {"bound": "alu", "kernel": "staged query pooled Newton kernel (k_stage_newton_pool)",
                     "achieved": round(ach32, 5), "peak": PEAK_FP32, "unit": "TFLOP/s",
                     "frac": round(ach32 / PEAK_FP32, 6), "traffic": traffic_bytes("newton_stream"),
                     "traffic_unit": "HBM bytes per launch",
                     "flop_per_iteration": FLOP_NEWTON_ITER, "fp32_iterations": int(h["it32"]),
                     "fp64_polish_iterations": int(h["it64"]),
                     "fp64_polish_achieved_tflops": round(ach64, 5), "fp64_peak": PEAK_FP64,
                     "flop_per_iteration_counted": FLOP_ITER_COUNTED,
                     "fp32_iterations_by_scene": {k: int(v["it32"]) for k, v in h["per_scene"].items()},
                     "achieved_counted_tflops": round(ach_counted, 5),
                     "frac_counted": round(ach_counted / PEAK_FP32, 6),
                     "unpacked_fp32_peak": round(PEAK_UNPACKED, 1),
                     "kernel_ms_total": round(h["newton_ms"], 3), "avg_launch_ms": round(h["newton_launch_ms"], 4),
                     "timing": "HIP events around every Newton launch of the plain form's timed pass"},
        "serving": {"saturated": {"served_queries_s": round(value, 1), "plain_queries_s": round(plain_qs, 1),
                                  "mean_batch_requests": round(h["st_cap"]["mean_batch_requests"], 2),
                                  "inflight_peak": h["st_cap"]["inflight_peak"],
                                  "arena_peak_bytes": h["st_cap"]["arena_peak_bytes"],
                                  "batches_as_hip_graphs": h["serve_graph"]},
                    "poisson": h["sweep"]},
        "resident": {r["key"]: {"first_build_ms": round(r["first_build_ms"], 1),
                                "device_bytes": r["B"].info()["device_bytes"],
                                "leaves": r["B"].info()["n_leaves"],
                                "grid_entries": r["B"].info()["n_grid_entries"]} for r in res},
    }
    out["matched_error"] = matched_error(bbc, torch, res)
    progress("matched error done")
    if not args.no_sections:
        sphere = res[0]
        out["sphere_whole_step"] = whole_step_section(bbc, torch, sphere)
        out["water_whole_step"] = whole_step_section(bbc, torch, res[1], steps=2, n_side=1024)
        out["walls_whole_step"] = whole_step_section(bbc, torch, res[2], steps=2, spp=256, n_side=256)
        progress("whole-step sections done")
        pts = torch.as_tensor(S.receiver_points(sphere["scene"], 512), device=dev)
        out["samplers"] = samplers_section(bbc, torch, sphere["B"], pts)
        progress("samplers done")
        out["refraction_implicit"] = implicit_section(bbc, S, torch)
        out["area_light"] = area_light_section(bbc, S, torch)
        out["literal_water"] = literal_water_section(bbc, S, torch)
        out["degree_reduction"] = degree_reduction_section(bbc, S, torch)
        progress("implicit, area-light, literal-water and degree-reduction sections done")
    if not args.no_cpu_baseline:
        timed0 = args.warmup * args.chunk
        out["cpu_baseline"] = cpu_baseline_section(bbc, torch, res, h["trace"][timed0:], h["reqs"][timed0:],
                                                   h["plain_out"][timed0:])
        progress("cpu baseline done")
    for r in res:
        r["B"].free()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
