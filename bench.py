#!/usr/bin/env python3
"""Benchmark of the bound-driven caustic estimator on one MI355X.

Workload: single reflection off a displaced sphere (octahedral geodesic sphere,
7 subdivisions = 131072 triangles, radius 1 + 0.02 value noise), one point light
at distance 3, receiver plane behind the sphere sampled at 512 x 512 shading
points, subdivision depth cap 8, 64 expected tuple samples per point.

A step is one pass of the whole hot path over the batch: bound construction
(tuple culling, domain initialisation, adaptive subdivision, grid recording)
followed by the query of every shading point (gather, bound-optimal
probabilities, Bernoulli selection, Newton root-finding, estimate).  Inputs
(scene and points) are resident in device memory before the timed region.

Prints one JSON line.  `value` is shading-point queries per second of whole
steps.  `roofline` is for the step's dominant kernel (the query kernel, timed
with HIP events on its stream inside the timed region) against the chip's
unpacked FP32 / FP64 vector peak; `cpu_baseline` is the FP64 oracle on the
host cores for the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = ("single reflection, displaced sphere 131072 triangles (octahedral geodesic, 7 subdivisions), "
            "point light at distance 3, 512x512 receiver shading points, depth cap 8, 64 samples/point")
METRIC = "shading-point caustic queries/s at matched error; p50/p99 batch latency"
# Chip constants: 256 compute units x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz
# = 78.6 TFLOP/s for unpacked FP32 and for FP64 vector arithmetic alike (packed
# FP32 instructions are not used by this library).
PEAK_VALU_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# Algorithmic flops of one path evaluation with its Jacobian (eval_path, reflection),
# counted from the formulas: FMA = 2 flops.
FLOPS_PER_PATH_EVAL = 290
# HBM traffic of one Newton launch of this workload, from rocprofv3 --pmc
# FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each scaled by what the counter
# reads for a 256 MiB device copy (FETCH_SIZE reads half the copied bytes on
# this GPU, WRITE_SIZE all of them); see
# profiles/query_newton_sphere131072_hbm_counters.md.  Valid only for the
# kernel sources with this digest: reported as null once they change.
NEWTON_COUNTERS = dict(
    sources=["paper_2504_19163_amd/csrc/query.hip", "paper_2504_19163_amd/csrc/path_dev.hpp",
             "paper_2504_19163_amd/csrc/geom_dev.hpp", "paper_2504_19163_amd/csrc/dev_common.hpp"],
    sha256="603355a3c565364cffa7f6e91227239917d38a61b76a12481e28c41850b40606",
    fetch_kib=40841.4375, write_kib=47877.5, fetch_scale=262144.0 / 131087.75, write_scale=1.0)


def newton_traffic_bytes():
    import hashlib
    h = hashlib.sha256()
    for f in NEWTON_COUNTERS["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != NEWTON_COUNTERS["sha256"]:
        return None
    c = NEWTON_COUNTERS
    return int(round((c["fetch_kib"] * c["fetch_scale"] + c["write_kib"] * c["write_scale"]) * 1024))


def cpu_cores():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def relmse(est, ref):
    return float(np.mean((est - ref) ** 2 / (ref ** 2 + 1e-2)))


def make_trace(n_req, n_scenes, seed):
    """Request stream of the serving workload: sizes floor(exp U[ln 256, ln 65536])
    points, spp uniform over {16, 32, 64, 128, 256}, scene uniform."""
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


def run_plain(bbc, torch, bounds, reqs, trace, outs, arrivals=None):
    """One batch per request through the one-launch-per-stage path on one
    stream, in arrival order; returns (makespan s, latencies ms)."""
    lat = []
    t0 = time.perf_counter()
    for k, r in enumerate(trace):
        if arrivals is not None:
            _wait_until(t0, arrivals[k])
        bounds[r["scene"]].query(reqs[k], r["spp"], r["seed"], mode=bbc.QUERY_STAGED, out=outs[k])
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        lat.append(1e3 * (t - (arrivals[k] if arrivals is not None else 0.0)))
    return time.perf_counter() - t0, lat


def run_served(bbc, srv, reqs, trace, arrivals=None):
    """Submit the trace to the server (at the arrival times, or all at once)
    and wait for every request; returns (makespan s, latencies ms, outputs)."""
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


def refraction_section(bbc, S, torch, n_side=1024, steps=3, flags=0):
    """Single refraction through a 513 x 513-vertex water surface (524288
    triangles, 4 lights, amplitudes scaled by 0.04), depth cap 6, 1024 x 1024
    shading points on the pool floor, 64 samples per point: build and query
    timed separately (inputs resident in device memory).  flags selects the
    irradiance bound (0: explicit, FLAG_IMPLICIT_IRR: implicit
    differentiation); the estimate's RelMSE against the exhaustive sum over
    the cell list is measured on 128 x 128 of the points."""
    dev = torch.device("cuda:0")
    sc = S.water_surface(m=512, amp_scale=0.04)
    params = dict(max_depth=6, sigma=1e-4, alpha=2.0, grid_res=512, flags=flags)
    t0 = time.perf_counter()
    B = bbc.Bounds(bbc.DeviceScene(sc), params)
    torch.cuda.synchronize()
    first_build = time.perf_counter() - t0
    pts = torch.as_tensor(S.receiver_points(sc, n_side), device=dev)
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
    _, _, qs = B.query(pts, 64, 1, mode=bbc.QUERY_STAGED, host_stats=True)
    sub = torch.as_tensor(S.receiver_points(sc, 128), device=dev)
    ex, _ = B.query(sub, 1, 0, mode=bbc.QUERY_STAGED | bbc.QUERY_EXHAUSTIVE)
    est, _ = B.query(sub, 64, 7, mode=bbc.QUERY_STAGED)
    ex, est = ex.double().cpu().numpy(), est.double().cpu().numpy()
    lit = ex > 0
    relmse = float(np.mean(((est[lit] - ex[lit]) / ex[lit]) ** 2)) if lit.any() else None
    info = B.info()
    B.free()
    n = pts.shape[1]
    b, q = float(np.median(tb)), float(np.median(tq))
    return {"workload": "single refraction, water surface 524288 triangles x 4 lights (amplitudes x 0.04), "
                        "depth cap 6, 1024x1024 floor points, 64 samples/point",
            "irradiance_bound": "implicit differentiation" if flags & bbc.FLAG_IMPLICIT_IRR else "explicit",
            "relmse_vs_exhaustive_128x128": relmse,
            "queries_s_whole_step": round(n / (b + q), 1), "build_ms": round(1e3 * b, 2),
            "query_ms": round(1e3 * q, 2), "query_only_queries_s": round(n / q, 1),
            "first_build_ms": round(1e3 * first_build, 1),
            "tuples": info["n_tuples"], "live_tuples": info["n_live_tuples"], "boxes": info["n_boxes"],
            "leaves": info["n_leaves"], "grid_entries": info["n_grid_entries"], "inf_leaves": info["n_inf_leaves"],
            "device_bytes": info["device_bytes"], "pairs": qs["n_pairs"], "roots": qs["n_roots"]}


def area_light_section(bbc, S, torch, steps=3):
    """Single reflection off a 65 x 65-vertex heightfield (8192 triangles) lit
    by a 0.4 x 0.4 area light centred where the point light sits, depth cap 3
    (a box's receiver footprint cannot shrink below the light's image, so
    subdivision runs to the cap), 512 x 512 receiver points, 64 samples per
    point (one light point per selected pair): build and query timed
    separately (inputs resident in device memory)."""
    dev = torch.device("cuda:0")
    sc = S.area_light(S.heightfield_mirror(64), [0.4, 0.0, 0.0], [0.0, 0.4, 0.0])
    params = dict(max_depth=3, sigma=1e-4, alpha=2.0, grid_res=512)
    t0 = time.perf_counter()
    B = bbc.Bounds(bbc.DeviceScene(sc), params)
    torch.cuda.synchronize()
    first_build = time.perf_counter() - t0
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
    _, _, qs = B.query(pts, 64, 1, mode=bbc.QUERY_STAGED, host_stats=True)
    info = B.info()
    B.free()
    n = pts.shape[1]
    b, q = float(np.median(tb)), float(np.median(tq))
    return {"workload": "single reflection, heightfield 8192 triangles, 0.4 x 0.4 area light, depth cap 3, "
                        "512x512 receiver points, 64 samples/point",
            "queries_s_whole_step": round(n / (b + q), 1), "build_ms": round(1e3 * b, 2),
            "query_ms": round(1e3 * q, 2), "query_only_queries_s": round(n / q, 1),
            "first_build_ms": round(1e3 * first_build, 1),
            "live_tuples": info["n_live_tuples"], "boxes": info["n_boxes"], "leaves": info["n_leaves"],
            "inf_leaves": info["n_inf_leaves"], "grid_entries": info["n_grid_entries"],
            "pairs": qs["n_pairs"], "roots": qs["n_roots"]}


def two_reflection_section(bbc, S, torch, steps=2):
    """Two reflections between two facing rippled walls (8192 triangles each,
    67,108,864 candidate pairs), depth cap 2, alpha 10, 256 x 256 floor points,
    256 samples per point: tuple construction + build and query timed."""
    dev = torch.device("cuda:0")
    sc = S.facing_walls(64)
    params = dict(max_depth=2, sigma=1e-4, alpha=10.0, grid_res=512)
    t0 = time.perf_counter()
    B = bbc.Bounds(bbc.DeviceScene(sc), params)
    torch.cuda.synchronize()
    first_build = time.perf_counter() - t0
    pts = torch.as_tensor(S.receiver_points(sc, 256), device=dev)
    tb, tq = [], []
    for k in range(steps):
        t = time.perf_counter()
        B.rebuild()
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t)
        t = time.perf_counter()
        B.query(pts, 256, 1 + k, mode=bbc.QUERY_STAGED)
        torch.cuda.synchronize()
        tq.append(time.perf_counter() - t)
    _, _, qs = B.query(pts, 256, 1, mode=bbc.QUERY_STAGED, host_stats=True)
    info = B.info()
    B.free()
    n = pts.shape[1]
    b, q = float(np.median(tb)), float(np.median(tq))
    return {"workload": "two reflections, facing walls 8192 + 8192 triangles (67.1M candidate pairs), depth cap 2, "
                        "256x256 floor points, 256 samples/point",
            "queries_s_whole_step": round(n / (b + q), 1), "build_ms": round(1e3 * b, 2),
            "query_ms": round(1e3 * q, 2), "first_build_ms": round(1e3 * first_build, 1),
            "candidate_pairs": info["n_tuples"], "live_tuples": info["n_live_tuples"], "boxes": info["n_boxes"],
            "leaves": info["n_leaves"], "grid_entries": info["n_grid_entries"], "device_bytes": info["device_bytes"],
            "mean_candidates_per_point": round(qs["sum_U"] / n, 1), "roots": qs["n_roots"]}


def samplers_section(bbc, torch, B, pts, spps=(4, 16), seeds=4, reps=5):
    """The sampling schemes side by side on the benchmark bounds (the paper's
    sampling-scheme comparison): RelMSE against the exhaustive sum over U at
    equal expected samples per point W (below the typical |U| of ~16, where
    the schemes differ), the staged query time, and samples and roots per
    point."""
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


def serving_section(bbc, S, torch, sphere_scene, sphere_bounds, n_req=1500, seed=5):
    """Continuous batching vs the plain per-request path on one request
    stream over device-resident bounds: the displaced sphere and a rippled
    plane mirror of 131072 triangles (256 x 256 heightfield)."""
    dev = torch.device("cuda:0")
    pool = S.heightfield_mirror(256)
    pool_B = bbc.Bounds(bbc.DeviceScene(pool), dict(max_depth=6, sigma=1e-4, alpha=2.0, grid_res=512))
    scenes = [sphere_scene, pool]
    bounds = [sphere_bounds, pool_B]
    pools = [torch.as_tensor(S.random_points(sc, 65536, seed=77 + j), device=dev) for j, sc in enumerate(scenes)]
    trace = make_trace(n_req, len(scenes), seed)
    reqs = [pools[r["scene"]][:, r["off"]:r["off"] + r["n"]].contiguous() for r in trace]
    n_pts = sum(r["n"] for r in trace)
    outs = [torch.empty(r["n"], dtype=torch.float32, device=dev) for r in trace]
    torch.cuda.synchronize()
    run_plain(bbc, torch, bounds, reqs, trace[:50], outs)  # warm-up
    t_plain, _ = run_plain(bbc, torch, bounds, reqs, trace, outs)
    cap_req = n_req / t_plain
    srv = bbc.Server(bounds, hbm_budget_bytes=64 << 30, max_inflight=4, max_batch_points=1 << 20,
                     max_batch_requests=1024, queue_capacity=1 << 16)
    try:
        run_served(bbc, srv, reqs, trace[:50])  # warm-up
        srv.stats(reset=True)
        t_srv, _, got = run_served(bbc, srv, reqs, trace)
        identical = all(torch.equal(g, o) for g, o in zip(got, outs))
        st_cap = srv.stats(reset=True)
        rng = np.random.default_rng(seed + 1)
        sweep = []
        for x in (0.5, 0.8, 1.0, 1.2, 2.0, 3.0):
            rate = x * cap_req
            arr = np.cumsum(rng.exponential(1.0 / rate, n_req))
            tp, lp = run_plain(bbc, torch, bounds, reqs, trace, outs, arrivals=arr)
            ts, ls, _ = run_served(bbc, srv, reqs, trace, arrivals=arr)
            st = srv.stats(reset=True)
            sweep.append({"rate_x_plain_capacity": x, "offered_req_s": round(rate, 1),
                          "plain": {"queries_s": round(n_pts / tp, 1), "p50_ms": round(float(np.percentile(lp, 50)), 3),
                                    "p99_ms": round(float(np.percentile(lp, 99)), 3)},
                          "served": {"queries_s": round(n_pts / ts, 1), "p50_ms": round(float(np.percentile(ls, 50)), 3),
                                     "p99_ms": round(float(np.percentile(ls, 99)), 3),
                                     "mean_batch_requests": round(st["mean_batch_requests"], 2)}})
    finally:
        srv.close()
        pool_B.free()
    return {
        "scenes": [sphere_scene["name"] if "name" in sphere_scene else "sphere", pool["name"]],
        "requests": n_req, "points": int(n_pts), "inputs": "device-resident points and outputs",
        "saturated": {"plain_queries_s": round(n_pts / t_plain, 1), "served_queries_s": round(n_pts / t_srv, 1),
                      "speedup": round(t_plain / t_srv, 3), "plain_req_s": round(cap_req, 1),
                      "served_req_s": round(n_req / t_srv, 1),
                      "mean_batch_requests": round(st_cap["mean_batch_requests"], 2),
                      "inflight_peak": st_cap["inflight_peak"]},
        "results_identical_to_plain": bool(identical),
        "poisson": sweep,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--form", choices=["auto", "fused", "staged"], default="auto")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-refraction", action="store_true")
    ap.add_argument("--no-two-reflections", action="store_true")
    ap.add_argument("--no-samplers", action="store_true")
    ap.add_argument("--no-area-light", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 256 MiB device-to-device tensor copy first (reference kernel for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (see DESIGN.md for how the "
              "method would shard); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2504_19163_amd import bbc, scenes as S

    if not os.path.exists(bbc.LIB_PATH):
        from paper_2504_19163_amd import build_lib
        build_lib.build()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    scene = S.displaced_sphere(7)
    params = dict(max_depth=8, sigma=1e-4, alpha=2.0, grid_res=512)
    spp = 64
    pts_np = S.receiver_points(scene, 512)
    pts = torch.as_tensor(pts_np, device=dev)
    n = pts.shape[1]
    ds = bbc.DeviceScene(scene)
    B = bbc.Bounds(ds, params)
    tuned = bbc.apply_tuning(B, "sphere131072_r")
    forms = {"fused": bbc.QUERY_FUSED, "staged": bbc.QUERY_STAGED}
    if args.form == "auto":
        form = tuned.get("form", "staged")
    else:
        form = args.form
    mode = forms[form]
    B.set_tuning(bbc.TUNE_TIMING, 1)
    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step(k):
        B.rebuild()
        E, _ = B.query(pts, spp, k, mode=mode)
        return E

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()

    step_ms, kern_ms = [], []
    t0 = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        E = step(1000 + k)
        kern_ms.append(B.kernel_ms())  # waits for the query's end event
        torch.cuda.synchronize()
        step_ms.append(1e3 * (time.perf_counter() - ts))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    total_s = t1 - t0
    value = n * args.steps / total_s

    # work counts of one query launch (same seeds, separate untimed call)
    _, _, qs = B.query(pts, spp, 1000, mode=mode, host_stats=True)
    evals = qs["n_iter_fp32"] + qs["n_iter_fp64"]
    kms = float(np.median(kern_ms))
    achieved = evals * FLOPS_PER_PATH_EVAL / (kms * 1e-3) / 1e12
    info = B.info()

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * total_s / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32+fp64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "triangles": int(scene["pos"].shape[1]), "shading_points": int(n),
                   "spp": spp, "depth_cap": params["max_depth"], "grid": params["grid_res"], "query_form": form,
                   "parallelism": "single GPU"},
        "latency_ms": {"p50": round(float(np.percentile(step_ms, 50)), 4),
                       "p99": round(float(np.percentile(step_ms, 99)), 4)},
        "roofline": {"bound": "alu", "kernel": "query (fused kernel)" if form == "fused" else "query Newton kernel",
                     "achieved": round(achieved, 4), "peak": round(PEAK_VALU_TFLOPS, 1), "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_VALU_TFLOPS, 5),
                     "traffic": newton_traffic_bytes() if form == "staged" else None, "traffic_unit": "HBM bytes per launch",
                     "kernel_ms": round(kms, 4), "path_evals": int(evals)},
        "work": {"leaves": info["n_leaves"], "grid_entries": info["n_grid_entries"], "pairs": qs["n_pairs"],
                 "newton_starts": qs["n_newton"], "roots": qs["n_roots"]},
    }

    if not args.no_samplers:
        out["samplers"] = samplers_section(bbc, torch, B, pts)
    if not args.no_serving:
        out["serving"] = serving_section(bbc, S, torch, scene, B)
    if not args.no_refraction:
        out["refraction"] = refraction_section(bbc, S, torch)
        out["refraction_implicit"] = refraction_section(bbc, S, torch, steps=2, flags=bbc.FLAG_IMPLICIT_IRR)
    if not args.no_two_reflections:
        out["two_reflections"] = two_reflection_section(bbc, S, torch)
    if not args.no_area_light:
        out["area_light"] = area_light_section(bbc, S, torch)

    if not args.no_cpu_baseline:
        from oracle import oracle as O
        cores = cpu_cores()
        osc = O.OracleScene(scene)
        tb = time.perf_counter()
        ob = O.OracleBuild(osc, params, n_threads=cores)
        t_build = time.perf_counter() - tb
        tq = time.perf_counter()
        OE, _ = ob.query(pts_np, spp, 1000 + args.steps - 1, mode=0, n_threads=cores)
        t_query = time.perf_counter() - tq
        out["cpu_baseline"] = {"value": round(n / (t_build + t_query), 1), "unit": "queries/s", "cores": cores,
                               "kind": "oracle",
                               "sample": f"full workload: FP64 oracle build ({t_build:.2f} s) + query of all {n} "
                                         f"points ({t_query:.2f} s), one step"}
        # matched error: the GPU estimate and the oracle's estimate with the same
        # seed against the oracle's exhaustive sum on a fixed subset of points
        sub = np.arange(0, n, 61)
        ex, _ = ob.query(pts_np[:, sub], spp, 0, mode=1, n_threads=cores)
        Eg = E.cpu().numpy().astype(np.float64)[sub]
        out["matched_error"] = {"relmse_gpu_vs_exhaustive": relmse(Eg, ex),
                                "relmse_oracle_vs_exhaustive": relmse(OE[sub], ex),
                                "points": int(len(sub))}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
