"""Autotuner of the library's launch-shape knobs (bbc_set_tuning) on the GPU
it runs on.

For each workload (the bench's three resident scenes) it builds the bound
hierarchy, then tunes one knob at a time (coordinate descent, the other knobs
at their best value so far), timing each candidate value on a fixed set of
requests shaped like the serving stream (log-uniform sizes in [256, 65536],
W over {16, ..., 256}) through the staged query, median of three passes; the
build knobs (workgroups per compute unit, graph replay) are timed on
rebuilds.  Knobs change launch shapes only, never
results (the library's tests check that), so the choice is free.  The table
is written as JSON {arch: {workload: {knob: value, "ms": {...}}}}, by default
to tuning.json beside this module, where bbc.apply_tuning reads it; the entry
"serving" holds the server's graph flag, timed on a mixed request stream.

    python -m paper_2504_19163_amd.autotune [--out PATH] [--workloads sphere131072,...]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# workload key -> (scene factory, build parameters)
WORKLOADS = {
    "sphere131072": (lambda S: S.displaced_sphere(7), dict(max_depth=8, alpha=2.0)),
    "water512x512": (lambda S: S.water_surface(m=512, amp_scale=0.04), dict(max_depth=6, alpha=2.0)),
    "walls64x64": (lambda S: S.facing_walls(64), dict(max_depth=6, alpha=10.0)),
}

# staged-query knobs in tuning order, with their candidate values
QUERY_KNOBS = [
    ("newton_steps", "TUNE_NEWTON_STEPS", [1, 2, 4, 8]),
    ("newton_grid_per_cu", "TUNE_NEWTON_GRID_PER_CU", [0, 8, 12, 16]),
    ("graph", "TUNE_GRAPH", [0, 1]),
]
FUSED_KNOBS = [
    ("query_waves", "TUNE_QUERY_WAVES", [2, 4]),
    ("query_tile", "TUNE_QUERY_TILE", [16, 32, 64]),
    ("query_grid", "TUNE_QUERY_GRID", [4096, 16384, 65536]),
]
BUILD_KNOBS = [("build_grid_per_cu", "TUNE_BUILD_GRID_PER_CU", [0, 4, 8, 16]), ("build_graph", "TUNE_BUILD_GRAPH", [0, 1])]


def _requests(scene, n_req, seed, torch, S):
    rng = np.random.default_rng(seed)
    sizes = np.floor(np.exp(rng.uniform(np.log(256), np.log(65536), n_req))).astype(np.int64)
    pool = torch.as_tensor(S.random_points(scene, 65536, seed=seed), device="cuda:0")
    out = []
    for k in range(n_req):
        n = int(sizes[k])
        o = int(rng.integers(0, 65536 - n + 1))
        out.append((pool[:, o:o + n].contiguous(), int(rng.choice([16, 32, 64, 128, 256])), int(rng.integers(0, 2**62))))
    return out


def _time_queries(bbc, torch, B, reqs, mode, reps=3):
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for pts, spp, seed in reqs:
            B.query(pts, spp, seed, mode=mode)
        torch.cuda.synchronize()
        ts.append(1e3 * (time.perf_counter() - t0))
    return float(np.median(ts))


def _time_rebuild(torch, B, reps=3):
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.rebuild()
        torch.cuda.synchronize()
        ts.append(1e3 * (time.perf_counter() - t0))
    return float(np.median(ts))


def tune_workload(bbc, torch, S, key, n_req=24, log=print):
    make, params = WORKLOADS[key]
    scene = make(S)
    B = bbc.Bounds(bbc.DeviceScene(scene), params)
    reqs = _requests(scene, n_req, 11, torch, S)
    best, ms = {}, {}
    staged = bbc.QUERY_STAGED
    _time_queries(bbc, torch, B, reqs[:4], staged, reps=1)  # warm-up
    for name, knob, values in QUERY_KNOBS:
        row = {}
        for v in values:
            B.set_tuning(getattr(bbc, knob), v)
            row[v] = _time_queries(bbc, torch, B, reqs, staged)
            log(f"{key} {name}={v}: {row[v]:.3f} ms")
        best[name] = min(row, key=row.get)
        ms[name] = {str(k): round(t, 3) for k, t in row.items()}
        B.set_tuning(getattr(bbc, knob), best[name])
    small = [r for r in reqs if r[0].shape[1] <= 16384][:8] or reqs[:4]
    for name, knob, values in FUSED_KNOBS:
        row = {}
        for v in values:
            B.set_tuning(getattr(bbc, knob), v)
            row[v] = _time_queries(bbc, torch, B, small, bbc.QUERY_FUSED)
            log(f"{key} fused {name}={v}: {row[v]:.3f} ms")
        best[name] = min(row, key=row.get)
        ms[name] = {str(k): round(t, 3) for k, t in row.items()}
        B.set_tuning(getattr(bbc, knob), best[name])
    for name, knob, values in BUILD_KNOBS:
        row = {}
        for v in values:
            B.set_tuning(getattr(bbc, knob), v)
            row[v] = _time_rebuild(torch, B)
            log(f"{key} {name}={v}: {row[v]:.3f} ms (rebuild)")
        best[name] = min(row, key=row.get)
        ms[name] = {str(k): round(t, 3) for k, t in row.items()}
        B.set_tuning(getattr(bbc, knob), best[name])
    B.free()
    return dict(best, ms=ms, requests=n_req)


def tune_serving(bbc, torch, S, table_arch, n_req=96, log=print):
    """The server's graph flag: one stream of requests over the three
    workloads' bounds (tuned knobs applied), all submitted at once, served with
    and without BBC_SERVER_GRAPH; median of three passes."""
    bounds, pools = [], []
    for j, key in enumerate(WORKLOADS):
        make, params = WORKLOADS[key]
        scene = make(S)
        B = bbc.Bounds(bbc.DeviceScene(scene), params)
        for knob, name in (("TUNE_NEWTON_STEPS", "newton_steps"), ("TUNE_NEWTON_GRID_PER_CU", "newton_grid_per_cu"),
                           ("TUNE_GRAPH", "graph")):
            if name in table_arch.get(key, {}):
                B.set_tuning(getattr(bbc, knob), table_arch[key][name])
        bounds.append(B)
        pools.append(torch.as_tensor(S.random_points(scene, 65536, seed=30 + j), device="cuda:0"))
    rng = np.random.default_rng(5)
    reqs = []
    for k in range(n_req):
        n = int(np.floor(np.exp(rng.uniform(np.log(256), np.log(65536)))))
        sc = int(rng.integers(0, len(bounds)))
        o = int(rng.integers(0, 65536 - n + 1))
        reqs.append((sc, pools[sc][:, o:o + n].contiguous(), int(rng.choice([16, 32, 64, 128, 256])),
                     int(rng.integers(0, 2**62))))
    row = {}
    for g in (0, 1):
        srv = bbc.Server(bounds, hbm_budget_bytes=64 << 30, max_inflight=4, max_batch_points=1 << 20,
                         max_batch_requests=1024, queue_capacity=1 << 16, graph=bool(g))
        ts = []
        for rep in range(4):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            tickets = [srv.submit(sc, p, spp, seed, sync_inputs=False) for sc, p, spp, seed in reqs]
            for t in tickets:
                srv.wait(t)
            if rep:
                ts.append(1e3 * (time.perf_counter() - t0))
        srv.close()
        row[g] = float(np.median(ts))
        log(f"serving graph={g}: {row[g]:.3f} ms")
    for B in bounds:
        B.free()
    best = min(row, key=row.get)
    return {"graph": best, "ms": {str(k): round(t, 3) for k, t in row.items()}, "requests": n_req}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default=os.path.join(HERE, "tuning.json"))
    ap.add_argument("--workloads", default=",".join(WORKLOADS))
    ap.add_argument("--requests", type=int, default=24)
    ap.add_argument("--no-serving", action="store_true", help="skip the server's graph flag")
    args = ap.parse_args()
    import torch
    from paper_2504_19163_amd import bbc, scenes as S
    bbc.lib()
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    table = {}
    if os.path.exists(args.out):
        with open(args.out) as f:
            table = json.load(f)
    for key in args.workloads.split(","):
        table.setdefault(arch, {})[key] = tune_workload(bbc, torch, S, key, n_req=args.requests,
                                                        log=lambda m: print(m, flush=True))
        with open(args.out, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    if not args.no_serving:
        table[arch]["serving"] = tune_serving(bbc, torch, S, table[arch], log=lambda m: print(m, flush=True))
        with open(args.out, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    print(json.dumps(table[arch]), flush=True)


if __name__ == "__main__":
    main()
