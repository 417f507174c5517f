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


def cpu_cores():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def relmse(est, ref):
    return float(np.mean((est - ref) ** 2 / (ref ** 2 + 1e-2)))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--form", choices=["auto", "fused", "staged"], default="auto")
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
                     "frac": round(achieved / PEAK_VALU_TFLOPS, 5), "traffic": None,
                     "kernel_ms": round(kms, 4), "path_evals": int(evals)},
        "work": {"leaves": info["n_leaves"], "grid_entries": info["n_grid_entries"], "pairs": qs["n_pairs"],
                 "newton_starts": qs["n_newton"], "roots": qs["n_roots"]},
    }

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
