"""Benchmark of the NEAREST time-step hot path on one MI355X.

Workload: 25 undulating filaments (N = 1000 force points, Q = 10000
quadrature points, n = 3150 unknowns), classical RK4 with dt = 2 pi / 100.
One step = four solves, each = geometry + nearest map + fused assembly +
rigid-body blocks + LU + triangular solves (+ FP64 refinement).  The metric
is time-step solves per second at <= 1e-8 relative force error against the
FP64 oracle (checked on the final state).

python bench.py [--gpus 1] [--steps K] [--warmup W] [--method fp32_ir|fp64_lu|fp32_gepp_ir]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METHODS = {"fp64_lu": 0, "fp32_ir": 1, "fp32_gepp_ir": 2}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=25)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--method", default="fp32_ir", choices=sorted(METHODS))
    ap.add_argument("--swimmers", type=int, default=25)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_2001_06468_amd as nrs

    dev = "cuda:0"
    M = args.swimmers
    scene = synth.filament_scene(M, seed=0)
    ds = nrs.DeviceScene(scene, dev)
    ctx = nrs.Context(0)
    method = METHODS[args.method]
    ws = torch.empty(nrs.nrs_rk4_workspace_size(ctx, ds, method), dtype=torch.uint8, device=dev)
    Y = torch.from_numpy(scene["Y0"].copy()).to(dev)
    dt = 2 * math.pi / 100
    t = 0.0
    for _ in range(args.warmup):
        nrs.nrs_rk4_step(ctx, ds, Y, t, dt, ws, method=method)
        t += dt
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        nrs.nrs_rk4_step(ctx, ds, Y, t, dt, ws, method=method)
        t += dt
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = e0.elapsed_time(e1)
    info = nrs.nrs_query_info(ctx, ws)
    solves = 4 * args.steps
    out = {
        "metric": "time-step solves/sec (assemble+solve) at <=1e-8 rel force err",
        "value": solves / (ms / 1e3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "wall_s": wall,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if method else "f64",
        "data": "synthetic",
        "config": {"workload": f"filaments_M{M}_rk4", "N": scene["N"], "Q": scene["Q"],
                   "n": 3 * scene["N"] + 6 * M, "method": args.method, "dt": dt},
        "last_step_info": info,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
