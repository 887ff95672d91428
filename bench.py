"""Benchmark of the NEAREST time-step hot path on one MI355X.

Workload (the time-stepping configuration): 25 undulating filaments of unit
length (N = 1000 force points, Q = 10000 quadrature points, n = 3150
unknowns), eps = 0.01, classical RK4 with dt = 2 pi / 100 from the seeded
initial state.  One step = four solves; each solve = geometry + nearest map
+ fused assembly + rigid-body blocks + LU + triangular solves + FP64
refinement (method fp32_ir).  The metric is time-step solves per second;
a synchronous solve of the seeded initial state is checked against the FP64
oracle (relative force error <= 1e-8) in the CPU leg.

Printed as one JSON line; `roofline` describes the dominant kernel (the
single-launch tile LU), timed here with HIP events around its own launch on
the benchmark matrix; `cpu_baseline` is the CPU oracle on a bounded sample
(the only part of this script that runs the oracle).  `field` is the flow at
806 tracers of a 10-swimmer channel (nrs_field_velocity) and the tracer RK4
step, with its own roofline and oracle sample.

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
PEAK_FP32_TFLOPS = 157.3      # MI355X dense FP32 (vector and matrix)
PEAK_FP64_TFLOPS = 78.6
# HBM bytes per launch of the tile LU at n = 3150 from the FETCH_SIZE and
# WRITE_SIZE counter runs (calibrated against a 256 MiB copy), valid only for
# the kernel source they were taken on (first 16 hex digits of its SHA-256).
LU_TRAFFIC = {"source_sha256_16": "ac86c9aaff497af9", "bytes_per_launch": 909496904, "n": 3150}
# HBM bytes per nrs_field_velocity call (sources + pair sum + chunk sum) on the
# tracer workload, from the same two counter runs, valid for that field.hip.
FIELD_TRAFFIC = {"source_sha256_16": "7f18d8d2f998ad7c", "bytes_per_call": 24459390, "Q": 73248,
                 "tracers": 806}


# Counter-derived figures (rocprofv3 --pmc runs of this benchmark, each counter
# scaled by what it reads for a kernel of known work run in the same
# process), valid only for the kernel source they were taken on.
COUNTERS = {
    "lu": {"source": "lu_tiles.hip", "source_sha256_16": "ac86c9aaff497af9", "n": 3150,
           "mfma_flops_per_launch": 2.202e10, "mfma_busy": 0.093,
           "calibration": "FP32 4096^3 matrix product: 0.954 busy at 150 TFLOP/s"},
    "assembly": {"source": "assemble.hip", "source_sha256_16": "cd14792605c821f9", "N": 1000,
                 "Q": 10000, "valu_fp32_flops_per_call": 4.061e8,
                 "fp32_rsqrt_per_call": 1.05e7, "valu_fp64_flops_per_call": 6.517e8,
                 "fp64_transcendental_per_call": 2.05e7,
                 "calibration": "elementwise multiplies of 2^26 elements read 2^20: x 64"},
}


def counter_summary(which, cur_sha=None):
    rec = COUNTERS.get(which)
    if rec is None:
        return None
    src = os.path.join(ROOT, "paper_2001_06468_amd", "csrc", rec["source"])
    import hashlib
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if sha != rec["source_sha256_16"]:
        return None
    return {k: v for k, v in rec.items() if k not in ("source", "source_sha256_16")}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_dgemm_gflops(nsz=2048, reps=3):
    """Host FP64 matrix-product rate (NumPy/BLAS), the CPU roofline figure."""
    import numpy as np
    a = np.random.default_rng(0).normal(size=(nsz, nsz))
    a @ a
    t0 = time.perf_counter()
    for _ in range(reps):
        a @ a
    return 2.0 * nsz ** 3 * reps / (time.perf_counter() - t0) / 1e9


def cpu_threads():
    try:
        from threadpoolctl import threadpool_info
        n = [p.get("num_threads", 0) for p in threadpool_info() if p.get("user_api") == "blas"]
        if n:
            return int(max(n))
    except Exception:
        pass
    return os.cpu_count() or 1


def train_model(ctx, nrs, solves=20000, steps=8000):
    """Warm-start network for the GMRES form: training data are solves of the
    method on seeded filament swimmers (random phases, times, M in {1,5,25}),
    fitted with the library's own forward/backward/Adam kernels."""
    import torch
    from paper_2001_06468_amd import learned
    t0 = time.perf_counter()
    states = learned.filament_states(solves, seed0=1000, m_choices=(1, 5, 25),
                                     m_probs=(0.7, 0.25, 0.05))
    data = learned.build_targets(ctx, learned.generate(ctx, states, batch=128))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    model, hist = learned.train(ctx, data, steps=steps, batch_bodies=256, lr=5e-3, lr_final=3e-5,
                                seed=0, log_every=steps)
    t2 = time.perf_counter()
    return model, {"solves": solves, "bodies": data.n_bodies, "generate_s": t1 - t0,
                   "train_s": t2 - t1, "adam_steps": steps, "batch_bodies": 256,
                   "final_loss": hist[-1]["loss"], "params": int(model.theta.numel())}


def device_problem(ctx, nrs, ds, scene, t, Y, dev):
    """Geometry and nearest map of a scene state on the GPU (nrs_geometry,
    nrs_nearest): the Problem and the prescribed velocities u [3N]."""
    import torch
    N, Q = scene["N"], scene["Q"]
    x = torch.empty((3, N), dtype=torch.float64, device=dev)
    X = torch.empty((3, Q), dtype=torch.float64, device=dev)
    w = torch.empty(Q, dtype=torch.float64, device=dev)
    u = torch.empty(3 * N, dtype=torch.float64, device=dev)
    nrs.nrs_geometry(ctx, ds, t, Y, x, X, w, u)
    nu = torch.empty(Q, dtype=torch.int32, device=dev)
    nrs.nrs_nearest(ctx, x, scene["group_off"], X, ds.t["groupX"], nu)
    return nrs.Problem(x, X, w, nu, ds.t["body"], Y, scene["eps"], scene["mu"]), u


FIELD_FLOPS_PER_PAIR = 32.0


def field_workload(synth):
    """Tracer workload: 10 sperm-like swimmers in the 4 x 1 x 0.5 channel
    (wall spacing 1/16: N = 4728 force and Q = 73248 quadrature points) and
    806 tracers on a 26 x 31 grid in the channel mid-plane."""
    scene = synth.sperm_channel_scene(10, h=1.0 / 16, seed=0)
    y = synth.tracer_grid(26, 31, (-1.9, 1.9), (-0.45, 0.45), 0.0)
    return scene, y


def run_field(ctx, nrs, synth, dev, reps=40):
    """Flow at the tracers (nrs_field_velocity: source gather, pair sum,
    chunk sum) with seeded force densities, timed with HIP events on the
    context's stream; then RK4 steps of the tracers through three
    precomputed flows (geometry at t, t + dt/2, t + dt)."""
    import numpy as np
    import torch
    scene, yh = field_workload(synth)
    N, Q, P = scene["N"], scene["Q"], yh.shape[1]
    ds = nrs.DeviceScene(scene, dev)
    Y = torch.from_numpy(scene["Y0"].copy()).to(dev)
    rng = np.random.default_rng(7)
    flows, fs = [], []
    dt = 2 * math.pi / 100
    for k, t in enumerate((0.0, 0.5 * dt, dt)):
        pb, _ = device_problem(ctx, nrs, ds, scene, t, Y, dev)
        flows.append(pb)
        fs.append(torch.from_numpy(rng.normal(size=(3, N))).to(dev))
    y = torch.from_numpy(yh).to(dev)
    u = torch.empty((3, P), dtype=torch.float64, device=dev)
    ws = torch.empty(nrs.nrs_field_workspace_size(ctx, P, Q), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(3):
        nrs.nrs_field_velocity(ctx, flows[0], fs[0], y, u, ws)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        nrs.nrs_field_velocity(ctx, flows[0], fs[0], y, u, ws)
    e1.record(stream)
    torch.cuda.synchronize()
    call_ms = e0.elapsed_time(e1) / reps
    pairs = float(P) * Q
    tflops = FIELD_FLOPS_PER_PAIR * pairs / (call_ms / 1e3) / 1e12
    import hashlib
    fsrc = os.path.join(ROOT, "paper_2001_06468_amd", "csrc", "field.hip")
    fh = hashlib.sha256(open(fsrc, "rb").read()).hexdigest()[:16]
    traffic = (FIELD_TRAFFIC["bytes_per_call"]
               if fh == FIELD_TRAFFIC["source_sha256_16"] and Q == FIELD_TRAFFIC["Q"]
               and P == FIELD_TRAFFIC["tracers"] else None)
    yt = y.clone()
    nrs.nrs_tracer_rk4_step(ctx, flows, fs, yt, dt, ws)
    torch.cuda.synchronize()
    ksteps = 10
    e0.record(stream)
    for _ in range(ksteps):
        nrs.nrs_tracer_rk4_step(ctx, flows, fs, yt, dt, ws)
    e1.record(stream)
    torch.cuda.synchronize()
    step_ms = e0.elapsed_time(e1) / ksteps
    return {"workload": f"sperm_K10_h16_tracers{P}", "tracers": P, "N": N, "Q": Q,
            "pairs_per_call": pairs, "ms_per_call": call_ms, "pairs_per_s": pairs / (call_ms / 1e3),
            "roofline": {"kernel": "nrs_field_velocity (k_field_sources + k_field_part + "
                                   "k_field_sum)", "bound": "alu", "achieved": tflops,
                         "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                         "frac": tflops / PEAK_FP64_TFLOPS, "traffic": traffic,
                         "flops_per_pair": FIELD_FLOPS_PER_PAIR},
            "tracer_rk4_ms_per_step": step_ms, "tracer_rk4_steps_per_s": 1e3 / step_ms,
            "note": "FP64; flops counted as 32 per (tracer, quadrature point) pair with the "
                    "reciprocal square root as one; the call time includes the gather of "
                    "w_q f[nu(q)] and the fixed-order chunk sum"}


def run_channel(ctx, nrs, synth, dev, sizes=((10, 16), (40, 24))):
    """Channel configuration (10 and 40 sperm-like swimmers in the 4 x 1 x 0.5
    channel, wall spacing 1/16 and 1/24, n = 14,244 and 39,504): one
    synchronous solve each with the GMRES-IR forms (and, at K = 10, the FP64
    partial-pivoting form) after a warm-up solve, and
    the tile LU alone (FP32 updates, and BF16-input updates) timed with HIP
    events.  Geometry and nearest map on the GPU."""
    import torch
    out = []
    for K, h in sizes:
        sc = synth.sperm_channel_scene(K, h=1.0 / h, seed=0)
        ds = nrs.DeviceScene(sc, dev)
        Y = torch.from_numpy(sc["Y0"].copy()).to(dev)
        pb, u = device_problem(ctx, nrs, ds, sc, 0.0, Y, dev)
        n = pb.n
        rec = {"workload": f"sperm_K{K}_h{h}", "N": pb.N, "Q": pb.Q, "n": n, "solves": {}}
        methods = [("fp32_gmres_ir", nrs.NRS_FP32_GMRES_IR)]
        if K == 10:
            # and the plain FP64 form (partial pivoting) as the reference rate
            methods += [("bf16_gmres_ir", nrs.NRS_BF16_GMRES_IR), ("fp64_lu", nrs.NRS_FP64_LU)]
        wsz = max(nrs.nrs_workspace_size(ctx, pb.N, pb.Q, pb.M, m) for _, m in methods)
        ws = torch.empty(wsz, dtype=torch.uint8, device=dev)
        sol = torch.empty(n, dtype=torch.float64, device=dev)
        for name, m in methods:
            nrs.nrs_solve(ctx, pb, u, None, sol, ws, method=m)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = nrs.nrs_solve(ctx, pb, u, None, sol, ws, method=m)
            wall = time.perf_counter() - t0
            rec["solves"][name] = {"ms": 1e3 * wall, "iterations": info["iterations"],
                                   "fell_back": info["fell_back"],
                                   "backward_error": info["backward_error"]}
        del ws
        lda = nrs.lda_for(n)
        A32 = torch.empty((n, lda), dtype=torch.float32, device=dev)
        wa = torch.empty(nrs.nrs_workspace_size(ctx, pb.N, pb.Q, pb.M, nrs.NRS_FP32_IR),
                         dtype=torch.uint8, device=dev)
        nrs.nrs_assemble(ctx, pb, 32, A32, lda, wa)
        del wa
        A0 = A32.clone()
        ipiv = torch.empty(n, dtype=torch.int32, device=dev)
        perm = torch.empty(n, dtype=torch.int32, device=dev)
        sing = torch.zeros(1, dtype=torch.int32, device=dev)
        for name, bf in (("lu_fp32", False), ("lu_bf16_updates", True)):
            A32.copy_(A0)
            wl = torch.empty(nrs.nrs_lu_factor_workspace_size(ctx, n, 16 if bf else 32),
                             dtype=torch.uint8, device=dev)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            nrs.nrs_lu_factor(ctx, A32, lda, ipiv, perm, sing, wl, pivot_scope=1, bf16_updates=bf)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            rec[name] = {"ms": ms, "tflops": 2.0 / 3.0 * n ** 3 / (ms / 1e3) / 1e12}
        del A32, A0
        torch.cuda.empty_cache()
        out.append(rec)
    return out


def run_dopri(ctx, nrs, ds, scene, dev, method, t1=2 * math.pi / 10, rtol=1e-6, atol=1e-9):
    """Adaptive Dormand-Prince 5(4) over a tenth of a beat period of the same
    25-filament workload (first step 2 pi / 100, the RK4 step): attempts,
    solves and solves per second of the whole integration (HIP events)."""
    import torch
    ws = torch.empty(nrs.nrs_dopri5_workspace_size(ctx, ds, method), dtype=torch.uint8,
                     device=dev)
    Y = torch.from_numpy(scene["Y0"].copy()).to(dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    st = nrs.nrs_dopri5_integrate(ctx, ds, Y, 0.0, t1, 2 * math.pi / 100, rtol, atol, ws,
                                  method=method)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    return {"t1": t1, "rtol": rtol, "atol": atol, "ms": ms, "solves_per_s": st["solves"] / (ms / 1e3),
            **st}


def cpu_oracle_leg(scene, dt, field_pairs_sample=200):
    """The CPU FP64 oracle on bounded samples of the same workloads (timed),
    and its solve of the seeded initial state (the accuracy reference)."""
    import numpy as np
    import oracle
    import synth
    Yc = scene["Y0"].copy()
    c0 = time.perf_counter()
    oracle.rk4_step(scene, Yc, 0.0, dt)
    c_el = time.perf_counter() - c0
    f_ref, UW_ref = oracle.solve_scene(scene, 0.0, scene["Y0"])
    fscene, yh = field_workload(synth)
    x, X, w, _ = oracle.geometry(fscene, 0.0, fscene["Y0"])
    nu = oracle.nearest(x, X, fscene["group_off"], fscene["groupX"])
    f = np.random.default_rng(7).normal(size=(3, fscene["N"]))
    ys = np.ascontiguousarray(yh[:, :field_pairs_sample])
    c1 = time.perf_counter()
    oracle.field_velocity(ys, X, w, nu, f, fscene["eps"], fscene["mu"])
    f_el = time.perf_counter() - c1
    # the same oracle solve on one thread
    single = None
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            c2 = time.perf_counter()
            oracle.solve_scene(scene, 0.0, scene["Y0"])
            single = time.perf_counter() - c2
    except Exception:
        pass
    cpu = {"value": 4.0 / c_el, "unit": "solves/s", "cores": cpu_threads(), "kind": "oracle",
           "sample": "one RK4 step (4 solves) of the same 25-filament workload from the "
                     "seeded initial state, NumPy/LAPACK FP64 oracle",
           "seconds": c_el, "cpu_model": cpu_model(), "logical_cpus": os.cpu_count(),
           "single_thread_solves_per_s": (1.0 / single) if single else None,
           "host_dgemm_gflops": host_dgemm_gflops()}
    field_cpu = {"value": ys.shape[1] * float(fscene["Q"]) / f_el, "unit": "pairs/s",
                 "cores": cpu_threads(), "kind": "oracle",
                 "sample": f"flow at the first {ys.shape[1]} tracers of the tracer workload",
                 "seconds": f_el}
    return cpu, field_cpu, f_ref, UW_ref


def run_small(ctx, nrs, synth, dev):
    """The small configurations: the unit sphere of the resistance problem
    (N = 96, Q = 1536, n = 288; synchronous-free repeated solves, 100 timed
    after 5 warm-up) and one and five filament swimmers (n = 126, 630;
    RK4 steps of dt = 2 pi / 100).  Mean and median per solve from HIP events
    around each solve or step, as the paper reports means over 100 runs."""
    import numpy as np
    import torch
    out = {}
    sc = synth.sphere_scene(4, 16)
    ds = nrs.DeviceScene(sc, dev)
    pb, u = device_problem(ctx, nrs, ds, sc, 0.0, None, dev)
    sol = torch.empty(pb.n, dtype=torch.float64, device=dev)
    rec = {"workload": "sphere_N96_Q1536", "n": pb.n}
    for name, m in (("fp64_lu", nrs.NRS_FP64_LU), ("fp32_ir", nrs.NRS_FP32_IR)):
        ws = torch.empty(nrs.nrs_workspace_size(ctx, pb.N, pb.Q, pb.M, m), dtype=torch.uint8,
                         device=dev)
        info = nrs.nrs_solve(ctx, pb, u, None, sol, ws, method=m)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(106)]
        for k in range(105):
            if k == 5:
                ev[0].record()
            nrs.nrs_solve(ctx, pb, u, None, sol, ws, method=m, info=False)
            if k >= 5:
                ev[k - 4].record()
        torch.cuda.synchronize()
        t = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(100)])
        rec[name] = {"solves_per_s": 1e3 / t.mean(), "ms_mean": float(t.mean()),
                     "ms_median": float(np.median(t)), "runs": 100,
                     "fell_back": info["fell_back"], "iterations": info["iterations"]}
    out["sphere"] = rec
    for M, steps in ((1, 100), (5, 50)):
        sc = synth.filament_scene(M, seed=0)
        ds = nrs.DeviceScene(sc, dev)
        rec = {"workload": f"filaments_M{M}_rk4", "n": 3 * sc["N"] + 6 * M}
        for name, m, k in (("fp32_ir", nrs.NRS_FP32_IR, steps), ("fp64_lu", nrs.NRS_FP64_LU,
                                                                   max(10, steps // 5))):
            ws = torch.empty(nrs.nrs_rk4_workspace_size(ctx, ds, m), dtype=torch.uint8,
                             device=dev)
            Y = torch.from_numpy(sc["Y0"].copy()).to(dev)
            dt = 2 * math.pi / 100
            for w in range(3):
                nrs.nrs_rk4_step(ctx, ds, Y, w * dt, dt, ws, method=m)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(k + 1)]
            ev[0].record()
            for j in range(k):
                nrs.nrs_rk4_step(ctx, ds, Y, (3 + j) * dt, dt, ws, method=m)
                ev[j + 1].record()
            torch.cuda.synchronize()
            t = np.array([ev[j].elapsed_time(ev[j + 1]) for j in range(k)]) / 4.0
            info = nrs.nrs_query_info(ctx, ws)
            rec[name] = {"solves_per_s": 1e3 / t.mean(), "ms_per_solve_mean": float(t.mean()),
                         "ms_per_solve_median": float(np.median(t)), "steps": k,
                         "fell_back": info["fell_back"]}
        out[f"filaments_M{M}"] = rec
    return out


def run_batched(ctx, nrs, synth, B, dev, reps=3, tune=True):
    """B independent rod-over-wall resistance problems (orders log-uniform in
    300..6000) in one nrs_solve_batched call: geometry and nearest map on the
    GPU (untimed inputs), then assembly + FP32 tile LU + FP64 refinement of
    every instance, timed with HIP events around the asynchronous call."""
    import numpy as np
    import torch
    scenes = synth.rod_wall_batch(B, seed=0)
    probs, us, keep = [], [], []
    for sc in scenes:
        ds = nrs.DeviceScene(sc, dev)
        N, Q = sc["N"], sc["Q"]
        x = torch.empty((3, N), dtype=torch.float64, device=dev)
        X = torch.empty((3, Q), dtype=torch.float64, device=dev)
        w = torch.empty(Q, dtype=torch.float64, device=dev)
        u = torch.empty(3 * N, dtype=torch.float64, device=dev)
        nrs.nrs_geometry(ctx, ds, 0.0, None, x, X, w, u)
        nu = torch.empty(Q, dtype=torch.int32, device=dev)
        nrs.nrs_nearest(ctx, x, sc["group_off"], X, ds.t["groupX"], nu)
        probs.append(nrs.Problem(x, X, w, nu, ds.t["body"], None, sc["eps"], sc["mu"]))
        us.append(u)
        keep.append(ds)
    ns = np.array([p.n for p in probs], dtype=np.float64)
    ws = torch.empty(nrs.nrs_solve_batched_workspace_size(ctx, probs), dtype=torch.uint8,
                     device=dev)
    tuned = {}
    tune_s = 0.0
    if tune:
        t0 = time.perf_counter()
        for p in probs:
            cls = (int(math.log2(p.N)), int(math.log2(max(1, p.Q // p.N))))
            if cls in tuned:
                continue
            wt = torch.empty(nrs.nrs_workspace_size(ctx, p.N, p.Q, p.M, nrs.NRS_FP32_IR),
                             dtype=torch.uint8, device=dev)
            r = nrs.nrs_autotune(ctx, p, wt)
            tuned[cls] = (r["block32"], r["strip32"])
        tune_s = time.perf_counter() - t0
    sols = [torch.empty(p.n, dtype=torch.float64, device=dev) for p in probs]
    infos = nrs.nrs_solve_batched(ctx, probs, us, sols, ws)
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        nrs.nrs_solve_batched(ctx, probs, us, sols, ws, info=False)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = float(np.mean(times))
    # the same batch captured once into a HIP graph and replayed
    gstream = torch.cuda.Stream()
    gctx = nrs.Context(0, stream=gstream.cuda_stream)
    if tune:
        for p in probs:
            cls = (int(math.log2(p.N)), int(math.log2(max(1, p.Q // p.N))))
            if cls in tuned and tuned[cls] is not None:
                wt = torch.empty(nrs.nrs_workspace_size(ctx, p.N, p.Q, p.M, nrs.NRS_FP32_IR),
                                 dtype=torch.uint8, device=dev)
                nrs.nrs_autotune(gctx, p, wt)
                tuned[cls] = None
    torch.cuda.synchronize()
    nrs.nrs_solve_batched(gctx, probs, us, sols, ws, info=False, graph=1)   # capture + first run
    gstream.synchronize()
    gtimes = []
    for _ in range(reps):
        g0 = torch.cuda.Event(enable_timing=True)
        g1 = torch.cuda.Event(enable_timing=True)
        g0.record(gstream)
        nrs.nrs_solve_batched(gctx, probs, us, sols, ws, info=False, graph=1)
        g1.record(gstream)
        gstream.synchronize()
        gtimes.append(g0.elapsed_time(g1))
    gctx.close()
    gms = float(np.mean(gtimes))
    lu_flops = float((2.0 / 3.0 * ns ** 3).sum())
    return {"workload": f"rodwall_B{B}", "instances": B, "n_min": int(ns.min()),
            "n_max": int(ns.max()), "n_mean": float(ns.mean()),
            "solves_per_s": B / (ms / 1e3), "ms_per_batch": ms, "reps": reps,
            "graph_solves_per_s": B / (gms / 1e3), "graph_ms_per_batch": gms,
            "tuned_size_classes": len(tuned), "tune_s": tune_s if tune else 0.0,
            "lu_flops_total": lu_flops,
            "lu_equiv_tflops": lu_flops / (ms / 1e3) / 1e12,
            "max_backward_error": max(i["backward_error"] for i in infos),
            "fell_back": int(sum(i["fell_back"] for i in infos)),
            "max_iterations": int(max(i["iterations"] for i in infos)),
            "note": "time covers assembly, every factorisation and the refinement of all "
                    "instances; lu_equiv_tflops = sum of (2/3) n^3 over the batch time"}


def run_batched_child(args):
    """run_batched in a fresh process (`bench.py --batch-only`); its JSON."""
    import subprocess
    cmd = [sys.executable, "-u", os.path.abspath(__file__), "--batch-only",
           "--batch", str(args.batch)] + (["--no-tune"] if args.no_tune else [])
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    if r.returncode != 0:
        raise RuntimeError(f"batched benchmark failed ({r.returncode}):\n{r.stderr[-2000:]}")
    line = [ln for ln in r.stdout.splitlines() if ln.startswith("{")][-1]
    out = json.loads(line)["batched"]
    out["process"] = "child (bench.py --batch-only)"
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=25)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--method", default="fp32_ir", choices=sorted(METHODS))
    ap.add_argument("--swimmers", type=int, default=25)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the other solution forms")
    ap.add_argument("--batch", type=int, default=512, metavar="B",
                    help="also time the batched rod-over-wall workload with B instances (0: skip)")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-shape autotuner")
    ap.add_argument("--batch-only", action="store_true",
                    help="time only the batched workload (profiling)")
    ap.add_argument("--no-field", action="store_true",
                    help="skip the flow-at-tracers workload")
    ap.add_argument("--no-channel", action="store_true",
                    help="skip the channel configuration (n = 14,244 and 39,504)")
    ap.add_argument("--channel-only", action="store_true",
                    help="time only the channel configuration (profiling)")
    ap.add_argument("--field-only", action="store_true",
                    help="time only the flow-at-tracers workload (profiling)")
    ap.add_argument("--block-only", action="store_true",
                    help="time only the learned block-preconditioned GMRES form (profiling)")
    ap.add_argument("--calib-copy", type=int, default=0, metavar="MIB",
                    help="also run one plain device copy of MIB MiB (counter calibration)")
    ap.add_argument("--calib-flops", action="store_true",
                    help="also run kernels of known flop counts (counter calibration)")
    ap.add_argument("--channel-k", type=int, default=0, choices=(0, 10, 40),
                    help="with --channel-only: only the 10- or 40-swimmer channel")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the small configurations (sphere, 1 and 5 filaments)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_2001_06468_amd as nrs

    dev = "cuda:0"
    M = args.swimmers
    scene = synth.filament_scene(M, seed=0)
    N, Q = scene["N"], scene["Q"]
    n = 3 * N + 6 * M
    ds = nrs.DeviceScene(scene, dev)
    ctx = nrs.Context(0)
    dt = 2 * math.pi / 100

    per_step = []

    def run_steps(method, warmup, steps, **opts):
        ws = torch.empty(nrs.nrs_rk4_workspace_size(ctx, ds, method), dtype=torch.uint8, device=dev)
        Y = torch.from_numpy(scene["Y0"].copy()).to(dev)
        t = 0.0
        for _ in range(warmup):
            nrs.nrs_rk4_step(ctx, ds, Y, t, dt, ws, method=method, **opts)
            t += dt
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        w0 = time.perf_counter()
        ev[0].record()
        for k in range(steps):
            nrs.nrs_rk4_step(ctx, ds, Y, t, dt, ws, method=method, **opts)
            t += dt
            ev[k + 1].record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        info = nrs.nrs_query_info(ctx, ws)
        per_step.clear()
        per_step.extend(ev[k].elapsed_time(ev[k + 1]) for k in range(steps))
        return ev[0].elapsed_time(ev[steps]), wall, Y, t, info

    if args.calib_copy > 0:
        src = torch.ones(args.calib_copy * (1 << 20) // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.calib_flops:
        # kernels of known work for the counter runs: one FP32 matrix product
        # (2 * 4096^3 flops on the matrix cores) and one FP32 and one FP64
        # elementwise multiply of 2^26 elements (2^26 flops each on the VALU)
        a = torch.ones(4096, 4096, dtype=torch.float32, device=dev)
        (a @ a).sum()
        v32 = torch.ones(1 << 26, dtype=torch.float32, device=dev)
        v32.mul_(1.5)
        v64 = torch.ones(1 << 26, dtype=torch.float64, device=dev)
        v64.mul_(1.5)
        torch.cuda.synchronize()
        del a, v32, v64

    if args.channel_only:
        sizes = ((10, 16), (40, 24)) if args.channel_k == 0 else \
            tuple(x for x in ((10, 16), (40, 24)) if x[0] == args.channel_k)
        print(json.dumps({"channel": run_channel(ctx, nrs, synth, dev, sizes)}), flush=True)
        return

    if args.field_only:
        print(json.dumps({"field": run_field(ctx, nrs, synth, dev)}), flush=True)
        return

    def block_forms(Yref, names=("gmres_block_exact", "gmres_block_learned")):
        # block-diagonal preconditioned GMRES from the previous stage's
        # solution: exact body-block inverses, and the learned block model
        # (Fourier fit in the beat phase of one filament's blocks)
        from paper_2001_06468_amd import learned as learned_mod
        bm = learned_mod.fit_block_model(ctx, synth.filament_scene(1, seed=0), S=48, H=6)
        block_info = {"fit_s": bm.fit_seconds, "phases": 48, "harmonics": bm.H, "order": bm.nb,
                      "source": "one filament in its own frame (the method's FP64 blocks)"}
        out = {}
        for name, opts in (("gmres_block_exact", {"precond": nrs.NRS_PRECOND_EXACT}),
                           ("gmres_block_learned", {"precond": nrs.NRS_PRECOND_MODEL,
                                                    "block_model": bm})):
            if name not in names:
                continue
            fm, _, Yb, _, finfo = run_steps(nrs.NRS_GMRES_BLOCK, args.warmup, args.steps,
                                            warm_start=nrs.NRS_WARM_PREVIOUS, **opts)
            out[name] = {"solves_per_s": 4 * args.steps / (fm / 1e3),
                         "ms_per_step": fm / args.steps,
                         "ms_per_step_median": float(np.median(per_step)),
                         "steps": args.steps, "fell_back": finfo["fell_back"],
                         "max_stage_iterations_last_step": finfo["iterations"]}
            if Yref is not None:
                out[name]["max_abs_state_diff_vs_headline"] = float((Yb - Yref).abs().max())
        if "gmres_block_learned" in out:
            out["gmres_block_learned"]["model"] = block_info
        return out

    if args.block_only:
        print(json.dumps({"forms": block_forms(None, ("gmres_block_learned",))}), flush=True)
        return

    if args.batch_only:
        print(json.dumps({"batched": run_batched(ctx, nrs, synth, max(args.batch, 1), dev,
                                                 tune=not args.no_tune)}),
              flush=True)
        return

    # autotune the assembly launch shape for this size class (never changes results)
    method = METHODS[args.method]
    tune = None
    Y0d = torch.from_numpy(scene["Y0"].copy()).to(dev)
    if not args.no_tune:
        pbt, _ = device_problem(ctx, nrs, ds, scene, 0.0, Y0d, dev)
        wst = torch.empty(nrs.nrs_workspace_size(ctx, N, Q, M, nrs.NRS_FP32_IR), dtype=torch.uint8,
                          device=dev)
        tune = nrs.nrs_autotune(ctx, pbt, wst)
        del wst
    ms, wall, Y, t_end, info = run_steps(method, args.warmup, args.steps)
    solves = 4 * args.steps
    value = solves / (ms / 1e3)
    step_ms = list(per_step)

    # --- one synchronous solve of the seeded initial state (accuracy check
    # against the oracle in the CPU leg) on the product's own geometry -------
    pb, u = device_problem(ctx, nrs, ds, scene, 0.0, Y0d, dev)
    # sized for the solve's method and for the FP32 assembly timed below
    ws1 = torch.empty(max(nrs.nrs_workspace_size(ctx, N, Q, M, method),
                          nrs.nrs_workspace_size(ctx, N, Q, M, nrs.NRS_FP32_IR)),
                      dtype=torch.uint8, device=dev)
    sol = torch.empty(n, dtype=torch.float64, device=dev)
    sinfo = nrs.nrs_solve(ctx, pb, u, None, sol, ws1, method=method)
    s = sol.cpu().numpy()

    # --- dominant kernel: the tile LU, one launch, timed with events ----------
    lda = nrs.lda_for(n)
    A32 = torch.empty((n, lda), dtype=torch.float32, device=dev)
    nrs.nrs_assemble(ctx, pb, 32, A32, lda, ws1)
    A0 = A32.clone()
    ipiv = torch.empty(n, dtype=torch.int32, device=dev)
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    sing = torch.zeros(1, dtype=torch.int32, device=dev)
    lu_ms = []
    wl = torch.empty(nrs.nrs_lu_factor_workspace_size(ctx, n, 32), dtype=torch.uint8, device=dev)
    for rep in range(12):
        A32.copy_(A0)
        a0 = torch.cuda.Event(enable_timing=True)
        a1 = torch.cuda.Event(enable_timing=True)
        a0.record()
        nrs.nrs_lu_factor(ctx, A32, lda, ipiv, perm, sing, wl, pivot_scope=1)
        a1.record()
        torch.cuda.synchronize()
        if rep >= 2:
            lu_ms.append(a0.elapsed_time(a1))
    lu_avg_ms = float(np.mean(lu_ms))
    lu_flops = 2.0 / 3.0 * n ** 3
    import hashlib
    src = os.path.join(ROOT, "paper_2001_06468_amd", "csrc", "lu_tiles.hip")
    cur = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    traffic = (LU_TRAFFIC["bytes_per_launch"]
               if cur == LU_TRAFFIC["source_sha256_16"] and n == LU_TRAFFIC["n"] else None)
    lu_tflops = lu_flops / (lu_avg_ms / 1e3) / 1e12

    # --- assembly rate: nrs_assemble (nu-sorted layout + fused kernel + rigid blocks)
    as_ms = []
    for rep in range(12):
        b0 = torch.cuda.Event(enable_timing=True)
        b1 = torch.cuda.Event(enable_timing=True)
        b0.record()
        nrs.nrs_assemble(ctx, pb, 32, A32, lda, ws1)
        b1.record()
        torch.cuda.synchronize()
        if rep >= 2:
            as_ms.append(b0.elapsed_time(b1))
    as_avg_ms = float(np.mean(as_ms))
    asm_flops = 33.0 * N * Q
    asm_tflops = asm_flops / (as_avg_ms / 1e3) / 1e12
    ws64 = torch.empty(nrs.nrs_workspace_size(ctx, N, Q, M, nrs.NRS_FP64_LU), dtype=torch.uint8,
                       device=dev)
    A64 = torch.empty((n, lda), dtype=torch.float64, device=dev)
    as64_ms = []
    for rep in range(12):
        b0 = torch.cuda.Event(enable_timing=True)
        b1 = torch.cuda.Event(enable_timing=True)
        b0.record()
        nrs.nrs_assemble(ctx, pb, 64, A64, lda, ws64)
        b1.record()
        torch.cuda.synchronize()
        if rep >= 2:
            as64_ms.append(b0.elapsed_time(b1))
    del A64, ws64
    as64_avg_ms = float(np.mean(as64_ms))
    asm64_tflops = asm_flops / (as64_avg_ms / 1e3) / 1e12

    forms = {}
    small = None
    batched = None
    learned_info = None
    # The 512-system batch runs in a child process of its own: its per-system
    # kernels use four streams, and in one process with the cooperative
    # launches of the partial-pivoting panel (fp64_lu, fp32_gepp_ir, the
    # small configurations) this runtime slows both: the batch after a
    # cooperative launch takes about 295 instead of 241 ms, and the FP64
    # partial-pivoting forms after the batch lose about a quarter.
    if args.batch > 0:
        batched = run_batched_child(args)
    if not args.no_forms:
        forms["dopri5_" + args.method] = run_dopri(ctx, nrs, ds, scene, dev, method)
        if method == nrs.NRS_FP32_IR:
            # the same steps with stages 2-4 refined against the first stage's
            # FP32 factors (no assembly or factorisation there); final state
            # compared with the headline run's
            fm, _, Yr, _, finfo = run_steps(method, args.warmup, args.steps,
                                            reuse_stage_factors=1)
            forms["fp32_ir_stage_factor_reuse"] = {
                "solves_per_s": 4 * args.steps / (fm / 1e3), "ms_per_step": fm / args.steps,
                "steps": args.steps, "fell_back": finfo["fell_back"],
                "max_stage_iterations_last_step": finfo["iterations"],
                "max_abs_state_diff_vs_headline": float((Yr - Y).abs().max())}
        for name, m in METHODS.items():
            if m == method:
                continue
            k = 2
            fm, _, _, _, finfo = run_steps(m, 1, k)
            forms[name] = {"solves_per_s": 4 * k / (fm / 1e3), "steps": k,
                           "fell_back": finfo["fell_back"]}
    # then the light, latency-bound small configurations, and last the
    # sustained GPU work of the learned forms (training data of 20,000 solves)
    if not args.no_small:
        small = run_small(ctx, nrs, synth, dev)
    if not args.no_forms:
        # GMRES forms: cold, previous-solve warm start, learned warm start
        model, learned_info = train_model(ctx, nrs)
        body_off = nrs.nrs_mlp_body_offsets(ctx, ds.t["body"], M)
        k = 3
        for name, opts in (("gmres_cold", {}),
                           ("gmres_previous", {"warm_start": nrs.NRS_WARM_PREVIOUS}),
                           ("gmres_learned", {"warm_start": nrs.NRS_WARM_MODEL, "model": model,
                                              "body_off": body_off})):
            fm, _, Yf, tf, finfo = run_steps(nrs.NRS_GMRES, 1, k, **opts)
            forms[name] = {"solves_per_s": 4 * k / (fm / 1e3), "steps": k,
                           "fell_back": finfo["fell_back"],
                           "max_stage_iterations_last_step": finfo["iterations"]}
        forms.update(block_forms(Y))

    field = None
    if not args.no_field:
        field = run_field(ctx, nrs, synth, dev)

    channel = None
    if not args.no_channel:
        channel = run_channel(ctx, nrs, synth, dev)

    cpu = None
    accuracy = None
    if not args.no_cpu_baseline:
        cpu, field_cpu, f_ref, UW_ref = cpu_oracle_leg(scene, dt)
        if field is not None:
            field["cpu_baseline"] = field_cpu
        err_f = float(np.linalg.norm(s[:3 * N] - f_ref.ravel()) / np.linalg.norm(f_ref))
        err_uw = float(np.linalg.norm(s[3 * N:] - UW_ref.ravel()) / np.linalg.norm(UW_ref))
        accuracy = {"rel_force_err": err_f, "rel_velocity_err": err_uw, "target": 1e-8,
                    "solve_info": sinfo, "step_info": info,
                    "note": "solve_info: synchronous solve of the seeded initial state "
                            "(compared with the oracle), backward_error at the returned "
                            "solution; step_info: worst of the last timed step's four stages, "
                            "backward_error at the iterate before the last correction"}

    out = {
        "metric": "time-step solves/sec (assemble+solve) at <=1e-8 rel force err",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "ms_per_step_median": float(np.median(step_ms)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if method else "f64",
        "data": "synthetic",
        "config": {"workload": f"filaments_M{M}_rk4", "swimmers": M, "N": N, "Q": Q, "n": n,
                   "eps": scene["eps"], "dt": dt, "method": args.method},
        "accuracy": accuracy,
        "roofline": {"kernel": "k_lu_tiles<float>", "bound": "mfma", "achieved": lu_tflops,
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": lu_tflops / PEAK_FP32_TFLOPS, "traffic": traffic,
                     "flops_per_launch": lu_flops, "avg_launch_ms": lu_avg_ms,
                     "median_launch_ms": float(np.median(lu_ms)),
                     "counters": counter_summary("lu", cur)},
        "assembly": {"tflops": asm_tflops, "frac_fp32_peak": asm_tflops / PEAK_FP32_TFLOPS,
                     "flops_per_call": asm_flops, "avg_call_ms": as_avg_ms,
                     "median_call_ms": float(np.median(as_ms)),
                     "fp64": {"tflops": asm64_tflops,
                              "frac_fp64_peak": asm64_tflops / PEAK_FP64_TFLOPS,
                              "avg_call_ms": as64_avg_ms,
                              "median_call_ms": float(np.median(as64_ms))},
                     "counters": counter_summary("assembly"),
                     "note": "33 flops per (force point, quadrature point) pair; call includes "
                             "the nu-sorted layout and rigid-body blocks"},
        "forms": forms,
        "small_configs": small,
        "learned_training": learned_info,
        "autotune": tune,
        "batched": batched,
        "field": field,
        "channel": channel,
        "cpu_baseline": cpu,
        "wall_s": wall,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
