"""Writes the stored expected values of the full-size parity tests.

Every value written here comes from the CPU FP64 oracle (``oracle/``) on the
seeded scenes of ``synth/``; nothing is read from the HIP library.

    python tests/golden/make_golden.py channel10   # channel_K10_h16.npz
    python tests/golden/make_golden.py channel40   # channel_K40_h24.npz (about 40 GB of RAM)
    python tests/golden/make_golden.py rk4         # rk4_filaments_M25_2steps.npz
    python tests/golden/make_golden.py batch       # rodwall_B512_sample16.npz

Files:
  channel_*.npz   the solution (f, then (U, Omega) per swimmer) of the
                  swimming problem of Sec. 4 for the sperm-in-a-channel scene
                  at t = 0 (LU with partial pivoting, FP64), the LAPACK
                  1-norm condition estimate of the full matrix, and the
                  SHA-256 of the nearest map (int32) the oracle computed, so
                  a test can confirm it solves the same system;
  rk4_*.npz       the body states after two classical RK4 steps (dt = 2 pi /
                  100) of 25 filament swimmers, every stage a full oracle
                  solve (geometry, nearest map, assembly, dgesv);
  rodwall_*.npz   oracle solutions of 16 instances of the 512-instance
                  rod-over-wall batch (seed 0), chosen at evenly spaced ranks
                  of the order n, with their indices.
"""
from __future__ import annotations

import hashlib
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402


def nu_digest(nu):
    return hashlib.sha256(np.ascontiguousarray(nu, dtype=np.int32).tobytes()).hexdigest()


def channel(K, hinv):
    t0 = time.time()
    scene = synth.sperm_channel_scene(K, h=1.0 / hinv, seed=0)
    N, M = scene["N"], scene["M"]
    Y = scene["Y0"]
    x, X, w, u = oracle.geometry(scene, 0.0, Y)
    nu = oracle.nearest(x, X, scene["group_off"], scene["groupX"])
    print(f"K={K}: N={N} Q={scene['Q']} n={3 * N + 6 * M}: geometry and nearest map "
          f"{time.time() - t0:.0f} s", flush=True)
    As = oracle.assemble_As(x, X, w, nu, scene["eps"], scene["mu"])
    W = oracle.patch_weights(w, nu, N)
    print(f"K={K}: A_s assembled {time.time() - t0:.0f} s", flush=True)
    A = oracle.assemble_system(As, x, W, scene["body"], Y, M)
    del As
    b = oracle.rhs(u, scene["ftext"])
    sol, kappa = oracle.solve_with_condition(A, b, overwrite=True)
    del A
    print(f"K={K}: solved {time.time() - t0:.0f} s, kappa_1 estimate {kappa:.3e}", flush=True)
    out = os.path.join(HERE, f"channel_K{K}_h{hinv}.npz")
    np.savez_compressed(out, sol=sol, kappa1=np.float64(kappa), N=np.int64(N), M=np.int64(M),
                        nu_sha256=np.array(nu_digest(nu)), scene=np.array(scene["name"]))
    print("wrote", out, flush=True)


def rk4():
    scene = synth.filament_scene(25, seed=0)
    dt = 2 * math.pi / 100
    Y = scene["Y0"].copy()
    t = 0.0
    states = []
    for _ in range(2):
        Y = oracle.rk4_step(scene, Y, t, dt)
        t += dt
        states.append(Y.copy())
        print(f"rk4: t = {t:.4f}", flush=True)
    out = os.path.join(HERE, "rk4_filaments_M25_2steps.npz")
    np.savez_compressed(out, Y1=states[0], Y2=states[1], dt=np.float64(dt),
                        scene=np.array(scene["name"]))
    print("wrote", out, flush=True)


def batch():
    scenes = synth.rod_wall_batch(512, seed=0)
    ns = np.array([3 * s["N"] + 6 * s["M"] for s in scenes])
    order = np.argsort(ns, kind="stable")
    ranks = np.round(np.linspace(0, len(order) - 1, 16)).astype(int)
    idx = order[ranks]
    sols, digests = [], []
    for k in idx:
        sc = scenes[k]
        f, UW, d = oracle.solve_scene(sc, 0.0, return_all=True)
        sols.append(d["sol"])
        digests.append(nu_digest(d["nu"]))
        print(f"batch: instance {k} n = {ns[k]}", flush=True)
    out = os.path.join(HERE, "rodwall_B512_sample16.npz")
    np.savez_compressed(out, idx=idx.astype(np.int64), n=ns[idx].astype(np.int64),
                        sol=np.concatenate(sols), nu_sha256=np.array(digests))
    print("wrote", out, flush=True)


if __name__ == "__main__":
    what = sys.argv[1:] or ["channel10", "rk4", "batch"]
    for w in what:
        if w == "channel10":
            channel(10, 16)
        elif w == "channel40":
            channel(40, 24)
        elif w == "rk4":
            rk4()
        elif w == "batch":
            batch()
        else:
            raise SystemExit(f"unknown item {w}")
