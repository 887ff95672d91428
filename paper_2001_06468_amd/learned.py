"""Training data and training loops of the learned parts of the GMRES forms:
the warm-start network and the block preconditioner model.

The network (include/nrs.h, "Learned warm start") maps body-frame features of
each free body's force points to the body-frame force density and the body's
(U, Omega).  Training data are solves of the method itself: undulating
filament swimmers with random seeds, beat phases, times and swimmer counts,
solved on the GPU (FP32 LU + FP64 refinement, batched); the network is then
fitted by the library's own forward/backward and Adam kernels.  This module
only sequences those calls: every feature, target, gradient and update is
computed by libnrs.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

import synth

from . import (BlockModel, Context, DeviceScene, Model, Problem, nrs_adam_step,  # noqa: F401
               nrs_assemble, nrs_block_invert, nrs_block_model_fit, nrs_geometry,
               nrs_workspace_size, NRS_FP64_LU,
               nrs_mlp_body_offsets, nrs_mlp_features, nrs_mlp_grad, nrs_mlp_grad_workspace_size,
               nrs_mlp_param_count, nrs_mlp_status, nrs_mlp_targets, nrs_nearest,
               nrs_solve_batched, nrs_solve_batched_workspace_size, NRS_FP32_IR)


class Dataset:
    """Features, targets and body offsets of many bodies (device tensors)."""

    def __init__(self, phi, sols, Ys, bodies, body_off, n_solves, meta):
        self.phi = phi            # [P, 7] float32
        self.sols = sols          # per-solve raw solutions (kept until targets are built)
        self.Ys = Ys
        self.bodies = bodies
        self.body_off = body_off  # [B + 1] int32
        self.n_solves = n_solves
        self.meta = meta          # per body: (solve index, seed, M)
        self.t_pt = None
        self.t_body = None
        self.scales = None

    @property
    def n_bodies(self):
        return self.body_off.numel() - 1


def filament_states(n_solves, seed0, m_choices=(1, 5, 25), m_probs=(0.8, 0.15, 0.05)):
    """Seeded (scene, t) pairs: filaments with random phases at random times."""
    rng = np.random.default_rng(seed0)
    out = []
    for i in range(n_solves):
        M = int(rng.choice(m_choices, p=m_probs))
        sc = synth.filament_scene(M, seed=seed0 + i, phase_random=True)
        out.append((sc, float(rng.random() * 2 * math.pi), seed0 + i))
    return out


def device_problem(ctx, sc, t, dev="cuda"):
    """Geometry and nearest map of a scene state on the GPU; returns
    (Problem, u, DeviceScene)."""
    ds = DeviceScene(sc, dev)
    N, Q = sc["N"], sc["Q"]
    x = torch.empty((3, N), dtype=torch.float64, device=dev)
    X = torch.empty((3, Q), dtype=torch.float64, device=dev)
    w = torch.empty(Q, dtype=torch.float64, device=dev)
    u = torch.empty(3 * N, dtype=torch.float64, device=dev)
    Y = ds.t["Y0"]
    nrs_geometry(ctx, ds, t, Y, x, X, w, u)
    nu = torch.empty(Q, dtype=torch.int32, device=dev)
    nrs_nearest(ctx, x, sc["group_off"], X, ds.t["groupX"], nu)
    pb = Problem(x, X, w, nu, ds.t["body"], Y, sc["eps"], sc["mu"])
    return pb, u, ds


def generate(ctx, states, batch=256, dev="cuda"):
    """Solve every (scene, t) state on the GPU and collect features.  Targets
    need the output scales, see build_targets()."""
    phis, sols, Ys, bodies, counts, meta = [], [], [], [], [], []
    for b0 in range(0, len(states), batch):
        chunk = states[b0:b0 + batch]
        pbs, us, dss = [], [], []
        for sc, t, seed in chunk:
            pb, u, ds = device_problem(ctx, sc, t, dev)
            pbs.append(pb)
            us.append(u)
            dss.append(ds)
        ws = torch.empty(nrs_solve_batched_workspace_size(ctx, pbs), dtype=torch.uint8, device=dev)
        xs = [torch.empty(p.n, dtype=torch.float64, device=dev) for p in pbs]
        fts = [ds.t["ftext"] for ds in dss]
        infos = nrs_solve_batched(ctx, pbs, us, xs, ws, ftexts=fts, method=NRS_FP32_IR)
        if any(i["fell_back"] for i in infos):
            raise RuntimeError("a training solve needed the FP64 fallback")
        for k, ((sc, t, seed), pb, u, ds, x) in enumerate(zip(chunk, pbs, us, dss, xs)):
            phi = torch.empty((pb.N, 7), dtype=torch.float32, device=dev)
            nrs_mlp_features(ctx, pb.x, u, ds.t["s"], ds.t["body"], pb.M, pb.Y, phi)
            phis.append(phi)
            sols.append(x)
            Ys.append(pb.Y)
            bodies.append(ds.t["body"])
            counts.append(np.bincount(sc["body"][sc["body"] >= 0], minlength=pb.M))
            meta.extend([(b0 + k, seed, pb.M)] * pb.M)
        del ws
    sizes = np.concatenate(counts)
    off = torch.from_numpy(np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)).to(dev)
    return Dataset(torch.cat(phis), sols, Ys, bodies, off, len(states), meta)


def solution_scales(data):
    """RMS force-density component and RMS U, Omega components of the
    training solutions."""
    f2, u2, o2, nf, nb = 0.0, 0.0, 0.0, 0, 0
    for x, body in zip(data.sols, data.bodies):
        N = body.numel()
        M = (x.numel() - 3 * N) // 6
        f2 += float((x[:3 * N] ** 2).sum())
        uw = x[3 * N:].view(M, 6)
        u2 += float((uw[:, :3] ** 2).sum())
        o2 += float((uw[:, 3:] ** 2).sum())
        nf += 3 * N
        nb += 3 * M
    return (math.sqrt(f2 / nf), math.sqrt(u2 / nb), math.sqrt(o2 / nb))


def build_targets(ctx, data, scales=None):
    scales = scales or solution_scales(data)
    t_pts, t_bs = [], []
    for x, Y, body in zip(data.sols, data.Ys, data.bodies):
        N = body.numel()
        M = Y.numel() // 12
        tp = torch.empty((N, 3), dtype=torch.float32, device=x.device)
        tb = torch.empty((M, 6), dtype=torch.float32, device=x.device)
        nrs_mlp_targets(ctx, body, M, Y, x, scales, tp, tb)
        t_pts.append(tp)
        t_bs.append(tb)
    data.t_pt = torch.cat(t_pts)
    data.t_body = torch.cat(t_bs)
    data.scales = tuple(scales)
    return data


def init_theta(seed=0, dev="cuda"):
    """Glorot-uniform weights, zero biases (flat order of include/nrs.h)."""
    rng = np.random.default_rng(seed)
    H = 64
    parts = []
    for rows, cols, bias in ((H, 7, H), (H, H, 0), (H, H, H), (3, H, 3), (6, H, 6)):
        a = math.sqrt(6.0 / (rows + cols))
        parts.append(rng.uniform(-a, a, size=rows * cols))
        if bias:
            parts.append(np.zeros(bias))
    theta = np.concatenate(parts).astype(np.float32)
    assert theta.size == nrs_mlp_param_count()
    return torch.from_numpy(theta).to(dev)


def train(ctx, data, steps=2000, batch_bodies=256, lr=3e-3, lr_final=3e-4, seed=0,
          val=None, log_every=200, theta=None):
    """Adam on minibatches of bodies; cosine-free exponential learning-rate
    decay from lr to lr_final.  Returns (Model, history)."""
    dev = data.phi.device
    theta = init_theta(seed, dev) if theta is None else theta.clone()
    P = theta.numel()
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    grad = torch.empty(P + 1, dtype=torch.float32, device=dev)
    nb = min(batch_bodies, data.n_bodies)
    ws = torch.empty(nrs_mlp_grad_workspace_size(nb), dtype=torch.uint8, device=dev)
    gen = torch.Generator(device="cpu").manual_seed(seed)
    perm = torch.randperm(data.n_bodies, generator=gen)
    pos = 0
    hist = []
    decay = (lr_final / lr) ** (1.0 / max(steps - 1, 1))
    t0 = time.perf_counter()
    for step in range(1, steps + 1):
        if pos + nb > data.n_bodies:
            perm = torch.randperm(data.n_bodies, generator=gen)
            pos = 0
        sel = perm[pos:pos + nb].to(torch.int32).to(dev)
        pos += nb
        nrs_mlp_grad(ctx, theta, data.n_bodies, data.body_off, data.phi, data.t_pt, data.t_body,
                     grad, ws, sel=sel)
        nrs_adam_step(ctx, theta, grad[:P], m, v, step, lr * decay ** (step - 1))
        if step % log_every == 0 or step == steps:
            rec = {"step": step, "loss": float(grad[P])}
            if val is not None:
                rec["val_loss"] = evaluate_loss(ctx, theta, val)
            hist.append(rec)
    torch.cuda.synchronize()
    if nrs_mlp_status(ctx):
        raise RuntimeError("a training body exceeded the network's point limit")
    model = Model(theta, data.scales)
    model.train_seconds = time.perf_counter() - t0
    return model, hist


def evaluate_loss(ctx, theta, data):
    """Loss over every body of a dataset (batched through the gradient kernel)."""
    P = theta.numel()
    dev = theta.device
    grad = torch.empty(P + 1, dtype=torch.float32, device=dev)
    total, count = 0.0, 0
    bs = 4096
    ws = torch.empty(nrs_mlp_grad_workspace_size(bs), dtype=torch.uint8, device=dev)
    for b0 in range(0, data.n_bodies, bs):
        sel = torch.arange(b0, min(b0 + bs, data.n_bodies), dtype=torch.int32, device=dev)
        nrs_mlp_grad(ctx, theta, data.n_bodies, data.body_off, data.phi, data.t_pt, data.t_body,
                     grad, ws, sel=sel)
        total += float(grad[P]) * sel.numel()
        count += sel.numel()
    return total / count


def fit_block_model(ctx, scene, S=48, H=6, dev="cuda"):
    """Learned body-block inverse of NRS_GMRES_BLOCK from the method's own
    blocks.  scene: host scene dict (``synth`` layout) of ONE free body whose
    points are all the body's (no fixed points), its frame at the origin with
    B = I.  At the S beat phases psi_s = 2 pi s / S (time t_s = (psi_s + phi)
    / omega of the body's wave part) the library assembles the one-body
    system in FP64 (geometry, nearest map, assembly: the body's diagonal
    block in its own frame), inverts the S blocks and fits the Fourier model
    of degree H.  Returns a BlockModel (with .fit_seconds)."""
    if int(scene["M"]) != 1 or np.any(np.asarray(scene["body"]) != 0):
        raise ValueError("the block model is fitted on a scene of one free body and nothing else")
    wave = np.asarray(scene["wave"], dtype=np.float64).reshape(-1, 6)
    part = np.asarray(scene["part"])
    parts = part[part >= 0]
    if parts.size == 0:
        if H != 0:
            raise ValueError("a body without a wave part has one block: use H = 0")
        omega, phi = 1.0, 0.0
    else:
        omega, phi = float(wave[parts[0], 4]), float(wave[parts[0], 5])
        if omega == 0.0 and H != 0:
            raise ValueError("a body whose wave does not move has one block: use H = 0")
        omega = omega or 1.0
    sc = dict(scene)
    Y = np.zeros((1, 12))
    Y[0, 3:] = np.eye(3).ravel()
    sc["Y0"] = Y
    t0 = time.perf_counter()
    ds = DeviceScene(sc, dev)
    N, Q = ds.N, ds.Q
    nb = 3 * N + 6
    x = torch.empty((3, N), dtype=torch.float64, device=dev)
    X = torch.empty((3, Q), dtype=torch.float64, device=dev)
    w = torch.empty(Q, dtype=torch.float64, device=dev)
    nu = torch.empty(Q, dtype=torch.int32, device=dev)
    blocks = torch.empty((S, nb, nb), dtype=torch.float64, device=dev)
    ws = torch.empty(nrs_workspace_size(ctx, N, Q, 1, NRS_FP64_LU), dtype=torch.uint8, device=dev)
    Yd = ds.t["Y0"]
    for s in range(S):
        t = (2.0 * math.pi * s / S + phi) / omega
        nrs_geometry(ctx, ds, t, Yd, x, X, w, None)
        nrs_nearest(ctx, x, ds.group_off, X, ds.t["groupX"], nu)
        pb = Problem(x, X, w, nu, ds.t["body"], Yd, ds.eps, ds.mu)
        nrs_assemble(ctx, pb, 64, blocks[s], nb, ws)
    singular = torch.zeros(1, dtype=torch.int32, device=dev)
    nrs_block_invert(ctx, blocks, singular)
    coef = torch.empty((2 * H + 1, nb, nb), dtype=torch.float64, device=dev)
    nrs_block_model_fit(ctx, blocks, H, coef)
    torch.cuda.synchronize()
    if int(singular.item()):
        raise RuntimeError("a sampled body block is singular")
    model = BlockModel(coef, nb, H)
    model.fit_seconds = time.perf_counter() - t0
    return model
