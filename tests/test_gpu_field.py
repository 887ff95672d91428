"""Parity of the field-point velocity and tracer entry points with the CPU
FP64 oracle (MI355X).

Tolerance of the field sum: both sides add the same terms in FP64 in
different orders, and the kernel's 1/sqrt is the hardware estimate refined
by two Newton steps (within rounding of the correctly rounded value), so each
component may differ by a few units of 2^-53 times the sum of the absolute
values of its terms, times the number of terms in the worst case.  The tests
allow 1e-13 of that absolute sum (bounded with |S g| <= (2|r|^2 + 2 eps^2)
|g| / (|r|^2 + eps^2)^(3/2)): two orders above the expected rounding at
these sizes, far below any wrong term, sign or index.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2001_06468_amd as nrs
    from gpu_util import T, prepare, gpu_solve, DEV


@pytest.fixture(scope="module")
def ctx():
    c = nrs.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _abs_bound(y, X, w, nu, f, eps, mu):
    """(8 pi mu)^-1 sum_q |S^eps(y - X_q)| |w_q f[nu_q]| per field point."""
    g = np.linalg.norm(f[:, nu] * w[None, :], axis=0)
    out = np.zeros(y.shape[1])
    for p in range(y.shape[1]):
        r2 = np.sum((y[:, p:p + 1] - X) ** 2, axis=0)
        out[p] = np.sum((2 * r2 + 2 * eps * eps) / (r2 + eps * eps) ** 1.5 * g)
    return out / (8 * math.pi * mu)


def _field_points(rng, host, P):
    """P points in the scene's bounding box; the first two sit exactly on a
    quadrature point and on a force point (r = 0 in the kernel)."""
    X = host["X"]
    lo, hi = X.min(axis=1), X.max(axis=1)
    span = np.maximum(hi - lo, 0.05)
    y = (lo - 0.1 * span)[:, None] + rng.random((3, P)) * (1.2 * span)[:, None]
    if P > 0:
        y[:, 0] = X[:, rng.integers(X.shape[1])]
    if P > 1:
        y[:, 1] = host["x"][:, rng.integers(host["x"].shape[1])]
    return np.ascontiguousarray(y)


def _gpu_field(ctx, pb, f, y):
    P = y.shape[1]
    ws = torch.empty(nrs.nrs_field_workspace_size(ctx, P, pb.Q), dtype=torch.uint8, device=DEV)
    u = torch.empty((3, P), dtype=torch.float64, device=DEV)
    nrs.nrs_field_velocity(ctx, pb, T(f), T(y), u, ws)
    return u.cpu().numpy()


SCENES = [
    ("filaments_M5", lambda: synth.filament_scene(5, seed=0)),
    ("sperm_K2_h8", lambda: synth.sperm_channel_scene(2, h=1.0 / 8, seed=1, Nh=30, Qh=300)),
    ("sphere_nc4_nq16", lambda: synth.sphere_scene(4, 16)),
]


@pytest.mark.parametrize("name,mk", SCENES, ids=[s[0] for s in SCENES])
@pytest.mark.parametrize("P", [1, 7, 64, 65, 300])
def test_field_velocity_matches_oracle(ctx, name, mk, P):
    scene = mk()
    print(f"field parity {name} P={P}", flush=True)
    pb, host = prepare(scene)
    rng = np.random.default_rng(P)
    f = rng.normal(size=(3, scene["N"]))
    y = _field_points(rng, host, P)
    u = _gpu_field(ctx, pb, f, y)
    ref = oracle.field_velocity(y, host["X"], host["w"], host["nu"], f, scene["eps"], scene["mu"])
    bound = _abs_bound(y, host["X"], host["w"], host["nu"], f, scene["eps"], scene["mu"])
    assert np.all(np.abs(u - ref) <= 1e-13 * bound[None, :]), np.max(np.abs(u - ref) / bound)


def test_field_of_solved_forces_reproduces_boundary_velocity(ctx):
    """At the force points the field of the solved forces is the prescribed
    velocity plus the rigid motion (the velocity rows of the system)."""
    scene = synth.filament_scene(5, seed=2)
    pb, host = prepare(scene)
    sol, info = gpu_solve(ctx, scene, pb, host, nrs.NRS_FP64_LU)
    N = scene["N"]
    f = sol[:3 * N].reshape(3, N)
    UW = sol[3 * N:].reshape(-1, 6)
    u = _gpu_field(ctx, pb, f, host["x"])
    want = host["u"].copy()
    for m in range(N):
        b = scene["body"][m]
        r = host["x"][:, m] - scene["Y0"][b, :3]
        want[:, m] += UW[b, :3] + np.cross(UW[b, 3:], r)
    assert np.abs(u - want).max() <= 1e-10 * np.abs(want).max()


def test_field_full_size_sampled(ctx):
    """Tracer-grid workload at full size (K = 10 sperm in the 4 x 1 x 0.5
    channel, wall spacing 1/16, 806 tracers on a 26 x 31 grid in the
    mid-plane): every tracer on the GPU, a seeded sample of 24 by the oracle."""
    scene = synth.sperm_channel_scene(10, h=1.0 / 16, seed=0)
    print(f"field full size N={scene['N']} Q={scene['Q']}", flush=True)
    pb, host = prepare(scene)
    rng = np.random.default_rng(5)
    f = rng.normal(size=(3, scene["N"]))
    y = synth.tracer_grid(26, 31, (-1.9, 1.9), (-0.45, 0.45), 0.0)
    u = _gpu_field(ctx, pb, f, y)
    assert np.all(np.isfinite(u))
    pick = np.sort(rng.choice(y.shape[1], 24, replace=False))
    ys = np.ascontiguousarray(y[:, pick])
    ref = oracle.field_velocity(ys, host["X"], host["w"], host["nu"], f, scene["eps"], scene["mu"])
    bound = _abs_bound(ys, host["X"], host["w"], host["nu"], f, scene["eps"], scene["mu"])
    assert np.all(np.abs(u[:, pick] - ref) <= 1e-13 * bound[None, :])


def test_field_edge_cases(ctx):
    scene = synth.filament_scene(2, seed=4)
    pb, host = prepare(scene)
    rng = np.random.default_rng(9)
    f = rng.normal(size=(3, scene["N"]))
    y = _field_points(rng, host, 33)
    # repeated calls give identical bits; u may alias y
    u1 = _gpu_field(ctx, pb, f, y)
    u2 = _gpu_field(ctx, pb, f, y)
    np.testing.assert_array_equal(u1, u2)
    ws = torch.empty(nrs.nrs_field_workspace_size(ctx, 33, pb.Q), dtype=torch.uint8, device=DEV)
    yd = T(y)
    nrs.nrs_field_velocity(ctx, pb, T(f), yd, yd, ws)
    np.testing.assert_array_equal(yd.cpu().numpy(), u1)
    # P = 0 is a no-op
    empty = torch.empty((3, 0), dtype=torch.float64, device=DEV)
    nrs.nrs_field_velocity(ctx, pb, T(f), empty, empty, ws)
    # quadrature points with nu outside [0, N) contribute nothing; w = NULL means 1
    nu_bad = host["nu"].copy()
    drop = rng.random(scene["Q"]) < 0.3
    nu_bad[drop] = np.where(rng.random(drop.sum()) < 0.5, -1, scene["N"] + 5)
    bad = nrs.Problem(pb.x, pb.X, None, T(nu_bad, torch.int32), pb.body, pb.Y, pb.eps, pb.mu)
    u = _gpu_field(ctx, bad, f, y)
    keep = ~drop
    ref = oracle.field_velocity(y, host["X"][:, keep], np.ones(keep.sum()), host["nu"][keep], f,
                                scene["eps"], scene["mu"])
    bound = _abs_bound(y, host["X"][:, keep], np.ones(keep.sum()), host["nu"][keep], f,
                       scene["eps"], scene["mu"])
    assert np.all(np.abs(u - ref) <= 1e-13 * bound[None, :])
    # errors
    with pytest.raises(nrs.NrsError, match="workspace"):
        nrs.nrs_field_velocity(ctx, pb, T(f), T(y), T(y), ws[:100])
    with pytest.raises(nrs.NrsError, match="invalid argument"):
        nrs.nrs_field_velocity(ctx, nrs.Problem(pb.x, pb.X, pb.w, pb.nu, pb.body, pb.Y, 0.0, 1.0),
                               T(f), T(y), T(y), ws)


def _flow(scene, t, Y, f_scale, rng):
    x, X, w, _ = oracle.geometry(scene, t, Y)
    nu = oracle.nearest(x, X, scene["group_off"], scene["groupX"])
    f = f_scale * rng.normal(size=(3, scene["N"]))
    host = dict(X=X, w=w, nu=nu, f=f, eps=scene["eps"], mu=scene["mu"])
    pb = nrs.Problem(T(x), T(X), T(w), T(nu, torch.int32), T(scene["body"], torch.int32),
                     T(Y), scene["eps"], scene["mu"])
    return pb, host


def test_tracer_rk4_step_matches_oracle(ctx):
    """Three precomputed flows (geometry at t, t + dt/2, t + dt, different
    forces) and 150 tracers, three steps."""
    scene = synth.filament_scene(5, seed=1)
    rng = np.random.default_rng(21)
    P = 150
    y0 = rng.normal(size=(3, P)) * 1.2
    yd = T(y0)
    yo = y0.copy()
    dt = 0.05
    ws = torch.empty(nrs.nrs_field_workspace_size(ctx, P, scene["Q"]), dtype=torch.uint8,
                     device=DEV)
    for step in range(3):
        t = step * dt
        flows = [_flow(scene, tt, scene["Y0"], 0.2, rng) for tt in (t, t + dt / 2, t + dt)]
        nrs.nrs_tracer_rk4_step(ctx, [fl[0] for fl in flows], [T(fl[1]["f"]) for fl in flows],
                                yd, dt, ws)
        yo = oracle.tracer_rk4_step([fl[1] for fl in flows], yo, dt)
    err = np.abs(yd.cpu().numpy() - yo).max()
    assert err <= 1e-12, err
    assert np.abs(yo - y0).max() > 1e-3   # the tracers did move


@pytest.mark.parametrize("method", ["FP64_LU", "FP32_IR"])
def test_rk4_step_tracers_matches_oracle(ctx, method):
    """Swimmers and tracers stepped together: the swimmer states equal
    nrs_rk4_step's bit for bit, the tracers match the oracle."""
    scene = synth.filament_scene(5, seed=0)
    ds = nrs.DeviceScene(scene)
    m = getattr(nrs, "NRS_" + method)
    P = 70
    rng = np.random.default_rng(3)
    y0 = scene["Y0"][:, :3].mean(axis=0)[:, None] + rng.normal(size=(3, P))
    ws = torch.empty(nrs.nrs_rk4_tracers_workspace_size(ctx, ds, m, P), dtype=torch.uint8,
                     device=DEV)
    ws0 = torch.empty(nrs.nrs_rk4_workspace_size(ctx, ds, m), dtype=torch.uint8, device=DEV)
    Y, Y0 = T(scene["Y0"]), T(scene["Y0"])
    yd = T(y0)
    Yo, yo = scene["Y0"].copy(), y0.copy()
    dt = 2 * math.pi / 100
    for step in range(2):
        nrs.nrs_rk4_step_tracers(ctx, ds, Y, yd, step * dt, dt, ws, method=m)
        nrs.nrs_rk4_step(ctx, ds, Y0, step * dt, dt, ws0, method=m)
        Yo, yo = oracle.rk4_step_tracers(scene, Yo, yo, step * dt, dt)
    info = nrs.nrs_query_info(ctx, ws)
    assert info["fell_back"] == 0
    np.testing.assert_array_equal(Y.cpu().numpy(), Y0.cpu().numpy())
    assert np.max(np.abs(Y.cpu().numpy().reshape(-1, 12) - Yo)) <= 1e-10
    err = np.abs(yd.cpu().numpy() - yo).max()
    assert err <= 1e-10, err
