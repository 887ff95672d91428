"""Pins of the field-point velocity and tracer oracles (oracle/field.py)
against textbook Stokes flows, asymptotics, the solve's own boundary rows,
and an independent adaptive integrator."""
import math

import numpy as np
from scipy.integrate import solve_ivp

import oracle
import oracle.field
import synth


def _flow(sc):
    f, UW, d = oracle.solve_scene(sc, return_all=True)
    return f, UW, d


def _random_dirs(rng, k):
    v = rng.normal(size=(3, k))
    return v / np.linalg.norm(v, axis=0)


def test_translating_sphere_exterior_field():
    """Outside a sphere of radius a translating at U the exact Stokes flow
    is (3a/4)(U/r + (U.y)y/r^3) + (a^3/4)(U/r^3 - 3(U.y)y/r^5) (Stokes'
    solution: a stokeslet plus a source dipole).  The discretised field
    agrees to the method's O(eps + h) error, which falls with refinement."""
    rng = np.random.default_rng(1)
    dirs = _random_dirs(rng, 12)
    U = np.array([1.0, 0.0, 0.0])
    errs = []
    for nc, nq in ((4, 16), (6, 24)):
        sc = synth.sphere_scene(nc, nq, eps=0.01, U=U)
        f, _, d = _flow(sc)
        worst = 0.0
        for R in (1.5, 3.0):
            y = dirs * R
            u = oracle.field_velocity(y, d["X"], d["w"], d["nu"], f, sc["eps"], sc["mu"])
            r = np.linalg.norm(y, axis=0)
            Uy = U @ y
            ex = (0.75 * (U[:, None] / r + Uy * y / r ** 3)
                  + 0.25 * (U[:, None] / r ** 3 - 3 * Uy * y / r ** 5))
            worst = max(worst, np.abs(u - ex).max() / np.abs(ex).max())
        errs.append(worst)
    assert errs[0] < 0.02 and errs[1] < errs[0]


def test_rotating_sphere_exterior_field():
    """A sphere rotating at Omega drives u = (a/r)^3 Omega x y outside."""
    sc = synth.sphere_scene(6, 24, eps=0.01, U=(0, 0, 0), Omega=(0.0, 0.0, 1.0))
    f, _, d = _flow(sc)
    y = _random_dirs(np.random.default_rng(2), 10) * 2.0
    u = oracle.field_velocity(y, d["X"], d["w"], d["nu"], f, sc["eps"], sc["mu"])
    ex = np.cross(np.array([0.0, 0.0, 1.0])[None, :], y.T).T / 8.0
    assert np.abs(u - ex).max() / np.abs(ex).max() < 0.03


def test_field_at_collocation_points_reproduces_boundary_velocity():
    """At a force point x_m the field sum is row m of A_s f, so the solved
    forces give back the point's velocity: the prescribed u_m on fixed
    points, u_m + U + Omega x r_m on a free swimmer (Sec. 4)."""
    sc = synth.filament_scene(M=2, seed=5, Nf=24, Qf=240)
    f, UW, d = _flow(sc)
    u = oracle.field_velocity(d["x"], d["X"], d["w"], d["nu"], f, sc["eps"], sc["mu"])
    want = d["u"].copy()
    Y = sc["Y0"]
    for m in range(sc["N"]):
        b = sc["body"][m]
        r = d["x"][:, m] - Y[b, :3]
        want[:, m] += UW[b, :3] + np.cross(UW[b, 3:], r)
    assert np.abs(u - want).max() < 1e-9 * np.abs(want).max()

    sph = synth.sphere_scene(4, 16, eps=0.01, U=(0.3, -0.2, 0.5))
    f, _, d = _flow(sph)
    u = oracle.field_velocity(d["x"], d["X"], d["w"], d["nu"], f, sph["eps"], sph["mu"])
    assert np.abs(u - d["u"]).max() < 1e-12


def test_far_field_is_a_stokeslet_of_the_total_force():
    """Far from the body the flow is that of a point force F = sum_q w_q f:
    u ~ (8 pi mu)^-1 (I + e e^T) F / R, relative error O(size / R)."""
    sc = synth.filament_scene(M=1, seed=7, Nf=20, Qf=200)
    x, X, w, _ = oracle.geometry(sc, 0.0, sc["Y0"])
    nu = oracle.nearest(x, X, sc["group_off"], sc["groupX"])
    rng = np.random.default_rng(3)
    f = rng.normal(size=(3, sc["N"]))
    F = (f[:, nu] * w[None, :]).sum(axis=1)
    centre = sc["Y0"][0, :3]
    for R in (1e3, 1e4):
        e = _random_dirs(rng, 1)[:, 0]
        u = oracle.field_velocity((centre + R * e)[:, None], X, w, nu, f, sc["eps"], 2.0)[:, 0]
        ex = (F + e * (e @ F)) / (8 * math.pi * 2.0 * R)
        assert np.linalg.norm(u - ex) / np.linalg.norm(ex) < 5.0 / R


def test_field_on_a_quadrature_point_is_the_regularized_core():
    """At r = 0 the regularized stokeslet is (2/eps) I (eq. 18), so a single
    quadrature point gives u = (8 pi mu)^-1 (2/eps) w f at its own position."""
    X = np.array([[0.3], [-0.1], [0.7]])
    f = np.array([[1.5], [-2.0], [0.25]])
    u = oracle.field_velocity(X, X, np.array([0.4]), np.array([0]), f, 0.05, 1.3)
    assert np.allclose(u[:, 0], 0.4 * f[:, 0] * 2 / 0.05 / (8 * math.pi * 1.3), rtol=1e-14)


def test_field_is_translation_and_rotation_equivariant():
    rng = np.random.default_rng(11)
    X = rng.normal(size=(3, 30))
    w = rng.random(30)
    nu = rng.integers(0, 6, size=30)
    f = rng.normal(size=(3, 6))
    y = rng.normal(size=(3, 9))
    u = oracle.field_velocity(y, X, w, nu, f, 0.1, 1.0)
    s = rng.normal(size=(3, 1))
    assert np.allclose(oracle.field_velocity(y + s, X + s, w, nu, f, 0.1, 1.0), u, atol=1e-13)
    R = synth.random_rotation(rng)
    uR = oracle.field_velocity(R @ y, R @ X, w, nu, R @ f, 0.1, 1.0)
    assert np.allclose(uR, R @ u, atol=1e-13)


def _sphere_flow():
    sc = synth.sphere_scene(4, 16, eps=0.01, U=(0, 0, 0), Omega=(0.0, 0.0, 1.0))
    f, _, d = _flow(sc)
    return dict(X=d["X"], w=d["w"], nu=d["nu"], f=f, eps=sc["eps"], mu=sc["mu"])


def test_tracer_rk4_is_fourth_order_against_an_adaptive_integrator():
    """Tracers in an unsteady flow (the rotating-sphere flow scaled by
    a(t) = 1 + 0.8 sin 3t): classical RK4 with the flows at t, t + dt/2 and
    t + dt converges at fourth order to a tight Dormand-Prince (DOP853)
    solution of dy/dt = a(t) u(y)."""
    fl = _sphere_flow()
    a = lambda t: 1.0 + 0.8 * math.sin(3.0 * t)  # noqa: E731
    rng = np.random.default_rng(4)
    y0 = _random_dirs(rng, 5) * 1.6

    def scaled(t):
        g = dict(fl)
        g["f"] = a(t) * fl["f"]
        return g

    def rhs(t, v):
        return oracle.field.flow_of(scaled(t))(v.reshape(3, -1)).ravel()

    T = 1.0
    ref = solve_ivp(rhs, (0.0, T), y0.ravel(), method="DOP853",
                    rtol=1e-12, atol=1e-14).y[:, -1].reshape(3, -1)
    errs = []
    for steps in (4, 8, 16):
        dt = T / steps
        y = y0.copy()
        for i in range(steps):
            t = i * dt
            y = oracle.tracer_rk4_step([scaled(t), scaled(t + dt / 2), scaled(t + dt)], y, dt)
        errs.append(np.abs(y - ref).max())
    assert errs[-1] < 1e-7
    for e0, e1 in zip(errs, errs[1:]):
        assert 12.0 < e0 / e1 < 20.0


def test_coupled_swimmer_and_tracer_step():
    """[Y; y] stepped together: the swimmer part is rk4_step's, and the
    tracers converge at fourth order to DOP853 on the coupled system."""
    sc = synth.filament_scene(M=2, seed=3, Nf=20, Qf=200)
    M = sc["M"]
    y0 = np.random.default_rng(2).normal(size=(3, 4)) * 0.8
    Y1, _ = oracle.rk4_step_tracers(sc, sc["Y0"], y0, 0.0, 0.1)
    assert np.array_equal(Y1, oracle.rk4_step(sc, sc["Y0"], 0.0, 0.1))

    def rhs(t, v):
        dY, dy = oracle.field.coupled_rates(sc, v[:12 * M].reshape(M, 12),
                                            v[12 * M:].reshape(3, -1), t)
        return np.concatenate([dY.ravel(), dy.ravel()])

    T = 0.4
    sol = solve_ivp(rhs, (0.0, T), np.concatenate([sc["Y0"].ravel(), y0.ravel()]),
                    method="DOP853", rtol=1e-11, atol=1e-13)
    ref = sol.y[12 * M:, -1].reshape(3, -1)
    errs = []
    for steps in (2, 4, 8):
        dt = T / steps
        Y, y = sc["Y0"].copy(), y0.copy()
        for i in range(steps):
            Y, y = oracle.rk4_step_tracers(sc, Y, y, i * dt, dt)
        errs.append(np.abs(y - ref).max())
    for e0, e1 in zip(errs, errs[1:]):
        assert 10.0 < e0 / e1 < 22.0
