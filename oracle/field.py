"""Plain FP64 reference of the flow at field points and of passive tracer
advection.  Test infrastructure only (see the package docstring).

The regularized single-layer equation of Sec. 3 (eq. 19) gives the velocity
at any point of the fluid, not only on the boundary; with the nearest-
neighbour discretisation (eq. 23) the velocity at a field point y is

    u_j(y) = (8 pi mu)^-1 sum_q S^eps_jk(y - X_q) w_q f_k[nu(q)],

the same sum that gives the collocation rows of A_s, with x_m replaced by y.
Tracers (the particle-tracking experiments of Sec. 4.3 and Sec. 5.2) are
carried by that flow: dy/dt = u(y, t).

Readings adopted here:
  * the flow at time t is the one defined by the geometry and the force
    densities of the solve at t; tracers do not act on the fluid;
  * tracer positions are integrated with the same classical RK4 as the
    swimmers.  With precomputed flows (forces known in advance, as in the
    node experiment) the two middle stages both use the flow at t + dt/2;
    coupled to the swimmers, each stage uses the flow of that stage's solve.
"""
from __future__ import annotations

import math

import numpy as np

from .core import (stokeslet_reg, solve_scene, rates, orthonormalise)


def field_velocity(y, X, w, nu, f, eps, mu, chunk=4096):
    """u (3, P) at field points y (3, P): the nearest-neighbour sum of
    Sec. 3 eq. 23 evaluated at y instead of a collocation point.  X (3, Q),
    w (Q,), nu (Q,) nearest force point of each quadrature point, f (3, N)
    force densities.  The Q dimension is taken in blocks of `chunk`."""
    y = np.asarray(y, dtype=np.float64).reshape(3, -1)
    X = np.asarray(X, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64).reshape(3, -1)
    P, Q = y.shape[1], X.shape[1]
    u = np.zeros((3, P))
    for q0 in range(0, Q, chunk):
        q1 = min(Q, q0 + chunk)
        g = f[:, nu[q0:q1]] * w[None, q0:q1]                       # (3, Qc)
        r = (y[:, :, None] - X[:, None, q0:q1]).transpose(1, 2, 0)  # (P, Qc, 3)
        S = stokeslet_reg(r, eps)                                   # (P, Qc, 3, 3)
        u += np.einsum("pqjk,kq->jp", S, g)
    return u / (8.0 * math.pi * mu)


def flow_of(problem):
    """Right-hand side u(y) of dy/dt for one frozen flow: a dict with keys
    X, w, nu, f, eps, mu."""
    return lambda y: field_velocity(y, problem["X"], problem["w"], problem["nu"],
                                    problem["f"], problem["eps"], problem["mu"])


def tracer_rk4_step(flows, y, dt):
    """One classical RK4 step of tracers y (3, P) through precomputed flows
    at t, t + dt/2 and t + dt (flows[0..2], dicts as in flow_of)."""
    u0, uh, u1 = (flow_of(p) for p in flows)
    y = np.asarray(y, dtype=np.float64).reshape(3, -1)
    k1 = u0(y)
    k2 = uh(y + 0.5 * dt * k1)
    k3 = uh(y + 0.5 * dt * k2)
    k4 = u1(y + dt * k3)
    return y + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def coupled_rates(scene, Y, ytr, t):
    """Rates of the swimmer states and of the tracers at one stage: solve
    the swimming problem at (Y, t), then evaluate its flow at the tracers."""
    M = scene["M"]
    f, UW, d = solve_scene(scene, t, np.asarray(Y).reshape(M, 12), return_all=True)
    dY = rates(np.asarray(Y).reshape(M, 12), UW)
    dy = field_velocity(ytr, d["X"], d["w"], d["nu"], f, scene["eps"], scene["mu"])
    return dY, dy


def rk4_step_tracers(scene, Y, ytr, t, dt):
    """One RK4 step of the swimmers and the tracers together: the state is
    [Y; y], every stage solves the swimming problem and moves the tracers
    with that stage's flow; the body frames (not the tracers) are then
    re-orthonormalised as in rk4_step."""
    M = scene["M"]
    Y = np.asarray(Y, dtype=np.float64).reshape(M, 12)
    y = np.asarray(ytr, dtype=np.float64).reshape(3, -1)
    a1, b1 = coupled_rates(scene, Y, y, t)
    a2, b2 = coupled_rates(scene, Y + 0.5 * dt * a1, y + 0.5 * dt * b1, t + 0.5 * dt)
    a3, b3 = coupled_rates(scene, Y + 0.5 * dt * a2, y + 0.5 * dt * b2, t + 0.5 * dt)
    a4, b4 = coupled_rates(scene, Y + dt * a3, y + dt * b3, t + dt)
    Yn = Y + (dt / 6.0) * (a1 + 2.0 * a2 + 2.0 * a3 + a4)
    yn = y + (dt / 6.0) * (b1 + 2.0 * b2 + 2.0 * b3 + b4)
    return orthonormalise(Yn), yn
