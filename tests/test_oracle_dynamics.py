"""Pins of the oracle's geometry evaluation and RK4 time stepping (Sec. 4:
state Y = [X0; B], Y' = F(Y, t))."""
import math

import numpy as np
from scipy.integrate import quad

import oracle
import synth


def test_filament_weights_integrate_arc_length():
    """Sum of the filament quadrature weights = arc length of
    (s - 1/2, 0.1 sin(2 pi s - t), 0) by adaptive quadrature."""
    sc = synth.filament_scene(M=1, seed=0)
    for t in (0.0, 1.3):
        _, _, w, _ = oracle.geometry(sc, t, sc["Y0"])
        L, _ = quad(lambda s: math.sqrt(1 + (0.2 * math.pi * math.cos(2 * math.pi * s - t)) ** 2), 0, 1)
        assert abs(w.sum() - L) < 1e-5


def test_geometry_rigid_placement_and_velocity():
    """x = x0 + B xi keeps body-frame distances; u equals the time derivative
    of the lab-frame positions (central differences)."""
    sc = synth.filament_scene(M=3, seed=2)
    Y = sc["Y0"]
    t, h = 0.7, 1e-5
    x, _, _, u = oracle.geometry(sc, t, Y)
    xp, _, _, _ = oracle.geometry(sc, t + h, Y)
    xm, _, _, _ = oracle.geometry(sc, t - h, Y)
    np.testing.assert_allclose(u, (xp - xm) / (2 * h), atol=1e-8)
    sel = sc["body"] == 1
    B = Y[1, 3:].reshape(3, 3)
    np.testing.assert_allclose(B.T @ B, np.eye(3), atol=1e-14)
    d_lab = np.linalg.norm(x[:, sel][:, :, None] - x[:, sel][:, None, :], axis=0)
    xi0 = oracle.geometry(dict(sc, body=np.full_like(sc["body"], -1),
                               bodyX=np.full_like(sc["bodyX"], -1)), t, Y)[0]
    d_body = np.linalg.norm(xi0[:, sel][:, :, None] - xi0[:, sel][:, None, :], axis=0)
    np.testing.assert_allclose(d_lab, d_body, atol=1e-13)


def test_rk4_order_on_linear_ode():
    errs = []
    for n in (10, 20, 40):
        y = np.array([1.0, 0.0])
        Aode = np.array([[0.0, 1.0], [-1.0, 0.0]])
        dt = 1.0 / n
        for i in range(n):
            y = oracle.rk4_generic(lambda v, t: Aode @ v, y, i * dt, dt)
        errs.append(np.linalg.norm(y - np.array([math.cos(1.0), -math.sin(1.0)])))
    assert 14 < errs[0] / errs[1] < 18 and 14 < errs[1] / errs[2] < 18


def test_rotation_rates_match_rodrigues():
    """Constant Omega: RK4 on dB/dt = [Omega]x B tends to exp(t[Omega]x) B0 at
    fourth order."""
    Om = np.array([0.3, -0.5, 0.8])
    th = np.linalg.norm(Om)
    k = Om / th
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    T = 2.0
    Rex = np.eye(3) + math.sin(th * T) * K + (1 - math.cos(th * T)) * K @ K
    UW = np.concatenate([np.zeros(3), Om])[None, :]
    errs = []
    for n in (8, 16):
        Y = np.concatenate([np.zeros(3), np.eye(3).ravel()])[None, :]
        dt = T / n
        for i in range(n):
            Y = oracle.rk4_generic(lambda y, t: oracle.rates(y, UW), Y, i * dt, dt)
        errs.append(np.abs(Y[0, 3:].reshape(3, 3) - Rex).max())
    assert errs[1] < 1e-4 and 12 < errs[0] / errs[1] < 20


def test_orthonormalise():
    rng = np.random.default_rng(0)
    Y = np.concatenate([np.zeros(3), (np.eye(3) + 1e-3 * rng.normal(size=(3, 3))).ravel()])[None, :]
    Z = oracle.orthonormalise(Y)
    B = Z[0, 3:].reshape(3, 3)
    np.testing.assert_allclose(B.T @ B, np.eye(3), atol=1e-15)
    R = synth.random_rotation(rng)
    Yr = np.concatenate([np.ones(3), R.ravel()])[None, :]
    np.testing.assert_allclose(oracle.orthonormalise(Yr), Yr, atol=1e-15)


def test_zero_beat_swimmer_stays_at_rest():
    sc = synth.filament_scene(M=2, seed=1, Nf=10, Qf=60, amp=0.0)
    Y1 = oracle.rk4_step(sc, sc["Y0"], 0.0, 0.1)
    np.testing.assert_allclose(Y1, sc["Y0"], atol=1e-14)


def test_swimmer_moves_and_is_force_free():
    sc = synth.filament_scene(M=1, seed=0, Nf=20, Qf=200)
    f, UW, d = oracle.solve_scene(sc, 0.4, return_all=True)
    F = (d["W"][None, :] * f).sum(axis=1)
    assert np.abs(F).max() < 1e-10 * np.abs(d["W"][None, :] * f).sum()
    assert np.linalg.norm(UW[0, :3]) > 1e-4
