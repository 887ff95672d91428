"""Pins of the warm-start network reference (oracle.mlp) and of the GMRES
reference (oracle.gmres), independent of how they are written:
  - gradients against central finite differences in FP64;
  - special cases that reduce to a plainer formula (zero weights, a body of
    one point, duplicated points under mean pooling);
  - invariance of the features / equivariance of the warm start under a rigid
    motion of the whole configuration;
  - Adam's closed form under a constant gradient;
  - a training run that fits a teacher network of the same architecture;
  - GMRES: exact solution of small systems, convergence in k iterations for
    a matrix with k distinct eigenvalues, and the effect of a warm start.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp

H = 8


def _data(seed, sizes=(5, 3, 7)):
    rng = np.random.default_rng(seed)
    off = np.concatenate([[0], np.cumsum(sizes)])
    N = off[-1]
    phi = rng.normal(size=(N, mlp.F_IN))
    theta = 0.5 * rng.normal(size=mlp.param_count(H))
    t_pt = rng.normal(size=(N, 3))
    t_b = rng.normal(size=(len(sizes), 6))
    return theta, phi, off, t_pt, t_b


def test_param_count():
    assert mlp.param_count(H) == H * 7 + H + 2 * H * H + H + 3 * H + 3 + 6 * H + 6


def test_gradient_matches_central_differences():
    theta, phi, off, t_pt, t_b = _data(0)
    L, g = mlp.gradient(theta, H, phi, off, t_pt, t_b)
    assert L == pytest.approx(mlp.loss(theta, H, phi, off, t_pt, t_b), rel=1e-15)
    h = 1e-6
    fd = np.empty_like(theta)
    for i in range(len(theta)):
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd[i] = (mlp.loss(tp, H, phi, off, t_pt, t_b) - mlp.loss(tm, H, phi, off, t_pt, t_b)) / (2 * h)
    # every parameter group is exercised
    assert np.all(np.abs(g) > 0) or np.count_nonzero(g) > 0.95 * len(g)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9)


def test_zero_weights_give_biases():
    theta, phi, off, _, _ = _data(1)
    p = mlp.unflatten(theta, H)
    for k in ("W1", "W2", "V2", "W3", "W4"):
        p[k] = np.zeros_like(p[k])
    y, z = mlp.forward(mlp.flatten(p, H), H, phi, off)
    np.testing.assert_array_equal(y, np.broadcast_to(p["b3"], y.shape))
    np.testing.assert_array_equal(z, np.broadcast_to(p["b4"], z.shape))


def test_single_point_body_is_a_plain_two_layer_network():
    """With one point the pooled context equals the point's own hidden state,
    so the network is y = W3 tanh((W2 + V2) tanh(W1 phi + b1) + b2) + b3 and
    z = W4 tanh(...) + b4."""
    theta, phi, _, _, _ = _data(2, sizes=(1,))
    p = mlp.unflatten(theta, H)
    y, z = mlp.forward(theta, H, phi, np.array([0, 1]))
    h = np.tanh((p["W2"] + p["V2"]) @ np.tanh(p["W1"] @ phi[0] + p["b1"]) + p["b2"])
    np.testing.assert_allclose(y[0], p["W3"] @ h + p["b3"], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(z[0], p["W4"] @ h + p["b4"], rtol=1e-13, atol=1e-15)


def test_permutation_and_duplication_within_a_body():
    theta, phi, off, _, _ = _data(3, sizes=(6,))
    y, z = mlp.forward(theta, H, phi, off)
    perm = np.random.default_rng(0).permutation(6)
    yp, zp = mlp.forward(theta, H, phi[perm], off)
    np.testing.assert_allclose(yp, y[perm], rtol=1e-13)
    np.testing.assert_allclose(zp, z, rtol=1e-13)
    # mean pooling: every point twice leaves every output unchanged
    yd, zd = mlp.forward(theta, H, np.repeat(phi, 2, axis=0), np.array([0, 12]))
    np.testing.assert_allclose(yd[::2], y, rtol=1e-13)
    np.testing.assert_allclose(zd, z, rtol=1e-13)


def _rotation(seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def test_features_invariant_and_warm_start_equivariant_under_rigid_motion():
    rng = np.random.default_rng(4)
    off = np.array([0, 4, 9])
    N, M = 9, 2
    x = rng.normal(size=(3, N))
    u = rng.normal(size=(3, N))
    s = rng.random(N)
    Y = np.zeros((M, 12))
    for b in range(M):
        Y[b, :3] = rng.normal(size=3)
        Y[b, 3:] = _rotation(10 + b).ravel()
    R, a = _rotation(99), rng.normal(size=3)
    Y2 = Y.copy()
    for b in range(M):
        Y2[b, :3] = R @ Y[b, :3] + a
        Y2[b, 3:] = (R @ Y[b, 3:].reshape(3, 3)).ravel()
    phi = mlp.features(x, u, s, Y, off)
    phi2 = mlp.features(R @ x + a[:, None], R @ u, s, Y2, off)
    np.testing.assert_allclose(phi2, phi, atol=1e-13)
    # the body frame of a point at x0 + B e_k is e_k
    e = mlp.features((Y[0, :3][:, None] + Y[0, 3:].reshape(3, 3)), np.zeros((3, 3)),
                     np.zeros(3), Y[:1], np.array([0, 3]))
    np.testing.assert_allclose(e[:, :3], np.eye(3), atol=1e-14)
    y = rng.normal(size=(N, 3))
    z = rng.normal(size=(M, 6))
    sc = (2.0, 3.0, 5.0)
    w1 = mlp.warm_start(y, z, Y, off, sc)
    w2 = mlp.warm_start(y, z, Y2, off, sc)
    f1, f2 = w1[:3 * N].reshape(3, N), w2[:3 * N].reshape(3, N)
    np.testing.assert_allclose(f2, R @ f1, atol=1e-13)
    g1, g2 = w1[3 * N:].reshape(M, 6), w2[3 * N:].reshape(M, 6)
    np.testing.assert_allclose(g2[:, :3], g1[:, :3] @ R.T, atol=1e-13)
    np.testing.assert_allclose(g2[:, 3:], g1[:, 3:] @ R.T, atol=1e-13)
    # targets() inverts warm_start()
    t_pt, t_b = mlp.targets(f1, g1, Y, off, sc)
    np.testing.assert_allclose(t_pt, y, atol=1e-13)
    np.testing.assert_allclose(t_b, z, atol=1e-13)


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the bias-corrected moments are g and g^2 at
    every step, so each step moves theta by -lr g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    theta = np.array([1.0, 2.0, 3.0, 4.0])
    m = np.zeros(4)
    v = np.zeros(4)
    lr, eps = 0.01, 1e-8
    th = theta.copy()
    for t in range(1, 6):
        th, m, v = mlp.adam_step(th, g, m, v, t, lr, eps=eps)
        np.testing.assert_allclose(th, theta - t * lr * g / (np.abs(g) + eps), rtol=1e-12)


def test_training_fits_a_teacher_network():
    rng = np.random.default_rng(5)
    sizes = [6] * 10
    off = np.concatenate([[0], np.cumsum(sizes)])
    phi = rng.normal(size=(off[-1], mlp.F_IN))
    teacher = 0.7 * rng.normal(size=mlp.param_count(H))
    t_pt, t_b = mlp.forward(teacher, H, phi, off)
    theta = 0.1 * rng.normal(size=mlp.param_count(H))
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    L0 = mlp.loss(theta, H, phi, off, t_pt, t_b)
    for t in range(1, 401):
        L, g = mlp.gradient(theta, H, phi, off, t_pt, t_b)
        theta, m, v = mlp.adam_step(theta, g, m, v, t, 0.01)
    assert mlp.loss(theta, H, phi, off, t_pt, t_b) < 0.05 * L0


# ---------------------------------------------------------------- GMRES pins

def test_gmres_solves_small_systems():
    rng = np.random.default_rng(6)
    A = rng.normal(size=(40, 40)) + 8 * np.eye(40)
    b = rng.normal(size=40)
    x, it, rr = oracle.gmres(A, b, tol=1e-12, restart=15)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-9, atol=1e-12)
    assert rr <= 1e-12 and it > 15   # restarted at least once


def test_gmres_k_distinct_eigenvalues_converges_in_k_steps():
    """The Krylov space of a diagonalisable matrix with k distinct eigenvalues
    contains the solution after k steps."""
    rng = np.random.default_rng(7)
    lam = np.repeat([1.0, 2.5, -3.0, 7.0], 10)
    V = np.linalg.qr(rng.normal(size=(40, 40)))[0]
    A = V @ np.diag(lam) @ V.T
    b = rng.normal(size=40)
    x, it, rr = oracle.gmres(A, b, tol=1e-11, restart=30)
    assert it == 4 and rr <= 1e-11
    np.testing.assert_allclose(A @ x, b, atol=1e-9)


def test_gmres_warm_start_at_solution_takes_no_step():
    rng = np.random.default_rng(8)
    A = rng.normal(size=(20, 20)) + 5 * np.eye(20)
    b = rng.normal(size=20)
    xs = np.linalg.solve(A, b)
    x, it, rr = oracle.gmres(A, b, x0=xs, tol=1e-8)
    assert it == 0 and rr <= 1e-8
    x, it, _ = oracle.gmres(A, b, tol=1e-8)
    assert it > 0 and math.isfinite(it)
