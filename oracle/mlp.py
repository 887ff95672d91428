"""FP64 reference of the learned warm-start network (test infrastructure).

TEST INFRASTRUCTURE ONLY: used by tests/ to check the HIP forward, backward
and Adam kernels and the warm-start mapping; the product path never imports
it.

The paper has no learned component; this follows the warm-start design of
the hot path: a per-point network with pooled body context that maps, for
each force point of a free body, body-frame features to a body-frame force
density, and for each body its body-frame (U, Omega).  Its gradients are
pinned by central finite differences and its invariances by rotation,
permutation and duplication tests; the quality of its predictions has no
pin ("parity unpinned": the GMRES residual judges a prediction).

Model (H hidden units, F = 7 inputs, O = 3 point outputs, P = 6 body outputs),
for body s with points m = 1..n_s:
    h1_m = tanh(W1 phi_m + b1)
    c_s  = mean_m h1_m
    h2_m = tanh(W2 h1_m + V2 c_s + b2)
    y_m  = W3 h2_m + b3                      (scaled body-frame force density)
    z_s  = W4 mean_m h2_m + b4               (scaled body-frame U, Omega)
Features phi_m = (B^T (x_m - x0), B^T u_m, s_m) with Y = (x0, B) the body
state.  Flat parameter order: W1 (H x F, row-major), b1, W2 (H x H), V2
(H x H), b2, W3 (O x H), b3, W4 (P x H), b4.
"""
from __future__ import annotations

import numpy as np

F_IN, O_PT, P_BODY = 7, 3, 6


def shapes(H):
    return [("W1", (H, F_IN)), ("b1", (H,)), ("W2", (H, H)), ("V2", (H, H)), ("b2", (H,)),
            ("W3", (O_PT, H)), ("b3", (O_PT,)), ("W4", (P_BODY, H)), ("b4", (P_BODY,))]


def param_count(H):
    return int(sum(np.prod(s) for _, s in shapes(H)))


def unflatten(theta, H):
    out, o = {}, 0
    for name, s in shapes(H):
        k = int(np.prod(s))
        out[name] = np.asarray(theta[o:o + k], dtype=np.float64).reshape(s)
        o += k
    return out


def flatten(p, H):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in shapes(H)])


def features(x, u, s, Y, body_off):
    """phi (N, 7) for points grouped by body: body b owns points
    body_off[b] .. body_off[b+1]-1; Y (M, 12) = [x0, B row-major]."""
    N = x.shape[1]
    phi = np.zeros((N, F_IN))
    Y = np.asarray(Y, dtype=np.float64).reshape(-1, 12)
    for b in range(len(body_off) - 1):
        lo, hi = body_off[b], body_off[b + 1]
        x0 = Y[b, :3]
        B = Y[b, 3:].reshape(3, 3)
        phi[lo:hi, 0:3] = (B.T @ (x[:, lo:hi] - x0[:, None])).T
        phi[lo:hi, 3:6] = (B.T @ u[:, lo:hi]).T
        phi[lo:hi, 6] = s[lo:hi]
    return phi


def forward(theta, H, phi, body_off, keep=False):
    """y (N, 3) per point and z (M, 6) per body."""
    p = unflatten(theta, H)
    N = phi.shape[0]
    M = len(body_off) - 1
    y = np.zeros((N, O_PT))
    z = np.zeros((M, P_BODY))
    acts = []
    for b in range(M):
        lo, hi = body_off[b], body_off[b + 1]
        h1 = np.tanh(phi[lo:hi] @ p["W1"].T + p["b1"])
        c = h1.mean(axis=0)
        h2 = np.tanh(h1 @ p["W2"].T + c @ p["V2"].T + p["b2"])
        y[lo:hi] = h2 @ p["W3"].T + p["b3"]
        d = h2.mean(axis=0)
        z[b] = p["W4"] @ d + p["b4"]
        acts.append((h1, c, h2, d))
    return (y, z, acts) if keep else (y, z)


def loss(theta, H, phi, body_off, t_pt, t_body):
    """Mean over bodies of (mean squared error of the body's point outputs +
    mean squared error of its body outputs)."""
    y, z = forward(theta, H, phi, body_off)
    M = len(body_off) - 1
    L = 0.0
    for b in range(M):
        lo, hi = body_off[b], body_off[b + 1]
        L += np.mean((y[lo:hi] - t_pt[lo:hi]) ** 2) + np.mean((z[b] - t_body[b]) ** 2)
    return float(L / M)


def gradient(theta, H, phi, body_off, t_pt, t_body):
    """(loss, dloss/dtheta) by reverse-mode differentiation of forward()."""
    p = unflatten(theta, H)
    y, z, acts = forward(theta, H, phi, body_off, keep=True)
    M = len(body_off) - 1
    L = loss(theta, H, phi, body_off, t_pt, t_body)
    dz = 2.0 * (z - t_body) / (M * P_BODY)
    g = {name: np.zeros(s) for name, s in shapes(H)}
    for b in range(M):
        lo, hi = body_off[b], body_off[b + 1]
        n_b = hi - lo
        h1, c, h2, d = acts[b]
        dyb = 2.0 * (y[lo:hi] - t_pt[lo:hi]) / (M * n_b * O_PT)
        g["W3"] += dyb.T @ h2
        g["b3"] += dyb.sum(axis=0)
        g["W4"] += np.outer(dz[b], d)
        g["b4"] += dz[b]
        dh2 = dyb @ p["W3"] + (p["W4"].T @ dz[b])[None, :] / n_b
        da2 = dh2 * (1.0 - h2 ** 2)
        g["W2"] += da2.T @ h1
        sa2 = da2.sum(axis=0)
        g["V2"] += np.outer(sa2, c)
        g["b2"] += sa2
        dh1 = da2 @ p["W2"] + (p["V2"].T @ sa2)[None, :] / n_b
        da1 = dh1 * (1.0 - h1 ** 2)
        g["W1"] += da1.T @ phi[lo:hi]
        g["b1"] += da1.sum(axis=0)
    return L, flatten(g, H)


def adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015, Algorithm 1) at step t >= 1.
    Returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def targets(f, UW, Y, body_off, scales):
    """Body-frame scaled training targets from a solution: f (3, N) force
    densities, UW (M, 6) lab-frame (U, Omega); scales = (force, U, Omega)."""
    Y = np.asarray(Y, dtype=np.float64).reshape(-1, 12)
    N = f.shape[1]
    M = len(body_off) - 1
    t_pt = np.zeros((N, O_PT))
    t_b = np.zeros((M, P_BODY))
    for b in range(M):
        lo, hi = body_off[b], body_off[b + 1]
        B = Y[b, 3:].reshape(3, 3)
        t_pt[lo:hi] = (B.T @ f[:, lo:hi]).T / scales[0]
        t_b[b, :3] = B.T @ UW[b, :3] / scales[1]
        t_b[b, 3:] = B.T @ UW[b, 3:] / scales[2]
    return t_pt, t_b


def warm_start(y, z, Y, body_off, scales):
    """Lab-frame initial guess [f_x; f_y; f_z; (U, Omega) per body] from the
    network outputs (inverse of targets())."""
    Y = np.asarray(Y, dtype=np.float64).reshape(-1, 12)
    N = y.shape[0]
    M = len(body_off) - 1
    f = np.zeros((3, N))
    UW = np.zeros((M, 6))
    for b in range(M):
        lo, hi = body_off[b], body_off[b + 1]
        B = Y[b, 3:].reshape(3, 3)
        f[:, lo:hi] = scales[0] * (B @ y[lo:hi].T)
        UW[b, :3] = scales[1] * (B @ z[b, :3])
        UW[b, 3:] = scales[2] * (B @ z[b, 3:])
    return np.concatenate([f.ravel(), UW.ravel()])
