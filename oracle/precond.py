"""Oracle of the block-diagonal preconditioner of the GMRES form and of its
learned block model (not part of the paper's method: a preconditioner for the
same linear system of Sec. 4, whose solution the GMRES residual decides).

TEST INFRASTRUCTURE ONLY (see the package docstring).

A free body's block is the square submatrix of the full swimming-problem
matrix (Sec. 2 and Sec. 4: the NEAREST operator of Sec. 3 eq. 23 on the
body's own force points, its rigid-body columns and its force and moment
balance rows) on the body's unknowns, taken in the order
    f_x of its points (increasing index), f_y, f_z, U_x, U_y, U_z, Omega_x,
    Omega_y, Omega_z.
The preconditioner applies the inverse of every body's block to that body's
unknowns and leaves every other unknown unchanged.

The learned model is a least-squares trigonometric fit, in the beat phase
psi, of the inverse block of a single body in its own frame; a body with
frame B then gets R K(psi) R^T, R = B on every 3-vector of its unknowns.

Pins (tests/test_oracle_precond.py): the fit reproduces trigonometric
polynomials exactly; the diagonal block of a body of a many-body scene equals
the rotated block of the same body alone in its own frame (an invariant of
the method, checked on the oracle's own assembly); on a block-diagonal matrix
the preconditioner is the exact inverse.
"""
from __future__ import annotations

import numpy as np

from .core import assemble_As, assemble_system, geometry, nearest, patch_weights


def body_rows(N, body, b):
    """Global unknowns of body b's block, in block order (Sec. 4 unknown
    ordering: component-major forces, then (U, Omega) of body b at 3N + 6b)."""
    pts = np.flatnonzero(np.asarray(body) == b)
    return np.concatenate([pts, N + pts, 2 * N + pts, 3 * N + 6 * b + np.arange(6)])


def diagonal_blocks(A, N, M, body):
    """The square blocks A[rows_b, rows_b] of the M free bodies."""
    out = []
    for b in range(M):
        r = body_rows(N, body, b)
        out.append(A[np.ix_(r, r)].copy())
    return out


def block_inverses(blocks):
    """Inverse of every block (the definition: LAPACK's general inverse)."""
    return [np.linalg.inv(B) for B in blocks]


def apply_block_preconditioner(inverses, N, body, v):
    """z = M^-1 v: body b's unknowns get inverses[b] @ v[rows_b], every other
    unknown is copied."""
    z = np.array(v, dtype=np.float64, copy=True)
    for b, K in enumerate(inverses):
        r = body_rows(N, body, b)
        z[r] = K @ np.asarray(v)[r]
    return z


def trig_basis(psi, H):
    """[1, cos psi, sin psi, cos 2 psi, sin 2 psi, ..., cos H psi, sin H psi]."""
    psi = np.atleast_1d(np.asarray(psi, dtype=np.float64))
    cols = [np.ones_like(psi)]
    for h in range(1, H + 1):
        cols += [np.cos(h * psi), np.sin(h * psi)]
    return np.stack(cols, axis=1)


def trig_fit(samples, psis, H):
    """Least-squares trigonometric polynomial of degree H through samples
    [S, ...] at phases psis [S]; returns coefficients [2H+1, ...] in the
    order of trig_basis."""
    samples = np.asarray(samples, dtype=np.float64)
    S = samples.shape[0]
    F = trig_basis(psis, H)
    coef, *_ = np.linalg.lstsq(F, samples.reshape(S, -1), rcond=None)
    return coef.reshape((2 * H + 1,) + samples.shape[1:])


def trig_eval(coef, psi, H):
    """The fitted polynomial at one phase psi."""
    f = trig_basis(psi, H)[0]
    return np.tensordot(f, coef, axes=1)


def frame_rotation(B, nbp):
    """R (order 3 nbp + 6) applying B to each point's force vector (entries
    (p, nbp + p, 2 nbp + p)) and to U and Omega."""
    nb = 3 * nbp + 6
    R = np.zeros((nb, nb))
    for p in range(nbp):
        for i in range(3):
            for j in range(3):
                R[i * nbp + p, j * nbp + p] = B[i, j]
    for g in range(2):
        o = 3 * nbp + 3 * g
        R[o:o + 3, o:o + 3] = B
    return R


def body_phase(scene, b, t):
    """psi = omega t - phi of the first wave point of body b (0 if none)."""
    body, part = np.asarray(scene["body"]), np.asarray(scene["part"])
    for m in np.flatnonzero(body == b):
        if part[m] >= 0:
            w = np.asarray(scene["wave"])[part[m]]
            return w[4] * t - w[5]
    return 0.0


def system_matrix(scene, t, Y):
    """The full FP64 matrix of a scene state (geometry, nearest map, Sec. 3
    eq. 23 operator, rigid-body rows)."""
    x, X, w, _ = geometry(scene, t, Y)
    nu = nearest(x, X, scene["group_off"], scene["groupX"])
    As = assemble_As(x, X, w, nu, scene["eps"], scene["mu"])
    W = patch_weights(w, nu, scene["N"])
    return assemble_system(As, x, W, scene["body"], Y, scene["M"])


def one_body_blocks(scene, psis):
    """The block of a one-body scene in its own frame (origin, B = I) at the
    beat phases psis: the scene's full matrix at t = (psi + phi) / omega."""
    if scene["M"] != 1:
        raise ValueError("one free body expected")
    Y = np.zeros((1, 12))
    Y[0, 3:] = np.eye(3).ravel()
    part = np.asarray(scene["part"])
    w = np.asarray(scene["wave"])[part[part >= 0][0]]
    return [system_matrix(scene, (psi + w[5]) / w[4], Y) for psi in np.atleast_1d(psis)]
