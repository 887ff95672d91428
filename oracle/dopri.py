"""Plain FP64 reference of adaptive Dormand-Prince 5(4) time stepping of the
swimmer state.  Test infrastructure only (see the package docstring).

The paper integrates Y' = F(Y, t) (Sec. 4) with MATLAB's ode45, an explicit
Runge-Kutta 5(4) pair with error control (Dormand and Prince, 1980).  Here:
  * the pair of Dormand and Prince (seven stages, the last one evaluated at
    the new state, so it is the first stage of the next step: "first same as
    last");
  * local error estimate e = h sum_i (b5_i - b4_i) k_i, measured as
    ||e / (atol + rtol max(|y|, |y_new|))||_rms;
  * a step is accepted when that norm is <= 1; the next step size is
    h * min(10, 0.9 norm^(-1/5)) after an acceptance (at most h right after a
    rejection), h * max(0.2, 0.9 norm^(-1/5)) after a rejection; the last
    step is cut to end at t1.
Readings: MATLAB's own controller differs in details (its norm is the max
norm, its factors differ), the paper does not state its tolerances; the
controller above is the common textbook one (Hairer, Norsett and Wanner) and
is the one SciPy's RK45 uses, which pins this code.  Swimmer frames are not
re-orthonormalised between steps (that would break "first same as last");
the error control bounds their drift, as in ode45.
"""
from __future__ import annotations

import numpy as np

from .core import solve_scene, rates

# Dormand-Prince 5(4): nodes, stage coefficients, 5th-order weights (= the
# last stage row) and 4th-order weights
C = np.array([0.0, 1 / 5, 3 / 10, 4 / 5, 8 / 9, 1.0, 1.0])
A = [
    [],
    [1 / 5],
    [3 / 40, 9 / 40],
    [44 / 45, -56 / 15, 32 / 9],
    [19372 / 6561, -25360 / 2187, 64448 / 6561, -212 / 729],
    [9017 / 3168, -355 / 33, 46732 / 5247, 49 / 176, -5103 / 18656],
    [35 / 384, 0.0, 500 / 1113, 125 / 192, -2187 / 6784, 11 / 84],
]
B5 = np.array([35 / 384, 0.0, 500 / 1113, 125 / 192, -2187 / 6784, 11 / 84, 0.0])
B4 = np.array([5179 / 57600, 0.0, 7571 / 16695, 393 / 640, -92097 / 339200, 187 / 2100, 1 / 40])
E = B5 - B4

SAFETY, MIN_FACTOR, MAX_FACTOR = 0.9, 0.2, 10.0


def dopri_attempt(F, y, t, h, k1):
    """One Dormand-Prince attempt from (t, y) with step h and first stage k1
    = F(y, t): returns (y_new, err_vector, k7) with k7 = F(y_new, t + h)."""
    k = [k1]
    for s in range(1, 7):
        ys = y + h * sum(A[s][j] * k[j] for j in range(s))
        k.append(F(ys, t + C[s] * h))
    y_new = y + h * sum(B5[j] * k[j] for j in range(7))
    err = h * sum(E[j] * k[j] for j in range(7))
    return y_new, err, k[6]


def error_norm(err, y, y_new, rtol, atol):
    scale = atol + rtol * np.maximum(np.abs(y), np.abs(y_new))
    return float(np.sqrt(np.mean((err / scale) ** 2)))


def dopri_integrate(F, y0, t0, t1, h0, rtol, atol, max_steps=100000):
    """Integrate y' = F(y, t) from t0 to t1 > t0 starting with step h0.
    Returns the final state and a list of (t, h, accepted, norm) for every
    attempt."""
    y = np.asarray(y0, dtype=np.float64).copy()
    t, h = float(t0), float(h0)
    k1 = F(y, t)
    log = []
    rejected = False
    while t < t1 and len(log) < max_steps:
        h = min(h, t1 - t)
        y_new, err, k7 = dopri_attempt(F, y, t, h, k1)
        nrm = error_norm(err, y, y_new, rtol, atol)
        if nrm <= 1.0:
            log.append((t, h, True, nrm))
            fac = MAX_FACTOR if nrm == 0.0 else min(MAX_FACTOR, SAFETY * nrm ** -0.2)
            if rejected:
                fac = min(1.0, fac)
            t = t + h
            y, k1 = y_new, k7
            h = h * fac
            rejected = False
        else:
            log.append((t, h, False, nrm))
            h = h * max(MIN_FACTOR, SAFETY * nrm ** -0.2)
            rejected = True
    return y, log


def swimmer_rhs(scene):
    """Y' = F(Y, t) of the swimming problem on the flattened state [M*12]."""
    M = scene["M"]

    def F(yv, t):
        Y = np.asarray(yv).reshape(M, 12)
        _, UW = solve_scene(scene, t, Y)
        return rates(Y, UW).ravel()
    return F


def dopri_swimmers(scene, Y0, t0, t1, h0, rtol, atol):
    """Adaptive Dormand-Prince integration of the swimmers from t0 to t1."""
    M = scene["M"]
    y, log = dopri_integrate(swimmer_rhs(scene), np.asarray(Y0).ravel(), t0, t1, h0, rtol, atol)
    return y.reshape(M, 12), log
