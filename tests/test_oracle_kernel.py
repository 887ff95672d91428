"""Pins of the oracle's kernels against closed forms and the Stokes equations
(Sec. 2 eqs. 3-6, Sec. 3 eqs. 14-18)."""
import math

import numpy as np
import pytest

import oracle

EPS = 0.3


def _fd_residuals(S_fn, P_fn, eps, pts, h=1e-3, mu=1.0):
    """Central-difference residuals of  mu lap u - grad p + phi_eps e_k  and
    div u for u = S e_k / (8 pi mu), p = P_k / (8 pi)."""
    res_mom, res_div = [], []
    E = np.eye(3)
    for x in pts:
        for k in range(3):
            u = lambda y: S_fn(y, eps)[:, k] / (8 * math.pi * mu)  # noqa: E731
            p = lambda y: P_fn(y, eps)[k] / (8 * math.pi)          # noqa: E731
            lap = np.zeros(3)
            div = 0.0
            gp = np.zeros(3)
            for a in range(3):
                lap += (u(x + h * E[a]) - 2 * u(x) + u(x - h * E[a])) / h ** 2
                div += (u(x + h * E[a])[a] - u(x - h * E[a])[a]) / (2 * h)
                gp[a] = (p(x + h * E[a]) - p(x - h * E[a])) / (2 * h)
            mom = mu * lap - gp + oracle.blob(x, eps) * E[k]
            res_mom.append(np.max(np.abs(mom)))
            res_div.append(abs(div))
    return max(res_mom), max(res_div)


def _pts():
    rng = np.random.default_rng(3)
    return [v for v in rng.normal(size=(6, 3)) * 0.4]


def test_regularized_stokeslet_solves_regularized_stokes():
    """u = S^eps e_k/(8 pi mu), p = P^eps_k/(8 pi) satisfy the forced Stokes
    equations with the blob as forcing (Sec. 3, eqs. 14-18)."""
    mom, div = _fd_residuals(oracle.stokeslet_reg, oracle.pressure_reg, EPS, _pts())
    scale = oracle.blob(np.zeros(3), EPS)
    assert mom < 1e-4 * scale
    assert div < 1e-6


@pytest.mark.parametrize("mutant", ["eps2_coefficient", "exponent", "outer_sign"])
def test_stokes_pin_catches_planted_kernel_mistakes(mutant):
    """The FD pin has teeth: plausible mistakes in S^eps fail it."""
    def bad(r, eps):
        r = np.asarray(r, float)
        r2 = r @ r
        c2 = {"eps2_coefficient": 1.0}.get(mutant, 2.0)
        ex = {"exponent": 1.0}.get(mutant, 1.5)
        sg = {"outer_sign": -1.0}.get(mutant, 1.0)
        return ((r2 + c2 * eps * eps) * np.eye(3) + sg * np.outer(r, r)) / (r2 + eps * eps) ** ex
    mom, div = _fd_residuals(bad, oracle.pressure_reg, EPS, _pts())
    scale = oracle.blob(np.zeros(3), EPS)
    assert mom > 1e-3 * scale or div > 1e-3


def test_value_at_origin_and_symmetry():
    for eps in (0.01, 0.1, 1.0):
        np.testing.assert_allclose(oracle.stokeslet_reg(np.zeros(3), eps), (2.0 / eps) * np.eye(3),
                                   rtol=1e-15)
    r = np.random.default_rng(1).normal(size=(50, 3))
    S = oracle.stokeslet_reg(r, 0.05)
    np.testing.assert_array_equal(S, np.swapaxes(S, -1, -2))
    np.testing.assert_array_equal(S, oracle.stokeslet_reg(-r, 0.05))


def test_far_field_tends_to_singular_stokeslet():
    """S^eps -> S as eps/|r| -> 0, with an O((eps/|r|)^2) relative gap."""
    d = np.array([0.3, -0.5, 0.81])
    d /= np.linalg.norm(d)
    prev = None
    for R in (1.0, 10.0, 100.0):
        S0 = oracle.stokeslet_singular(R * d)
        Se = oracle.stokeslet_reg(R * d, 0.05)
        gap = np.max(np.abs(Se - S0)) / np.max(np.abs(S0))
        assert gap < 3 * (0.05 / R) ** 2
        if prev is not None:
            assert gap < prev
        prev = gap


def test_blob_integrates_to_one():
    from scipy.integrate import quad
    for eps in (0.01, 0.1, 1.0):
        val, _ = quad(lambda r: 4 * math.pi * r * r * oracle.blob(np.array([r, 0, 0]), eps),
                      0, np.inf, limit=200)
        assert abs(val - 1.0) < 1e-8
