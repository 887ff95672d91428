"""Pins of the adaptive Dormand-Prince oracle (oracle/dopri.py): SciPy's
RK45 (the same 5(4) pair, error norm and step-size rule) on the swimmer ODE
and on a linear system, fifth-order convergence of the pair with fixed steps,
and the embedded estimate's fourth order."""
import math

import numpy as np
from scipy.integrate import solve_ivp

import synth
from oracle import dopri


def test_tableau_order_conditions():
    """Row sums give the nodes; both weight sets are consistent (sum 1) and
    reproduce the quadrature conditions up to their orders."""
    for s in range(1, 7):
        assert abs(sum(dopri.A[s]) - dopri.C[s]) < 1e-15
    for b, order in ((dopri.B5, 5), (dopri.B4, 4)):
        for q in range(1, order + 1):
            assert abs(np.dot(b, dopri.C ** (q - 1)) - 1.0 / q) < 1e-14, (order, q)


def test_matches_scipy_rk45_on_swimmers():
    """Two undulating filaments, rtol 1e-6, atol 1e-9: the same accepted
    times and the same final state as scipy.integrate.solve_ivp(RK45) from
    the same first step."""
    sc = synth.filament_scene(M=2, seed=3, Nf=20, Qf=200)
    F = dopri.swimmer_rhs(sc)
    y0 = sc["Y0"].ravel()
    y, log = dopri.dopri_integrate(F, y0, 0.0, 1.0, 0.05, 1e-6, 1e-9)
    ref = solve_ivp(lambda t, v: F(v, t), (0.0, 1.0), y0, method="RK45", rtol=1e-6, atol=1e-9,
                    first_step=0.05)
    acc = [t for t, h, ok, _ in log if ok] + [1.0]
    np.testing.assert_allclose(acc, ref.t, rtol=0, atol=1e-12)
    assert np.abs(ref.y[:, -1] - y).max() < 1e-13
    assert ref.nfev == 1 + 6 * len(log)   # first same as last


def test_matches_scipy_rk45_with_rejections():
    """A stiff-ish linear system started with far too large a step: the same
    accepted and rejected steps as SciPy (its step log is reconstructed from
    the accepted times) and the same result."""
    Am = np.array([[-2.0, 1.0, 0.0], [0.5, -30.0, 2.0], [0.0, 1.0, -0.3]])
    F = lambda y, t: Am @ y + np.array([math.sin(t), 0.0, 1.0])  # noqa: E731
    y0 = np.array([1.0, -1.0, 0.5])
    y, log = dopri.dopri_integrate(F, y0, 0.0, 3.0, 1.0, 1e-8, 1e-10)
    assert sum(1 for entry in log if not entry[2]) >= 1
    ref = solve_ivp(lambda t, v: F(v, t), (0.0, 3.0), y0, method="RK45", rtol=1e-8, atol=1e-10,
                    first_step=1.0)
    acc = [t for t, h, ok, _ in log if ok] + [3.0]
    # same steps; the step sizes differ by rounding of the factor, which adds
    # up to ~1e-10 in t over 142 steps
    np.testing.assert_allclose(acc, ref.t, rtol=0, atol=1e-8)
    assert np.abs(ref.y[:, -1] - y).max() < 1e-12


def test_fifth_order_fixed_steps():
    """y' = A y (exact solution by the matrix exponential): one attempt of
    step h has error O(h^6) in the fifth-order solution and O(h^5) in the
    embedded difference."""
    from scipy.linalg import expm
    Am = np.array([[0.0, 1.0], [-4.0, -0.1]])
    F = lambda y, t: Am @ y  # noqa: E731
    y0 = np.array([1.0, 0.0])
    errs, ests = [], []
    for h in (0.2, 0.1, 0.05):
        y1, e, _ = dopri.dopri_attempt(F, y0, 0.0, h, F(y0, 0.0))
        errs.append(np.abs(y1 - expm(Am * h) @ y0).max())
        ests.append(np.abs(e).max())
    for a, b in zip(errs, errs[1:]):
        assert 50 < a / b < 80          # 2^6 = 64
    for a, b in zip(ests, ests[1:]):
        assert 25 < a / b < 40          # 2^5 = 32
