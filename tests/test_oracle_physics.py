"""Textbook physics and the paper's own accuracy claim as pins of the oracle
(Stokes drag, rotating-sphere torque, sedimentation; Sec. 3 sphere
resistance example)."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_claims.json")


def _drag(nc, nq, eps=0.01):
    sc = synth.sphere_scene(nc, nq, eps=eps)
    f, _, d = oracle.solve_scene(sc, return_all=True)
    return (d["W"][None, :] * f).sum(axis=1)


def _torque(nc, nq, eps=0.01):
    sc = synth.sphere_scene(nc, nq, eps=eps, U=(0, 0, 0), Omega=(0, 0, 1))
    f, _, d = oracle.solve_scene(sc, return_all=True)
    return (d["W"][None, :] * np.cross(d["x"].T, f.T).T).sum(axis=1)


def test_sphere_drag_converges_to_stokes_law():
    """Sum of patch forces -> +6 pi mu a U (force on the fluid; + sign of the
    nearest-neighbour form, Sec. 3 eq. 23); error decreases with refinement."""
    errs = []
    for nc in (4, 6, 8):
        F = _drag(nc, 4 * nc)
        assert abs(F[1]) < 1e-10 and abs(F[2]) < 1e-10
        errs.append(abs(F[0] / (6 * math.pi) - 1))
    assert errs[0] < 0.10
    assert errs[0] > errs[1] > errs[2]


def test_rotating_sphere_torque():
    T = _torque(6, 24)
    assert abs(T[2] / (8 * math.pi) - 1) < 0.05
    assert np.all(np.abs(T[:2]) < 1e-10)


def test_paper_sphere_resistance_accuracy_claim():
    """Sec. 3: resistance matrix of a sphere to within about 2 % with N = 864,
    Q = 3456 at eps = 0.01 (asserted as <= 2.5 %)."""
    with open(GOLDEN) as fh:
        claim = json.load(fh)["sphere_resistance_nearest"]
    nc, nq = claim["cube_sphere_nc"], claim["cube_sphere_nq"]
    assert 6 * nc * nc == claim["N"] and 6 * nq * nq == claim["Q"]
    F = _drag(nc, nq, claim["eps"])
    T = _torque(nc, nq, claim["eps"])
    assert abs(F[0] / (6 * math.pi) - 1) <= claim["asserted_max_rel_error"]
    assert abs(T[2] / (8 * math.pi) - 1) <= claim["asserted_max_rel_error"]


def test_sedimenting_sphere_velocity():
    """Free sphere under force F: U -> F/(6 pi mu a), no rotation."""
    sc = synth.sphere_scene(6, 24, free=True, force=np.array([0.0, 0.0, -1.0]))
    _, UW = oracle.solve_scene(sc)
    assert abs(UW[0, 2] * 6 * math.pi + 1) < 0.02
    assert np.abs(UW[0, 3:]).max() < 1e-9


def test_torque_driven_sphere_rotation():
    sc = synth.sphere_scene(6, 24, free=True, torque=np.array([0.0, 1.0, 0.0]))
    _, UW = oracle.solve_scene(sc)
    assert abs(UW[0, 4] * 8 * math.pi - 1) < 0.05
    assert np.abs(UW[0, :3]).max() < 1e-9
