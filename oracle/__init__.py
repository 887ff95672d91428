"""CPU FP64 oracle for the nearest-neighbour regularized stokeslet method.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package's smoke entry
and the benchmark's CPU-baseline leg may import this package.  The product
path (the HIP library and its Python binding) never calls it, and the two
share no code: the only common input is the seeded scene description from
the ``synth`` package.

Everything here is plain NumPy/SciPy in float64, written to be checked by
eye against Gallagher & Smith, "Passively parallel regularized stokeslets"
(arXiv:2001.06468).  Section and equation numbers refer to that paper.

Parity pins: every function here is pinned by the ``-m "not gpu"`` tests in
tests/test_oracle_*.py (closed forms, invariants, brute force, textbook
physics).  The one exception is the learned warm-start network reference
(``mlp``), whose gradients are pinned by central finite differences but whose
*output quality* has no pin in the paper ("parity unpinned": the GMRES
residual is the only judge of a prediction).
"""
from .core import (  # noqa: F401
    stokeslet_reg, pressure_reg, blob, stokeslet_singular,
    geometry, nearest, assemble_As, patch_weights, assemble_system, rhs,
    solve_system, solve_scene, split_solution, doolittle_solve,
    rates, rk4_step, orthonormalise, rk4_generic, gmres, condition_1,
    solve_with_condition,
)
from .field import (  # noqa: F401
    field_velocity, tracer_rk4_step, rk4_step_tracers,
)
from .dopri import (  # noqa: F401
    dopri_attempt, dopri_integrate, dopri_swimmers, error_norm,
)

from . import precond  # noqa: F401
