"""Seeded synthetic inputs: convection-diffusion matrices, right-hand sides and
request traces.

This package holds test and benchmark INPUTS only.  It contains none of the
spaQR arithmetic (ordering, factorization, apply, Krylov); both the CPU oracle
and the GPU engine consume what it produces.
"""

from .grids import (  # noqa: F401
    convdiff,
    smoothed_gaussian_field,
    perturb_offdiagonals,
    make_rhs,
    config_problem,
    CONFIGS,
)
from .trace import serving_trace  # noqa: F401
