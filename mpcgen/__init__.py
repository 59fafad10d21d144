"""Seeded synthetic workload generator for batched centroidal MPC problems.

This package only draws inputs: it builds the time-varying dynamics, weights,
references and contact schedules of the problems to be solved.  It holds none
of the solver's arithmetic and is shared by the FP64 oracle, the tests and the
benchmark, so that both sides of every parity check receive identical data.
"""
from .centroidal import (  # noqa: F401
    CONFIGS,
    NX,
    NU,
    NC,
    GRAVITY,
    make_batch,
    problem_slice,
    problem_fp64,
)
