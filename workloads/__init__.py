"""Seeded synthetic inputs for the dense Krylov solvers (shared by tests and bench).

This package only draws random numbers and assembles the test systems
A, b = A x_true. It contains none of the solvers' arithmetic.
"""
from .gen import (  # noqa: F401
    Problem,
    spd_problem,
    nonsym_problem,
    nonsym_swept_problem,
    multi_rhs_problem,
    stream_requests,
    seed_words,
)
