"""Seeded synthetic aquifer workloads.

This package only draws random inputs (log-conductivity fields, storage
fields, well coordinates, time lists) and states the configurations the
solver and the oracle are run on.  It holds none of the solver's or the
oracle's arithmetic: no discretisation, no contour, no linear algebra on
the operator.  Both the CPU oracle and the GPU path read their inputs
from here.
"""
from .grf import gaussian_random_field
from .configs import C5_BATCH, CONFIGS, T_D, make_batch, make_problem, Problem

__all__ = ["gaussian_random_field", "CONFIGS", "C5_BATCH", "T_D", "make_batch", "make_problem", "Problem"]
