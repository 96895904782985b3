"""CPU FP64 oracle for the Laplace-transform shifted-system path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything here: only the test suite, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the HIP library: it
assembles its own finite-volume operator, computes its own Talbot contour
and solves every shifted system with a sparse direct factorisation, which
is the plain definition of what the flexible Krylov method approximates.

Modules
-------
fv        cell-centred finite-volume K, lumped M, point-source weights
contour   optimised Talbot nodes and trapezoid weights (Section 2.2)
heads     heads at receivers by one direct solve per shift (eqn:half)
jacobian  sensitivities to ln(kappa), ln(S) by the discrete adjoint (Section 5.2)
krylov    Algorithm 1 (flexible shifted FOM/GMRES) with exact shift-and-invert
          preconditioners, and the preconditioner schedule of Section 3
geostat   the quasi-linear geostatistical inversion (Section 5.1, Algorithm 2)
timestep  Crank-Nicolson heads (the inversion's data with model error, Section 5.3)
p1        piecewise-linear finite elements on a triangulated rectangle, lumped mass (Section 2.1)
"""
from .fv import assemble, point_weights
from .contour import talbot_nodes, talbot_full
from .heads import heads, shifted_fields
from .jacobian import jacobian
from .krylov import flexible_shifted, shift_invert, tau_schedule
from .geostat import exp_covariance, gauss_newton_step, saddle_update
from .timestep import crank_nicolson_heads
from .p1 import assemble_p1, point_weights_p1, heads_p1

__all__ = ["assemble", "point_weights", "talbot_nodes", "talbot_full", "heads",
           "shifted_fields", "jacobian", "flexible_shifted", "shift_invert", "tau_schedule",
           "exp_covariance", "gauss_newton_step", "saddle_update", "crank_nicolson_heads",
           "assemble_p1", "point_weights_p1", "heads_p1"]
