"""CPU FP64 oracle of the reduced-space hot path.

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's CPU
baseline import this package.  It shares no code with the GPU library and
imports nothing from it; its only input module is ``gridgen``.

It computes the plain definitions of the method (power-flow solution,
augmented-Lagrangian value, reduced gradient, reduced Jacobian of the
constraints, reduced Hessian, Cholesky step, the bounded QP of the real-time
step, the static OPF by the augmented-Lagrangian method) with SciPy/NumPy: bus-wise complex admittance formulas, SuperLU, the
dense Schur-complement form of the reduced Hessian, a textbook Cholesky.
Pins for each function are in the ``-m "not gpu"`` tests.
"""
from .model import Model, term_hessian, PQ, PV, REF
from .reduced import (PFResult, Point, PowerFlowError, al_objective, cholesky_lower,
                      delta_ladder, factor_solve, full_gradient, hvp_adjoint_adjoint,
                      lagrangian_hessian_full, reduced_gradient, reduced_hessian, reduced_jacobian,
                      slack_minimiser, solve_pf, tracking_step)
from .rtqp import box_qp_ipm, kkt_error, qp_data, rt_step_qp, tracking_step_qp
from .static_opf import projected_gradient, static_opf
