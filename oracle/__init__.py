"""CPU complex128 oracle for the augmented-wavefield solve, source estimate,
objective and gradient.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the GPU library.  Parity status of every function is listed in its
docstring; all are pinned by the CPU tests in tests/test_oracle_pins.py.
"""
from .wri_oracle import *  # noqa: F401,F403
from .wri_oracle import (KNOWN, ESTIMATE, sponge, laplacian, helmholtz, restriction,  # noqa: F401
                         unit_vector, system_operators, normal_matrix, factor, solve_known,
                         solve_estimate, objective_terms, gradient_term, objective_grad,
                         plain_helmholtz_solution, observed_data, apply_S, apply_SH,
                         rhs_vector, normal_residual, cgls, paper_S_and_b, paper_f2, fwi_alpha,
                         fwi_objective_grad, receiver_source_solution, resample_matrix,
                         objective_grad_model, trilinear_point, offgrid_operators,
                         solve_estimate_general, objective_grad_offgrid)
