"""FP64 CPU reference for the OTLM scaling algorithm -- test infrastructure.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The GPU library neither imports nor links anything from here.
"""
from .otlm_oracle import *  # noqa: F401,F403
from .otlm_oracle import (omega, gibbs_kernel, prox_datafit, mm_step, prox_P_exact,  # noqa: F401
                          prox_objective, penalty_value, penalty_grad, initial_weights,
                          solve, objective)
from . import mlp_oracle as mlp  # noqa: F401,E402
