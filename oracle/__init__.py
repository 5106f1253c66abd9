"""FP64 CPU oracle for the accelerated sharing-ADMM radar imager.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link this package; it is used by the
tests, by the smoke check, by the CPU-baseline leg of the benchmark, and by the
scripts that write stored reference values.  It shares no code with the GPU
engine: plain NumPy/SciPy in complex128, written from the paper's equations.

Modules
  sadmm       plain SADMM and pruned ASADMM (eq. (3), Alg. 1), KKT certificate
  lambda_max  smallest l1 weight with an all-zero optimum image
  cnn         FP64 reference of the pixel-pruning CNN (forward, backward, BCE)
  render      back-projection image and dynamic-range rendering (Sec. IV, Fig. 1)
"""

from .sadmm import (Params, Result, solve, soft_threshold, kkt_gradient, residual_norms,
                    matched_filter, nonneg_threshold, stack_real)
from .lambda_max import lambda_max
from .render import back_projection, render_db, db_thresholds

__all__ = ["Params", "Result", "solve", "soft_threshold", "nonneg_threshold", "stack_real", "kkt_gradient",
           "residual_norms", "lambda_max", "matched_filter", "back_projection", "render_db",
           "db_thresholds"]
