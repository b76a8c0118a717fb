"""FP64 CPU oracle for greedy adaptive TT cross -- test infrastructure only.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the GPU library.
"""
from .oracle import (Oracle, fn_eval, matrix_residual, mix64, pairwise_sumsq, sample_indices,  # noqa: F401
                     splitmix64, tt_eval)
