"""FastPI on one MI355X: low-rank SVD of a reordered sparse feature matrix and the
pseudoinverse apply (Jung & Sael, arXiv 2011.04235), as a HIP library with a thin binding."""
from ._lib import (Batch, CoreSolver, FastPIError, Handle, Inner, Labels, Plan, Tuning, inner_applies, load,  # noqa: F401
                   rank_allocate, rank_inputs, reorder,
                   target_rank, SIGNATURES, LIB_PATH)
