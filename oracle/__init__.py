"""FP64 CPU oracle for randomized Tucker compression (R-HOSVD, R-STHOSVD,
adaptive R-STHOSVD) after Minster, Saibaba and Kilmer, "Randomized Algorithms
for Low-rank Tensor Decompositions in the Tucker Format".

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference that the HIP path is checked against.  Only the test-suite, the
smoke check in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py``
may import it.  The product library never imports, links or calls anything in
here, and nothing in here imports the product package: the two share no code.

Everything is NumPy in float64 with the host LAPACK.  Each function cites the
passage of the paper it follows.  Parity status of every function is listed
in its module header; none is "parity unpinned" except where stated.
"""

from .philox import philox4x32_10, omega_block, omega, PHILOX_M0, PHILOX_M1, PHILOX_W0, PHILOX_W1
from .tensor import unfold, fold, ttm, reconstruct, fro2
from .randsvd import randsvd, range_basis, qb_truncate, orth_householder, sign_fix_columns
from .tucker import (rhosvd, rsthosvd, hosvd, sthosvd, default_order, TuckerResult,
                     per_mode_residuals)
from .adaptive import adapt_range_finder, adaptive_rsthosvd, adaptive_rhosvd
from .precision import split_bf16, sketch_bf16x3
from .structure import pivoted_rows, select_rows, sp_sthosvd
from .sparse import unfold_coo, fold_coo, densify, sketch_coo, sp_sthosvd_coo

__all__ = [
    "philox4x32_10", "omega_block", "omega", "PHILOX_M0", "PHILOX_M1", "PHILOX_W0", "PHILOX_W1",
    "unfold", "fold", "ttm", "reconstruct", "fro2",
    "randsvd", "range_basis", "qb_truncate", "orth_householder", "sign_fix_columns",
    "rhosvd", "rsthosvd", "hosvd", "sthosvd", "default_order", "TuckerResult",
    "per_mode_residuals",
    "adapt_range_finder", "adaptive_rsthosvd", "adaptive_rhosvd",
    "pivoted_rows", "select_rows", "sp_sthosvd",
    "unfold_coo", "fold_coo", "densify", "sketch_coo", "sp_sthosvd_coo",
    "split_bf16", "sketch_bf16x3",
]
