"""The library's bfloat16 sketch, oracle side.

Test infrastructure only (see the package header).

The paper's method computes in one working precision.  The library also
offers a sketch run on the bfloat16 matrix cores: every float32 operand (the
matrix and Omega of Alg. 1's first product) is split by truncation into two
bfloat16 pieces, x = h + m + remainder (h: x with all but the top 8 significant
bits cleared; m: the same of x - h, which float32 holds exactly), and the
product keeps the three piece products of weight above 2^-16, h h' + h m' + m h'
(the bf16x3 scheme of Henry, Tang and Heinecke, ARITH 2019).  The oracle forms
those three products in float64, where products of bfloat16 values are exact.

split_bf16 is pinned by tests/test_oracle_precision.py: both pieces are
bfloat16 values (torch's bfloat16 conversion leaves them unchanged), each is
the bfloat16 value next to its argument towards zero, the three-piece sum
h + m + (x - h - m) equals x with the remainder again a bfloat16 value, and
the remainder is below 2^-15 |x|; sketch_bf16x3 against its expansion on
hand-built operands and against the exact product within the bound.
"""
import numpy as np


def _trunc_bf16(f32):
    """float32 array -> float32 array with the low 16 bits of every value cleared."""
    u = np.ascontiguousarray(f32, dtype=np.float32).view(np.uint32) & np.uint32(0xFFFF0000)
    return u.view(np.float32)


def split_bf16(a):
    """(h, m) of each entry (rounded to float32 first, the precision the library
    holds data and Omega in), as float64 arrays."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    h = _trunc_bf16(f)
    m = _trunc_bf16(f - h)            # f - h is exact in float32
    return h.astype(np.float64), m.astype(np.float64)


def sketch_bf16x3(A, B):
    """A @ B as the library's bfloat16 sketch forms it: h_A h_B + h_A m_B + m_A h_B."""
    hA, mA = split_bf16(A)
    hB, mB = split_bf16(B)
    return hA @ hB + hA @ mB + mA @ hB
