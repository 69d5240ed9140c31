"""Reduced-precision rounding used by the oracle's bfloat16-sketch variant.

Test infrastructure only (see the package header).

The paper's method computes in one working precision.  The library also
offers a sketch whose products are formed from bfloat16-rounded operands
(float32 accumulation), the rest of the method unchanged; the oracle models
that variant by rounding the two operands of Alg. 1 step 1 (the matrix and
Omega) to bfloat16 and forming the product in float64, which is exact for
products of bfloat16 values.

round_bf16 is pinned by tests/test_oracle_precision.py against hand-checked
values (ties to even) and against torch's float32 -> bfloat16 conversion.
"""
import numpy as np


def round_bf16(a):
    """Nearest bfloat16 value of each entry (ties to even), as float64.  The
    entries are first rounded to float32 (the precision the library's data and
    Omega are held in)."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
