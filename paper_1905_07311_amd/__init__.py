"""rtucker: randomized Tucker compression (R-HOSVD, R-STHOSVD, adaptive
R-STHOSVD) for AMD Instinct MI355X (gfx950).

All compute runs in hand-written HIP kernels inside the shared library
``librtucker.so`` (C ABI, declared in include/rtucker.h).  The Python layer in
``paper_1905_07311_amd.rtucker`` only marshals torch device buffers and
streams into that ABI; it raises if the library is missing.
"""

__all__ = ["rtucker", "inputs"]
