"""MI355X (gfx950) HIP implementation of the hot path of the positivity-preserving
fractional algorithm for the four-equation HRM (arXiv:2208.04488).

Submodules are imported explicitly: ``inputs`` (seeded initial conditions, no
GPU needed) and ``hrm`` (the ctypes binding of the C-ABI library ``libhrm.so``).
"""
__all__ = ["inputs", "hrm"]
