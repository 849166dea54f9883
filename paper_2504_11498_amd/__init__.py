"""MI355X-native batched point projection and inversion on B-spline curves via
cubic Bezier matrix representations (Wu & Zou, arXiv 2504.11498).

The compute path is the HIP library ``libmrep.so`` built from ``csrc/``; the
Python module ``mrep`` is a thin ctypes binding to its C ABI (``include/mrep.h``).
Importing this package does not load the library; ``paper_2504_11498_amd.mrep``
does, and raises if it has not been built.
"""
__all__ = ["gen", "mrep"]
