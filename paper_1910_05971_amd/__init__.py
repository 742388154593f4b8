"""FastSV connected components on MI355X (gfx950).

Solver entry points (``cc_csr``, ``cc_edges``, ``cc_batch_csr``, ...) are thin
ctypes wrappers over the C ABI in ``include/fastsv.h``; every step of the
method runs in the HIP kernels of ``libfastsv.so``.  Importing the package
does not load the library; the first solver call does, and fails loudly if it
is missing.
"""
from .binding import *  # noqa: F401,F403
