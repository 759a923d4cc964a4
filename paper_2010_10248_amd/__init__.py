"""MI355X-native temporal blocking of FD wave propagators with sparse
off-the-grid sources (Bisbas et al., arXiv 2010.10248).

The compute path is a C-ABI shared library of hand-written HIP kernels for
gfx950 (``include/tb.h``); ``paper_2010_10248_amd.tb`` is its thin ctypes
binding. Importing this package loads nothing: the library is opened on first
use and a missing library is an error, never a fallback.
"""
__all__ = ["workloads"]
