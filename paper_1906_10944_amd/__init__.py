"""GenEO two-level overlapping Schwarz preconditioner inside PCG, for AMD
Instinct MI355X (gfx950).

The product is ``libgeneo.so`` (HIP kernels behind the C ABI of
``include/geneo.h``); :mod:`paper_1906_10944_amd.geneo` is its thin ctypes
binding.  Nothing here falls back to CPU arithmetic: without the built
library (or without a GPU) the calls fail.
"""
from . import geneo  # noqa: F401

__all__ = ["geneo"]
