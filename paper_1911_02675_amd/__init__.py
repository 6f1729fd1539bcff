"""Sketch-preconditioned least squares on AMD Instinct MI355X (gfx950).

Method: Lacotte & Pilanci, "Faster Least Squares Optimization" (arXiv 1911.02675).  The compute
path is the HIP library liblsq.so (C ABI in include/lsq.h); `lsq` is its thin Python binding.
"""
from . import lsq  # noqa: F401

__all__ = ["lsq"]
