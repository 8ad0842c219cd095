"""Exact sparse spherical k-means on AMD MI355X (gfx950).

The hot path lives in HIP kernels behind the C ABI of ``include/skm.h``
(``libskm.so``); ``skm`` is its ctypes binding.
"""
from . import skm  # noqa: F401
from .skm import Context, SkmError, kmeanspp, load  # noqa: F401
