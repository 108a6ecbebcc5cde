"""SOFA exact k-NN search over z-normalised data series, MI355X (gfx950) native.

The compute lives in libsofa.so (HIP kernels behind the C ABI of
include/sofa.h); ``sofa`` is its ctypes binding.
"""
from . import sofa  # noqa: F401
