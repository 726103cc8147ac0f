"""MI355X (gfx950) library for the LiFE sparse-Tucker products and SBB-NNLS.

The compute lives in liblife.so (HIP, C ABI in include/life.h); ``life`` is its
Python binding.  Importing the package does not load the library.
"""
__all__ = ["life", "build"]
