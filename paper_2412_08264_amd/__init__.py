"""MI355X-native recycled-Krylov hypergradient solves (arXiv 2412.08264).

The compute lives in libbilevel_hip.so (C ABI: include/bilevel.h); ``bilevel`` is its
ctypes binding.  Import ``paper_2412_08264_amd.bilevel`` to load the library.
"""
__all__ = ["bilevel"]
