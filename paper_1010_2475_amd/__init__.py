"""MI355X-native hot path of the multi-moment vortex method (arXiv:1010.2475).

The compute path lives in the HIP/C++ library ``libmmvm.so`` (``csrc/``),
declared in ``include/mmvm.h``; :mod:`paper_1010_2475_amd.mmvm` is a thin
ctypes binding with the same names.  Importing this package loads nothing;
the library is loaded on first use of the binding.
"""
__all__ = ["workloads", "mmvm"]
