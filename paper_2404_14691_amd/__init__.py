"""Function-setup and shared read-only memory for many invocations of GPU
functions on one AMD MI355X: a HIP/C++ library (``lib/libsage.so``, C ABI in
include/sage.h) with a thin Python binding (``paper_2404_14691_amd.sage``).

The package import is light: ``synth`` (seeded inputs) needs no GPU and no
built library; import ``paper_2404_14691_amd.sage`` for the library.
"""
__all__ = ["synth", "build"]
