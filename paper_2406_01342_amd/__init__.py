"""PolyCLEAN measurement-operator hot path for MI355X (gfx950).

The compute lives in libpolyclean.so (HIP kernels behind a C ABI declared in
include/polyclean.h).  ``paper_2406_01342_amd.api`` is the Python binding:
argument marshalling only, with the same function names as the C ABI.
Importing the binding loads the library and fails loudly if it is missing.
"""
__all__ = ["api"]
