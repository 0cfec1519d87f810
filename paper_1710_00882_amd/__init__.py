"""MI355X-native Tersoff energy / force / virial evaluation.

The compute path lives in libtersoff.so (HIP kernels for gfx950 behind the C
ABI of include/tersoff.h); ``Tersoff`` is its thin ctypes binding.  Importing
this package does not load the library; the first ``Tersoff(...)`` does, and
raises if it has not been built.
"""
from ._lib import FP64, MIXED, SINGLE, Tersoff, TersoffError, clock_ns, load, parse_params  # noqa: F401

__all__ = ["Tersoff", "TersoffError", "load", "parse_params", "clock_ns", "FP64", "MIXED", "SINGLE"]
