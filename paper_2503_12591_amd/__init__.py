"""MI355X-native link-cell parallel swap Monte Carlo (EPI model).

The compute path lives in ``libsmcx.so`` (HIP kernels for gfx950 behind a
C ABI declared in ``include/smcx.h``); :mod:`paper_2503_12591_amd.smcx` is the
thin ctypes binding.  Importing the package does not load the library.
"""
__all__ = ["smcx", "inputs"]
