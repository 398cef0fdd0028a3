"""MI355X-native implicit 7-point finite-volume solver (BiCGStab hot path).

The compute path lives in ``libwfa.so`` (HIP kernels for gfx950 behind a
C-ABI); ``paper_2209_13768_amd.wfa`` is its thin Python binding.  Importing
this package loads nothing; the binding loads the library on first use and
raises if it is missing.
"""
