"""MI355X-native distance reporting by sorting along a space-filling curve.

The compute path is the HIP library ``libsfc.so`` built from ``csrc/`` for
gfx950; :mod:`paper_2508_19891_amd.sfc` is its thin ctypes binding.  Importing
this package loads nothing: the library is opened on first use, and the
binding raises if it has not been built.
"""
__all__ = ["sfc", "workload"]
