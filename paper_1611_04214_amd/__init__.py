"""MI355X-native MOL^T Cahn-Hilliard hot path (arXiv:1611.04214).

The solver lives in the HIP library ``libmolt.so`` (C-ABI declared in
``include/molt.h``); ``molt`` is its thin ctypes binding.  Importing the package
loads nothing: the library is opened on first use and a missing library is an
error, never a silent fallback.
"""
__all__ = ["molt", "synth"]
