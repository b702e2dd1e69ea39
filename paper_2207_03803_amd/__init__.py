"""MI355X-native sparse-GP (GAP) fit: K_NM build, Cholesky, Householder QR, solve.

The compute lives in ``libgap.so`` (hand-written HIP kernels behind a C ABI,
declared in ``include/gap.h``); ``gap`` is its thin ctypes binding.  Importing
this package does not load the library: ``gap.lib()`` does, and raises if it
has not been built.
"""
__all__ = ["gap", "synth"]
