"""MI355X-native sparse matrix-vector product and Krylov solvers.

The compute path is the C-ABI library ``libmxs.so`` (hand-written HIP for
gfx950, built from ``csrc/``) declared in ``include/mxs.h``; ``mxs`` is its
thin ctypes binding.  ``inputs`` holds the seeded synthetic input generators.
Nothing is loaded at import time: ``from paper_2103_10116_amd import mxs``
loads the library and fails loudly if it has not been built.
"""
__all__ = ["inputs", "mxs"]
