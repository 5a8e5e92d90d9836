"""Anderson-accelerated Lloyd K-Means on AMD Instinct MI355X (gfx950).

The compute path is a HIP shared library (``libkmaa.so``) with a plain C ABI
declared in ``include/km.h``; this package binds it with ctypes.  Importing
the package does not load the library; the first call does, and fails loudly
if the library has not been built.
"""

__all__ = ["kmeans_g", "kmeans_solve", "Context", "KMError", "synth"]


def __getattr__(name):
    if name in ("kmeans_g", "kmeans_solve", "Context", "KMError", "SolveStats",
                "GStats", "kmeans_solve_batched", "load_library"):
        from . import _lib
        return getattr(_lib, name)
    if name == "synth":
        from . import synth
        return synth
    raise AttributeError(name)
