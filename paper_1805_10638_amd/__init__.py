"""Anderson-accelerated Lloyd K-Means on AMD Instinct MI355X (gfx950).

The compute path is a HIP shared library (``libkmaa.so``) with a plain C ABI
declared in ``include/km.h``; this package binds it with ctypes.  Importing
the package does not load the library; the first call does, and fails loudly
if the library has not been built.
"""

import importlib

__all__ = ["kmeans_g", "kmeans_g_noalloc", "kmeans_solve", "kmeans_solve_batch", "Engine", "Context", "KMError", "synth"]

_LIB_NAMES = ("kmeans_g", "kmeans_g_noalloc", "kmeans_solve", "kmeans_solve_batch", "Engine", "Context", "KMError",
              "SolveStats", "GStats", "JobResult", "load_library")


def __getattr__(name):
    if name in _LIB_NAMES:
        return getattr(importlib.import_module("._lib", __name__), name)
    if name in ("synth", "build", "_lib"):
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
