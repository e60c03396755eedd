"""hns: MI355X-native PCG solves of the shallow-basin projection step.

The solver library (libhns.so, C ABI in include/hns.h) assembles the P1
operators and runs Jacobi-preconditioned conjugate gradients in hand-written
HIP kernels for gfx950.  This package is its thin Python binding plus the
drivers built on it (projection-step right-hand sides, serving loop).
"""
from ._lib import LibraryMissing, LIB_PATH  # noqa: F401


def __getattr__(name):
    # import the torch-based binding lazily so that `import paper_1207_0486_amd`
    # (e.g. for build()) does not require a GPU
    if name in ("Operator", "SolveInfo", "HNSError"):
        from . import hns
        return getattr(hns, name)
    raise AttributeError(name)
