"""MI355X (gfx950) hot path of the adaptive algebraic multigrid CP decomposition.

The compute path is libcpamg.so (hand-written HIP kernels behind the C ABI in
include/cpamg.h); ``api`` marshals PyTorch device tensors into those calls and
``drivers`` holds the host-side stopping loops.  ``synth`` draws the seeded
synthetic inputs.  Importing this package does not load the library; the first
call does, and it raises if the library has not been built.
"""
from ._lib import (CP_FLAG_NONFINITE, CP_FLAG_NOT_SPD, CP_FLAG_PINV_FALLBACK, CP_FP64,  # noqa: F401
                   CP_MIXED, CP_SOLVE_CHOL, CP_SOLVE_GS)

__all__ = ["api", "drivers", "synth", "CP_FP64", "CP_MIXED", "CP_SOLVE_CHOL", "CP_SOLVE_GS"]


def __getattr__(name):
    if name in ("api", "drivers", "synth"):
        import importlib
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
