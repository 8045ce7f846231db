"""MI355X-native dense Krylov solvers (CG, GMRES(m), BiCGSTAB, FP32/BF16-inner
iterative refinement, GMRES-IR with a binary32 block LU) and the stationary
Jacobi / Gauss-Seidel iterations, behind the C ABI of include/ks.h; this
package is its Python binding.  The kernels live in csrc/ and are built into
libks.so by build.py.
"""
from ._native import EXPORTS, KsError, LIB_PATH, STATUS_NAMES, lib  # noqa: F401

__all__ = ["solve", "Solver", "gemv", "symv", "lu32_factor", "convert", "read_ceiling", "lib", "KsError"]


def __getattr__(name):
    # the torch-based front end is imported lazily so that loading the C ABI
    # (e.g. to list its exports) does not need torch
    if name in ("solve", "Solver", "gemv", "symv", "lu32_factor", "convert", "read_ceiling",
                "make_params"):
        from . import krylov

        return getattr(krylov, name)
    raise AttributeError(name)
