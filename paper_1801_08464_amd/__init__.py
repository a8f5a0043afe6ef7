"""MGR-preconditioned GMRES for block-structured NCP Jacobians on MI355X (gfx950).

The solver lives in libmgr.so (HIP kernels behind the C ABI of include/mgr.h);
this package holds its build script and a thin torch/ctypes binding."""

__all__ = ["MGRSolver", "MGRSolve", "DifferentiableMGR", "NCPNewton", "MGRError", "load_library", "build"]


def __getattr__(name):
    if name in ("MGRSolver", "MGRSolve", "DifferentiableMGR"):
        from . import solver
        return getattr(solver, name)
    if name == "NCPNewton":
        from .newton import NCPNewton
        return NCPNewton
    if name in ("MGRError", "load_library"):
        from . import binding
        return getattr(binding, name)
    if name == "build":
        from .build import build
        return build
    raise AttributeError(name)
