"""PyTorch-facing wrapper of libmgr: device memory and streams come from torch,
every computation runs in the library's HIP kernels.

``MGRSolver``  — one hierarchy (mgr_setup) and its solves (mgr_solve).
``MGRSolve``   — torch.autograd.Function: x = A^{-1} b with a hand-written
                 backward that runs the adjoint solve A^T lambda = dL/dx on a
                 hierarchy built on A^T and scatters dL/dvals = -lambda x^T
                 onto the sparsity pattern (mgr_pattern_outer).
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import numpy as np
import torch

from . import binding as B

_OPTION_NAMES = {f[0] for f in B.MgrOptions._fields_} - {"stream"}


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


def _dev(t, dtype, device) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(np.ascontiguousarray(t))
    return t.to(device=device, dtype=dtype).contiguous()


@dataclass
class SolveInfo:
    status: int
    iterations: int
    rel_residual: float
    setup_ms: float
    solve_ms: float
    level_n: list = field(default_factory=list)
    level_nnz: list = field(default_factory=list)
    history: np.ndarray = None


class MGRSolver:
    """MGR-preconditioned GMRES on one GPU.

    A is given as CSR arrays (row_ptr int32, col_idx int32, values float64) on
    the GPU (or anything torch.as_tensor accepts; it is moved there).
    labels[u] = MGR level at which unknown u is an F-point (max label = the
    AMG coarse grid).  Options are the fields of mgr_options (include/mgr.h);
    precision="fp64" or "mixed"."""

    def __init__(self, row_ptr, col_idx, values, labels, block_size=3, precision="fp64", transpose=False,
                 device="cuda", **opts):
        if not torch.cuda.is_available():
            raise RuntimeError("MGRSolver needs a ROCm GPU (torch.cuda is unavailable)")
        self.lib = B.load_library()
        self.device = torch.device(device)
        self.row_ptr = _dev(row_ptr, torch.int32, self.device)
        self.col_idx = _dev(col_idx, torch.int32, self.device)
        self.values = _dev(values, torch.float64, self.device)
        self.labels = _dev(labels, torch.int32, self.device)
        self.n = self.row_ptr.numel() - 1
        self.nnz = self.col_idx.numel()
        o = B.default_options()
        o.precision = {"fp64": 0, "mixed": 1}[precision] if isinstance(precision, str) else int(precision)
        o.transpose = int(bool(transpose))
        for k, v in opts.items():
            if k not in _OPTION_NAMES:
                raise TypeError(f"unknown option {k!r}")
            setattr(o, k, v)
        self.stream = torch.cuda.current_stream(self.device)
        o.stream = self.stream.cuda_stream
        self.opts = o
        csr = B.MgrCsr(self.n, self.nnz, _ptr(self.row_ptr), _ptr(self.col_idx), _ptr(self.values))
        h = C.c_void_p()
        rc = self.lib.mgr_setup(C.byref(csr), int(block_size), _ptr(self.labels), C.byref(o), C.byref(h))
        if rc != B.OK:
            raise B.MGRError(rc, B.last_error(None))
        self.h = h

    # ---- lifecycle ----
    def close(self):
        if getattr(self, "h", None):
            self.lib.mgr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow=(B.OK,)):
        if rc not in allow:
            raise B.MGRError(rc, B.last_error(self.h))
        return rc

    def update_values(self, values):
        """New values on the setup's pattern and labels (mgr_update_values): the
        hierarchy's values are redone and its AMG parts rebuilt; the patterns,
        level maps and workspace are kept.  The next solve's setup_ms is the
        update's time."""
        v = _dev(values, torch.float64, self.device)
        if v.numel() != self.nnz:
            raise ValueError(f"expected {self.nnz} values, got {v.numel()}")
        self.values = v
        self._check(self.lib.mgr_update_values(self.h, _ptr(self.values)))

    # ---- solves ----
    def solve(self, b, tol=1e-8, x0=None, history=True):
        b = _dev(b, torch.float64, self.device)
        if x0 is not None:
            if not self.opts.use_x0:
                raise ValueError("x0 given but the solver was built without use_x0=1")
            x = _dev(x0, torch.float64, self.device).clone()
        else:
            x = torch.empty(self.n, dtype=torch.float64, device=self.device)
        st = B.MgrStats()
        hist = np.zeros(max(self.opts.max_iter, 1) + 1)
        if history:
            st.res_history = hist.ctypes.data_as(C.POINTER(C.c_double))
            st.res_history_cap = hist.shape[0]
        rc = self.lib.mgr_solve(self.h, _ptr(b), _ptr(x), float(tol), C.byref(st))
        self._check(rc, allow=(B.OK, B.NOT_CONVERGED, B.E_BREAKDOWN))
        info = SolveInfo(rc, st.iterations, st.rel_residual, st.setup_ms, st.solve_ms,
                         list(st.level_n[: st.n_levels]), list(st.level_nnz[: st.n_levels]),
                         hist[: st.res_history_len].copy())
        return x, info

    def apply_preconditioner(self, r):
        r = _dev(r, torch.float64, self.device)
        z = torch.empty_like(r)
        self._check(self.lib.mgr_apply_preconditioner(self.h, _ptr(r), _ptr(z)))
        return z

    def spmv(self, x):
        x = _dev(x, torch.float64, self.device)
        y = torch.empty_like(x)
        self._check(self.lib.mgr_spmv(self.h, _ptr(x), _ptr(y)))
        return y

    def pattern_outer(self, lam, x):
        lam = _dev(lam, torch.float64, self.device)
        x = _dev(x, torch.float64, self.device)
        d = torch.empty(self.nnz, dtype=torch.float64, device=self.device)
        self._check(self.lib.mgr_pattern_outer(self.h, _ptr(lam), _ptr(x), _ptr(d)))
        return d

    # ---- introspection ----
    @property
    def levels(self):
        nm, na = C.c_int(), C.c_int()
        self._check(self.lib.mgr_num_levels(self.h, C.byref(nm), C.byref(na)))
        return nm.value, na.value

    def get_matrix(self, kind, level):
        """kind 0 MGR A_l, 1 MGR P_l, 2 MGR R_l, 3 AMG A_k, 4 AMG P_k, 5 AMG S_k.
        Returns (indptr int32, indices int32, data float64 or None, shape) on the host."""
        nr, nc, nz = C.c_int64(), C.c_int64(), C.c_int64()
        self._check(self.lib.mgr_get_matrix(self.h, kind, level, C.byref(nr), C.byref(nc), C.byref(nz),
                                            None, None, None))
        rp = np.empty(nr.value + 1, np.int32)
        ci = np.empty(max(nz.value, 1), np.int32)
        v = np.empty(max(nz.value, 1), np.float64) if kind != 5 else None
        self._check(self.lib.mgr_get_matrix(self.h, kind, level, None, None, None, rp.ctypes.data,
                                            ci.ctypes.data, v.ctypes.data if v is not None else None))
        return rp, ci[: nz.value], (v[: nz.value] if v is not None else None), (nr.value, nc.value)

    def get_vector(self, kind, level=0):
        """kind 0 cell-block inverses, 1 dinv_l, 2 F list_l, 3 C list_l, 4 AMG C/F_k,
        5 AMG l1_k, 6 coarsest LU, 7 coarsest LU permutation; 8..11 the same as 4..7
        for the F-relaxation AMG of MGR level l with level = (l << 8) | k."""
        n = C.c_int64()
        self._check(self.lib.mgr_get_vector(self.h, kind, level, None, C.byref(n)))
        dtype = np.int32 if kind in (2, 3, 4, 7, 8, 11) else np.float64
        out = np.empty(max(n.value, 1), dtype)
        self._check(self.lib.mgr_get_vector(self.h, kind, level, out.ctypes.data, C.byref(n)))
        return out[: n.value]

    # ---- timing of the fine-level kernel ----
    def set_kernel_timing(self, on=True):
        self._check(self.lib.mgr_set_kernel_timing(self.h, int(on)))

    def kernel_time(self, kernel=0):
        """(total ms, launches, algorithmic bytes) since timing was switched on or
        last read; kernel 0 = level-0 sliced-ELL kernel, 1 = whole V-cycles,
        2 = the l1-Jacobi sweeps on the coarse-grid matrix."""
        ms, cnt, byt = C.c_double(), C.c_int64(), C.c_double()
        self._check(self.lib.mgr_kernel_time(self.h, int(kernel), C.byref(ms), C.byref(cnt), C.byref(byt)))
        return ms.value, cnt.value, byt.value


class MGRSolve(torch.autograd.Function):
    """x = A(values)^{-1} b.  Backward: lambda = A^{-T} g (hierarchy built on A^T),
    grad_b = lambda, grad_values = -lambda[row] * x[col] on the pattern."""

    @staticmethod
    def forward(ctx, values, b, problem):
        fwd = problem.solver(values, transpose=False)
        x, info = fwd.solve(b.detach(), problem.tol)
        if info.status != B.OK:
            raise B.MGRError(info.status, f"forward solve did not converge ({info.iterations} iterations)")
        problem.last_forward = info
        ctx.problem = problem
        ctx.save_for_backward(values, x)
        return x

    @staticmethod
    def backward(ctx, g):
        values, x = ctx.saved_tensors
        problem = ctx.problem
        adj = problem.solver(values, transpose=True)
        lam, info = adj.solve(g.contiguous(), problem.tol)
        if info.status != B.OK:
            raise B.MGRError(info.status, f"adjoint solve did not converge ({info.iterations} iterations)")
        problem.last_adjoint = info
        dvals = adj.pattern_outer(lam, x)
        return dvals, lam, None


class DifferentiableMGR:
    """A fixed sparsity pattern and C/F labels; call with (values, b) to get x with
    autograd support.  Hierarchies are cached per values tensor version."""

    def __init__(self, row_ptr, col_idx, labels, block_size=3, tol=1e-8, device="cuda", **opts):
        self.device = torch.device(device)
        self.row_ptr = _dev(row_ptr, torch.int32, self.device)
        self.col_idx = _dev(col_idx, torch.int32, self.device)
        self.labels = _dev(labels, torch.int32, self.device)
        self.block_size = block_size
        self.tol = tol
        self.opts = opts
        self._cache = {}
        self.last_forward = None
        self.last_adjoint = None

    def solver(self, values, transpose):
        key = (values.data_ptr(), values._version, bool(transpose))
        s = self._cache.get(key)
        if s is None:
            for k in [k for k in self._cache if k[2] == bool(transpose)]:
                self._cache.pop(k).close()
            s = MGRSolver(self.row_ptr, self.col_idx, values.detach(), self.labels, self.block_size,
                          transpose=transpose, device=self.device, **self.opts)
            self._cache[key] = s
        return s

    def __call__(self, values, b):
        return MGRSolve.apply(values, b, self)

    def close(self):
        for s in self._cache.values():
            s.close()
        self._cache.clear()
