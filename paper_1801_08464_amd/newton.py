"""Semi-smooth Newton outer loop (Section 3.1, algorithm "Semi-smooth Newton
Method") around the MGR-GMRES solver, for the complementarity system with
unknowns (p, rho, S) per cell.  Argument marshalling only: the residual, the
active set, the labels, the generalised Jacobian and the update run in the
library (mgr_ncp_eval, mgr_ncp_jacobian); each step solves J x = R with
MGR-GMRES (mgr_solve), then u -= x.  A step whose labels (active set) are those
of the hierarchy's setup keeps the Jacobian's pattern, so the hierarchy takes
the new values only (mgr_update_values); otherwise it is set up anew (mgr_setup).
"""
from __future__ import annotations

import ctypes as C
import time
from dataclasses import dataclass, field

import torch

from . import binding as B
from .solver import MGRSolver, _dev, _ptr


@dataclass
class NewtonStep:
    rnorm: float               # ||R(u)|| after the step (before it for step 0)
    nactive: int               # |A| at that u
    lin_iterations: int = 0
    lin_status: int = 0
    setup_ms: float = 0.0
    solve_ms: float = 0.0
    values_only: bool = False  # the hierarchy took new values on its setup's pattern


@dataclass
class NewtonResult:
    u: torch.Tensor
    converged: bool
    steps: list = field(default_factory=list)
    seconds: float = 0.0


class NCPNewton:
    """L: the two PDE rows of every cell as CSR (S rows empty or ignored);
    henry: H per cell; f: right-hand side of the PDE rows (n)."""

    def __init__(self, l_indptr, l_indices, l_data, henry, f, device="cuda"):
        if not torch.cuda.is_available():
            raise RuntimeError("NCPNewton needs a ROCm GPU (torch.cuda is unavailable)")
        self.lib = B.load_library()
        self.device = torch.device(device)
        self.rp = _dev(l_indptr, torch.int32, self.device)
        self.ci = _dev(l_indices, torch.int32, self.device)
        self.v = _dev(l_data, torch.float64, self.device)
        self.henry = _dev(henry, torch.float64, self.device)
        self.f = _dev(f, torch.float64, self.device)
        self.n = self.rp.numel() - 1
        if self.n % 3:
            raise ValueError("3 unknowns per cell expected")
        self.csr = B.MgrCsr(self.n, self.ci.numel(), _ptr(self.rp), _ptr(self.ci), _ptr(self.v))
        self.R = torch.empty(self.n, dtype=torch.float64, device=self.device)
        self.labels = torch.empty(self.n, dtype=torch.int32, device=self.device)
        cap = self.ci.numel() + 2 * (self.n // 3)
        self.Jrp = torch.empty(self.n + 1, dtype=torch.int32, device=self.device)
        self.Jci = torch.empty(cap, dtype=torch.int32, device=self.device)
        self.Jv = torch.empty(cap, dtype=torch.float64, device=self.device)

    def _stream(self):
        return torch.cuda.current_stream(self.device).cuda_stream

    def eval(self, u, du=None, alpha=1.0):
        """u += alpha du (if du is given), then R(u) and the labels; returns
        (||R||, |A|).  u is updated in place; self.nchanged is the number of
        cells whose labels the call changed."""
        rn, na, nch = C.c_double(), C.c_int64(), C.c_int64()
        rc = self.lib.mgr_ncp_eval(C.byref(self.csr), _ptr(self.henry), _ptr(self.f), _ptr(u),
                                   _ptr(du) if du is not None else None, float(alpha), _ptr(self.R),
                                   _ptr(self.labels), C.byref(rn), C.byref(na), C.byref(nch), self._stream())
        if rc != B.OK:
            raise B.MGRError(rc, B.last_error(None))
        self.nchanged = nch.value
        return rn.value, na.value

    def jacobian(self):
        """The generalised Jacobian for the current labels: (row_ptr, col_idx, values)."""
        nnz = C.c_int64()
        rc = self.lib.mgr_ncp_jacobian(C.byref(self.csr), _ptr(self.henry), _ptr(self.labels), _ptr(self.Jrp),
                                       _ptr(self.Jci), _ptr(self.Jv), self.Jci.numel(), C.byref(nnz),
                                       self._stream())
        if rc != B.OK:
            raise B.MGRError(rc, B.last_error(None))
        k = nnz.value
        return self.Jrp, self.Jci[:k], self.Jv[:k]

    def solve(self, u0=None, tol=1e-8, max_newton=30, lin_tol=1e-10, **solver_opts) -> NewtonResult:
        """Semi-smooth Newton from u0 (default 0) until ||R(u)|| <= tol ||R(u0)||."""
        t0 = time.perf_counter()
        u = torch.zeros(self.n, dtype=torch.float64, device=self.device) if u0 is None else \
            _dev(u0, torch.float64, self.device).clone()
        r0, na = self.eval(u)
        steps = [NewtonStep(r0, na)]
        rn = r0
        g = None
        try:
            for _ in range(max_newton):
                if rn <= tol * r0:
                    break
                rp, ci, vals = self.jacobian()
                values_only = g is not None and self.nchanged == 0
                if values_only:
                    g.update_values(vals)
                else:
                    if g is not None:
                        g.close()
                    g = MGRSolver(rp, ci, vals, self.labels, **solver_opts)
                x, info = g.solve(self.R, lin_tol, history=False)
                rn, na = self.eval(u, x, -1.0)
                steps.append(NewtonStep(rn, na, info.iterations, info.status, info.setup_ms, info.solve_ms,
                                        values_only))
        finally:
            if g is not None:
                g.close()
        torch.cuda.synchronize(self.device)
        return NewtonResult(u, rn <= tol * r0, steps, time.perf_counter() - t0)
