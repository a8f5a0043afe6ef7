"""Semi-smooth Newton outer loop of the paper (Section 3.1, algorithm "Semi-smooth
Newton Method") on the synthetic complementarity problem of synth.ncp_problem.

TEST INFRASTRUCTURE ONLY: plain numpy around the C oracle's SpMV and MGR-GMRES.
Only tests/, the smoke check and the benchmark's CPU-baseline leg may use it.

Residual R(u) = [H(u); Theta(u)] per cell: the PDE rows H(u) = L u - f (L the p
and rho rows, row sums in ascending column order), and the constraint
Theta_c = min(F_c, G_c) with F_c = S_c and G_c = rho_c - H_c p_c.

Step (1) of the algorithm: the active set A = {c : F_c >= G_c} (there the minimum
is G), the inactive set I = {c : F_c < G_c}.  Step (2): the constraint row of the
generalised Jacobian is G' = [-H_c, 1, 0] on A (a zero diagonal: the gas-present
row) and F' = [0, 0, 1] on I; the PDE rows are L.  Step (3): solve J du = -R with
MGR-GMRES (labels: p -> 3, rho -> 1, S -> 2 on A and 0 on I, the three-stage
reduction of Section 5).  Step (4): u <- u + du.
"""
from __future__ import annotations

import numpy as np

from . import oracle as O


def residual(L: O.CSR, henry, f, u):
    """R(u) and the active set (bool per cell)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    Lu = O.spmv(L, u)
    R = np.zeros_like(u)
    R[0::3] = Lu[0::3] - f[0::3]
    R[1::3] = Lu[1::3] - f[1::3]
    F = u[2::3]
    G = u[1::3] - henry * u[0::3]
    active = F >= G
    R[2::3] = np.where(active, G, F)  # min(F, G)
    return R, active


def labels(active):
    lab = np.empty(3 * active.shape[0], dtype=np.int32)
    lab[0::3] = 3
    lab[1::3] = 1
    lab[2::3] = np.where(active, 2, 0)
    return lab


def jacobian(L: O.CSR, henry, active) -> O.CSR:
    """The generalised Jacobian: the rows of L, and per cell the constraint row
    [-H_c, 1] at (p, rho) if active, [1] at S if not (columns ascending)."""
    n = L.shape[0]
    N = n // 3
    lens = np.diff(L.indptr)
    lens[2::3] = np.where(active, 2, 1)
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=indptr[1:])
    indices = np.empty(indptr[-1], dtype=np.int32)
    data = np.empty(indptr[-1])
    # the PDE rows: entry q of L row r goes to position indptr[r] + (q - L.indptr[r])
    row_of = np.repeat(np.arange(n), np.diff(L.indptr))
    dest = indptr[row_of] + (np.arange(L.indices.shape[0]) - L.indptr[row_of])
    indices[dest] = L.indices
    data[dest] = L.data
    c = np.arange(N)
    s_rows = 3 * c + 2
    start = indptr[s_rows]
    act = np.nonzero(active)[0]
    ina = np.nonzero(~active)[0]
    indices[start[act]] = 3 * act
    data[start[act]] = -henry[act]
    indices[start[act] + 1] = 3 * act + 1
    data[start[act] + 1] = 1.0
    indices[start[ina]] = 3 * ina + 2
    data[start[ina]] = 1.0
    return O.CSR(indptr, indices, data, (n, n))


def newton(L: O.CSR, henry, f, u0=None, tol=1e-8, max_newton=30, lin_tol=1e-10, **solver_opts):
    """Run the semi-smooth Newton iteration from u0 (default 0) until
    ||R(u)|| <= tol ||R(u0)||.  Returns (u, history); history[k] holds the
    residual norm, the active-set size and the linear iterations of step k."""
    n = L.shape[0]
    u = np.zeros(n) if u0 is None else np.array(u0, dtype=np.float64)
    R, active = residual(L, henry, f, u)
    r0 = float(np.linalg.norm(R))
    hist = [dict(rnorm=r0, nactive=int(active.sum()), lin_its=0, lin_status=0)]
    for _ in range(max_newton):
        if float(np.linalg.norm(R)) <= tol * r0:
            break
        J = jacobian(L, henry, active)
        o = O.Oracle(J, labels(active), **solver_opts)
        res = o.solve(-R, lin_tol)
        o.close()
        u = u + res.x
        R, active = residual(L, henry, f, u)
        hist.append(dict(rnorm=float(np.linalg.norm(R)), nactive=int(active.sum()), lin_its=res.iterations,
                         lin_status=res.status))
    return u, hist
