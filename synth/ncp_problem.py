"""Seeded synthetic nonlinear complementarity problem for the semi-smooth Newton
outer loop (Section 3.1, algorithm "Semi-smooth Newton Method").

Unknowns u = (p, rho, S) per cell as in ncp_jacobian.  The two PDE residual rows
of every cell are linear, H(u) = L u - f, with L the p and rho rows of the seeded
Jacobian of make_system (its S rows left empty).  The constraint of cell c is
Theta_c(u) = min(F_c, G_c) with F_c = S_c (the gas saturation) and
G_c = rho_c - H_c p_c (a Henry's-law-type bound between dissolved density and
pressure).  The orientation of G is chosen for well-posedness: eliminating p and
rho through the PDE rows leaves the complementarity problem S >= 0,
G = q + M S >= 0, S G = 0, and with this generator's coefficient signs M is
positive definite for G = rho - H p (a unique solution) but negative definite for
the opposite orientation (many solutions).  The two-phase Jacobian row is then
[-H_c, 1, 0], the generator's row [H_c, -1, 0] times -1.

A manufactured solution fixes f: the two-phase set of make_system (the seeded
region) is the active set of u*: there S* > 0 and G(u*) = 0; elsewhere S* = 0 and
G(u*) > 0.  Then f = L u* on the PDE rows, so R(u*) = 0 exactly up to rounding.

This module only builds inputs; the Newton iteration lives in the oracle and in
the library.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .ncp_jacobian import NCPSystem, make_system


@dataclass
class NCPProblem:
    system: NCPSystem        # the Jacobian at u* (its S rows follow the region)
    l_indptr: np.ndarray     # int32 n+1: L = the p and rho rows, S rows empty
    l_indices: np.ndarray    # int32
    l_data: np.ndarray       # float64
    henry: np.ndarray        # float64 per cell
    f: np.ndarray            # float64 n (zero on the S rows)
    u_star: np.ndarray       # float64 n
    active_star: np.ndarray  # bool per cell: the two-phase set of u*

    @property
    def n(self) -> int:
        return int(self.l_indptr.shape[0] - 1)

    @property
    def n_cells(self) -> int:
        return self.n // 3


def make_ncp_problem(grid, sigma, region, frac, seed) -> NCPProblem:
    s = make_system(grid, sigma, region, frac, seed)
    N, n = s.n_cells, s.n
    # L: copy the p and rho rows, leave the S rows empty
    keep = np.ones(n, dtype=bool)
    keep[2::3] = False
    lens = np.diff(s.indptr.astype(np.int64))
    lens = np.where(keep, lens, 0)
    l_indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=l_indptr[1:])
    mask = np.repeat(keep, np.diff(s.indptr.astype(np.int64)))
    l_indices = s.indices[mask]
    l_data = s.data[mask]
    # manufactured solution, drawn after the system from its own stream
    rng = np.random.Generator(np.random.PCG64([seed, 7]))
    two = s.two_phase
    p = rng.standard_normal(N)
    gap = np.where(two, 0.0, rng.uniform(0.1, 1.0, N))
    S = np.where(two, rng.uniform(0.1, 1.0, N), 0.0)
    u = np.empty(n)
    u[0::3] = p
    u[1::3] = s.henry * p + gap
    u[2::3] = S
    # f = L u* on the PDE rows (row sums in entry order), 0 on the S rows
    row_of = np.repeat(np.arange(n), np.diff(l_indptr))
    f = np.bincount(row_of, weights=l_data * u[l_indices], minlength=n)
    return NCPProblem(system=s, l_indptr=l_indptr.astype(np.int32), l_indices=l_indices.astype(np.int32),
                      l_data=np.ascontiguousarray(l_data), henry=s.henry.copy(), f=f, u_star=u,
                      active_star=two.copy())
