"""Seeded synthetic Jacobians shaped like the linearised two-phase, two-component
NCP system of the paper (Section 2, eq. linear_system and eq. 2p2c_matrix).

This module only builds *inputs*: a CSR matrix, a right-hand side, the true
solution it was made from, the per-unknown C/F level labels and (optionally)
observation cells.  It holds none of the solver's arithmetic and imports
neither the oracle nor the HIP library; both sides read the same arrays.

Layout: cell c = i + nx*(j + ny*k); unknown u = 3c + v with v = 0 pressure p,
v = 1 dissolved-hydrogen density rho, v = 2 liquid saturation S.  The paper
orders the variables as (P_l, S_l, rho_l^h) (Section 2, end); the order here is
a symmetric permutation of it, with the complementarity row paired with S.

Rows of cell c (two-point flux, harmonic-mean transmissibility T_cd):
  p   row: diag m_w*(sum_d T_cd + T_b), off-diag -m_w*T_cd, S column +a_S
  rho row: p diag sum_d T_cd*w_cd, p off-diag -T_cd*w_cd (w per directed face),
           rho diag D*(sum_d T_cd + T_b) + acc_rho, rho off-diag -D*T_cd,
           S column -acc_S
  S   row: two-phase cells [H, -1, 0] (zero diagonal: the gas-present NCP row
           of Section 3.2), single-phase cells [0, 0, 1].
T_b = 2 k_c is a Dirichlet outlet on the x = max face; all other faces are
no-flow.  The accumulation signs make every 3x3 cell block invertible.

Level labels (u -> MGR level at which u is an F-point; the max label is the
final coarse grid solved by AMG), following the three-stage reduction of
Section 5:
  0  S in single-phase cells (constraint rows with a nonzero diagonal, C_33)
  1  rho in every cell (the second PDE variable)
  2  S in two-phase cells (constraint rows whose diagonal is zero in A)
  3  p (the pressure-like coarse grid)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

M_W = 1.0  # water-mass scaling of the pressure row


@dataclass
class NCPSystem:
    grid: tuple
    n_cells: int
    indptr: np.ndarray      # int32, n+1
    indices: np.ndarray     # int32, nnz (sorted within each row)
    data: np.ndarray        # float64, nnz
    b: np.ndarray           # float64, n  (b = A x_true)
    x_true: np.ndarray      # float64, n
    labels: np.ndarray      # int32, n
    two_phase: np.ndarray   # bool, n_cells
    obs_cells: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int64))
    henry: np.ndarray = field(default_factory=lambda: np.zeros(0))  # H per cell (S-row p coefficient)

    @property
    def n(self) -> int:
        return int(self.indptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.indices.shape[0])

    def scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.data, self.indices, self.indptr), shape=(self.n, self.n))

    def fingerprint(self) -> str:
        """SHA-256 over the bytes of the CSR arrays, the labels and b (to check
        that a stored result belongs to this very input)."""
        import hashlib
        h = hashlib.sha256()
        for a in (self.indptr, self.indices, self.data, self.labels, self.b):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()


# The five workloads: grid, permeability contrast sigma, two-phase region shape and
# fraction, seed, number of observation cells.
CONFIGS = {
    1: dict(grid=(32, 32), sigma=1.0, region="disk", frac=0.40, seed=1, n_obs=0),
    2: dict(grid=(256, 256), sigma=2.0, region="band", frac=0.30, seed=2, n_obs=0),
    3: dict(grid=(64, 64, 64), sigma=1.5, region="ball", frac=0.35, seed=3, n_obs=0),
    4: dict(grid=(128, 128, 128), sigma=2.0, region="ball", frac=0.30, seed=4, n_obs=0),
    5: dict(grid=(48, 48, 48), sigma=1.5, region="ball", frac=0.35, seed=5, n_obs=64),
}


def _neighbour_pairs(grid):
    """Directed faces (c, d) between face neighbours, ordered by c then d."""
    dims = len(grid)
    nx = grid[0]
    ny = grid[1]
    nz = grid[2] if dims == 3 else 1
    N = nx * ny * nz
    c = np.arange(N, dtype=np.int64)
    i = c % nx
    j = (c // nx) % ny
    k = c // (nx * ny)
    cs, ds = [], []
    # directions in ascending neighbour index: -z, -y, -x, +x, +y, +z
    steps = []
    if dims == 3:
        steps.append((k > 0, -nx * ny))
    steps.append((j > 0, -nx))
    steps.append((i > 0, -1))
    steps.append((i < nx - 1, 1))
    steps.append((j < ny - 1, nx))
    if dims == 3:
        steps.append((k < nz - 1, nx * ny))
    for mask, s in steps:
        cc = c[mask]
        cs.append(cc)
        ds.append(cc + s)
    cs = np.concatenate(cs)
    ds = np.concatenate(ds)
    order = np.lexsort((ds, cs))
    return cs[order], ds[order], (i, j, k), N


def _smooth(g, cs, ds, N, passes=3):
    deg = np.bincount(cs, minlength=N).astype(np.float64)
    for _ in range(passes):
        s = np.bincount(cs, weights=g[ds], minlength=N)
        g = (g + s) / (1.0 + deg)
    return g


def _region(rng, grid, ijk, N, region, frac):
    dims = len(grid)
    centres = [ijk[a].astype(np.float64) + 0.5 for a in range(dims)]
    m = int(round(frac * N))
    if region in ("disk", "ball"):
        if dims == 2:
            r = math.sqrt(frac * N / math.pi)
        else:
            r = (3.0 * frac * N / (4.0 * math.pi)) ** (1.0 / 3.0)
        u = rng.uniform(0.0, 1.0, dims)
        ctr = []
        for a in range(dims):
            lo, hi = r, grid[a] - r
            ctr.append(lo + u[a] * (hi - lo) if hi >= lo else grid[a] / 2.0)
        dist = sum((centres[a] - ctr[a]) ** 2 for a in range(dims))
    elif region == "band":
        theta = rng.uniform(0.0, math.pi)
        nrm = (-math.sin(theta), math.cos(theta))
        dist = np.abs((centres[0] - grid[0] / 2.0) * nrm[0] + (centres[1] - grid[1] / 2.0) * nrm[1])
    else:
        raise ValueError(f"unknown region {region!r}")
    order = np.argsort(dist, kind="stable")
    two = np.zeros(N, dtype=bool)
    two[order[:m]] = True
    return two


def make_system(grid, sigma, region, frac, seed, n_obs=0, smoothing_passes=3) -> NCPSystem:
    """Build one seeded NCP-shaped Jacobian with b = A x_true.

    Draw order (fixed): g; per-cell a_S, D, acc_rho, acc_S, H; per directed face
    w; region parameters; x_true; observation cells."""
    grid = tuple(int(g) for g in grid)
    if len(grid) not in (2, 3):
        raise ValueError("grid must be 2D or 3D")
    rng = np.random.Generator(np.random.PCG64(seed))
    cs, ds, ijk, N = _neighbour_pairs(grid)
    nd = cs.shape[0]

    g = rng.standard_normal(N)
    g = _smooth(g, cs, ds, N, smoothing_passes)
    sd = g.std()
    g = (g - g.mean()) / (sd if sd > 0 else 1.0)
    kperm = np.exp(sigma * g)

    a_S = rng.uniform(0.1, 1.0, N)
    D = rng.uniform(0.01, 0.1, N)
    acc_rho = rng.uniform(0.1, 1.0, N)
    acc_S = rng.uniform(0.1, 1.0, N)
    H = rng.uniform(0.5, 2.0, N)
    w = rng.uniform(0.1, 1.0, nd)
    two = _region(rng, grid, ijk, N, region, frac)
    n = 3 * N
    x_true = rng.standard_normal(n)
    obs = np.sort(rng.choice(N, size=n_obs, replace=False)) if n_obs > 0 else np.zeros(0, np.int64)

    T = 2.0 * kperm[cs] * kperm[ds] / (kperm[cs] + kperm[ds])
    sumT = np.bincount(cs, weights=T, minlength=N)
    sumTw = np.bincount(cs, weights=T * w, minlength=N)
    Tb = np.where(ijk[0] == grid[0] - 1, 2.0 * kperm, 0.0)
    cell = np.arange(N, dtype=np.int64)

    rows, cols, vals = [], [], []

    def put(r, c, v):
        rows.append(r)
        cols.append(c)
        vals.append(np.broadcast_to(np.asarray(v, dtype=np.float64), r.shape))

    # p rows
    put(3 * cs, 3 * ds, -M_W * T)
    put(3 * cell, 3 * cell, M_W * (sumT + Tb))
    put(3 * cell, 3 * cell + 2, a_S)
    # rho rows
    put(3 * cs + 1, 3 * ds, -T * w)
    put(3 * cs + 1, 3 * ds + 1, -D[cs] * T)
    put(3 * cell + 1, 3 * cell, sumTw)
    put(3 * cell + 1, 3 * cell + 1, D * (sumT + Tb) + acc_rho)
    put(3 * cell + 1, 3 * cell + 2, -acc_S)
    # S rows (complementarity)
    tp = cell[two]
    sp1 = cell[~two]
    put(3 * tp + 2, 3 * tp, H[tp])
    put(3 * tp + 2, 3 * tp + 1, np.full(tp.shape, -1.0))
    put(3 * sp1 + 2, 3 * sp1 + 2, np.ones(sp1.shape))

    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    A = sp.csr_matrix((v, (r, c)), shape=(n, n))
    A.sort_indices()
    if A.nnz != r.shape[0]:
        raise AssertionError("duplicate entries in the assembled Jacobian")
    indptr = A.indptr.astype(np.int32)
    indices = A.indices.astype(np.int32)
    data = np.ascontiguousarray(A.data, dtype=np.float64)
    b = A @ x_true

    labels = np.empty(n, dtype=np.int32)
    labels[0::3] = 3
    labels[1::3] = 1
    labels[2::3] = np.where(two, 2, 0)
    return NCPSystem(grid=grid, n_cells=N, indptr=indptr, indices=indices, data=data,
                     b=np.ascontiguousarray(b), x_true=x_true, labels=labels, two_phase=two,
                     obs_cells=obs, henry=H)


def make_config(cfg: int) -> NCPSystem:
    p = CONFIGS[cfg]
    return make_system(p["grid"], p["sigma"], p["region"], p["frac"], p["seed"], p["n_obs"])


def make_poisson(grid, seed=0):
    """Scalar pressure block with sigma = 0 (homogeneous permeability): the
    m_w-weighted 5/7-point Laplacian with the Dirichlet outlet.  Returns CSR
    arrays (indptr, indices, data) and a seeded right-hand side."""
    grid = tuple(int(g) for g in grid)
    cs, ds, ijk, N = _neighbour_pairs(grid)
    T = np.ones(cs.shape[0])
    sumT = np.bincount(cs, weights=T, minlength=N)
    Tb = np.where(ijk[0] == grid[0] - 1, 2.0, 0.0)
    cell = np.arange(N, dtype=np.int64)
    r = np.concatenate([cs, cell])
    c = np.concatenate([ds, cell])
    v = np.concatenate([-M_W * T, M_W * (sumT + Tb)])
    A = sp.csr_matrix((v, (r, c)), shape=(N, N))
    A.sort_indices()
    rng = np.random.Generator(np.random.PCG64(seed))
    b = rng.standard_normal(N)
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64), b


def random_vector(n, seed):
    """Seeded N(0,1) vector (used for parity inputs such as V-cycle residuals)."""
    return np.random.Generator(np.random.PCG64(seed)).standard_normal(n)
