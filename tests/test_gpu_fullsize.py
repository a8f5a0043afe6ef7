"""Full-size checks in the configuration the benchmark times: config 4 (128^3,
6.3M unknowns) with sampled outputs the oracle computes one by one and
properties that hold at any size, and config 5 (48^3) for the differentiable
solve against central finite differences."""
import json
import os

import numpy as np
import pytest

from gpu_common import assert_vcycle_close
from synth import make_config, random_vector

pytestmark = pytest.mark.gpu

SOLVER_OPTS = dict(frelax_amg_mask=2, frelax_amg_pre=1, frelax_amg_post=1)


@pytest.fixture(scope="module")
def cfg4():
    s = make_config(4)
    from paper_1801_08464_amd.solver import MGRSolver
    g = MGRSolver(s.indptr, s.indices, s.data, s.labels, **SOLVER_OPTS)
    yield s, g
    g.close()


def test_cfg4_fine_spmv_sampled_rows_bitwise(orc, cfg4):
    s, g = cfg4
    x = np.random.default_rng(3).standard_normal(s.n)
    y = g.spmv(x).cpu().numpy()
    rows = np.random.default_rng(4).choice(s.n, 4000, replace=False)
    for i in rows:
        a, b = s.indptr[i], s.indptr[i + 1]
        acc = 0.0
        for p in range(a, b):
            acc += s.data[p] * x[s.indices[p]]
        assert y[i] == acc, i


def test_cfg4_level0_coarse_operator_closed_form(cfg4):
    # first reduction exact (A_FF = I on the single-phase constraint rows): A_1 = A_CC
    import scipy.sparse as sp
    s, g = cfg4
    rp, ci, v, shape = g.get_matrix(0, 1)
    C = np.where(s.labels > 0)[0]
    Acc = sp.csr_matrix((s.data, s.indices, s.indptr), shape=(s.n, s.n))[C][:, C]
    Acc.sort_indices()
    np.testing.assert_array_equal(rp, Acc.indptr)
    np.testing.assert_array_equal(ci, Acc.indices)
    np.testing.assert_array_equal(v, Acc.data)


def test_cfg4_galerkin_rows_against_oracle_spgemm(orc, cfg4):
    s, g = cfg4
    A = orc.as_csr(*g.get_matrix(3, 0)[:3])
    rp, ci, v, shape = g.get_matrix(4, 0)
    P = orc.as_csr(rp, ci, v, shape)
    T = orc.spgemm(A, P)
    PT = orc.transpose(P)
    crp, cci, cv, cshape = g.get_matrix(3, 1)
    rows = np.random.default_rng(5).choice(cshape[0], 300, replace=False)
    for i in rows:
        a, b = PT.indptr[i], PT.indptr[i + 1]
        row = orc.as_csr([0, b - a], PT.indices[a:b], PT.data[a:b], (1, PT.shape[1]))
        ref = orc.spgemm(row, T)
        np.testing.assert_array_equal(cci[crp[i]:crp[i + 1]], ref.indices)
        np.testing.assert_array_equal(cv[crp[i]:crp[i + 1]], ref.data)


def test_cfg4_pmis_invariants(cfg4):
    import scipy.sparse as sp
    s, g = cfg4
    cf = g.get_vector(4, 0)
    srp, sci, _, shape = g.get_matrix(5, 0)
    S = sp.csr_matrix((np.ones(sci.shape[0]), sci, srp), shape=shape)
    lam = np.asarray(S.sum(axis=0)).ravel()
    isC = (cf == 1).astype(float)
    strongC = S @ isC
    F = cf == -1
    assert np.all((lam[F] == 0) | (strongC[F] > 0))
    assert set(np.unique(cf)) <= {-1, 1}
    # no two C points depend strongly on each other
    Cm = sp.diags(isC) @ S @ sp.diags(isC)
    assert (Cm.multiply(Cm.T)).count_nonzero() == 0


def test_cfg4_level2_fblock_has_no_strong_connections(orc, cfg4):
    # the F-block of the last reduction (S in two-phase cells) at the benchmark
    # size: negative diagonal, only negative off-diagonals, so the classical
    # strength graph is empty and an F-block AMG could not coarsen it (one Jacobi
    # sweep relaxes it instead)
    import scipy.sparse as sp
    s, g = cfg4
    rp, ci, v, shape = g.get_matrix(0, 2)
    M = sp.csr_matrix((v, ci, rp), shape=shape)
    F = g.get_vector(2, 2)
    Aff = M[F][:, F].tocsr()
    Aff.sort_indices()
    dg = Aff.diagonal()
    off = (Aff - sp.diags(dg)).tocsr()
    off.eliminate_zeros()
    print(f"[cfg4 level-2 A_FF] rows {Aff.shape[0]} off-diagonals {off.nnz}", flush=True)
    assert Aff.shape[0] == int(0.3 * 128 ** 3 + 0.5) and off.nnz > 0
    assert np.all(dg < 0) and np.all(off.data < 0)
    S = orc.strength(orc.from_scipy(Aff))
    assert S.indices.shape[0] == 0


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_solve_cfg4.json")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cfg4_column_forms_bitwise(cfg4, precision):
    """The solve-phase copies with 16-bit column offsets (the default: the
    level-0 operator's sliced ELL, and in the mixed-precision hierarchy the
    coarse-grid matrix's jagged copy) and with 32-bit columns give the same
    V-cycle and the same solve, bit for bit: config 4's coarse-grid matrix
    (2,097,152 rows, 24 entries per row) takes the jagged copy.  The FP64
    hierarchy's jagged copies keep 32-bit columns either way."""
    import torch
    from paper_1801_08464_amd.solver import MGRSolver
    s, _ = cfg4
    r = random_vector(s.n, 43)
    out = {}
    for c16 in (1, 0):
        print(f"[config 4 {precision}] index16={c16}", flush=True)
        g = MGRSolver(s.indptr, s.indices, s.data, s.labels, precision=precision, index16=c16, **SOLVER_OPTS)
        g.set_kernel_timing(True)
        z = g.apply_preconditioner(r).cpu().numpy()
        _, sweeps, sweep_bytes = g.kernel_time(2)
        _, fines, fine_bytes = g.kernel_time(0)
        g.set_kernel_timing(False)
        x, info = g.solve(s.b, 1e-8)
        out[c16] = (z, x.cpu().numpy(), info.iterations, sweep_bytes / sweeps, info.level_nnz[3], fine_bytes / fines)
        g.close()
        torch.cuda.synchronize()
    # the coarse-grid sweeps read 2 bytes less per entry in the 16-bit form (and
    # 4 more per slot-table entry): the form was taken where it applies
    nnz3 = out[1][4]  # the coarse grid A_3 follows the three MGR levels
    if precision == "mixed":
        assert out[0][3] - out[1][3] > 1.9 * nnz3, (out[0][3], out[1][3], nnz3)
    else:
        assert out[0][3] == out[1][3], (out[0][3], out[1][3])
    # and so does the level-0 operator (the V-cycle's level-0 residual)
    assert out[0][5] - out[1][5] > 1.9 * s.nnz, (out[0][5], out[1][5], s.nnz)
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][2] == out[1][2]
    assert np.array_equal(out[0][1], out[1][1])


@pytest.fixture(scope="module")
def golden4():
    with open(GOLDEN) as f:
        return json.load(f)


def _form(cfg4, precision):
    s, g0 = cfg4
    if precision == "fp64":
        return g0, False
    from paper_1801_08464_amd.solver import MGRSolver
    return MGRSolver(s.indptr, s.indices, s.data, s.labels, precision="mixed", **SOLVER_OPTS), True


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cfg4_vcycle_elementwise(orc, cfg4, precision):
    # one V-cycle of the benchmark's hierarchy (the 2.1 M-row coarse-grid sweeps,
    # AMG level 1 of 0.70 M rows, the F-block AMG of 2.1 M rows, the full
    # XCD-grouped grids) against the oracle's, entry by entry
    s, _ = cfg4
    o = orc.Oracle(orc.as_csr(s.indptr, s.indices, s.data), s.labels, precision=1 if precision == "mixed" else 0,
                   **SOLVER_OPTS)
    r = random_vector(s.n, 44)
    ze = o.vcycle(r)
    o.close()
    g, own = _form(cfg4, precision)
    z = g.apply_preconditioner(r).cpu().numpy()
    if own:
        g.close()
    assert_vcycle_close(z, ze, precision, "config 4")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cfg4_solve_matches_oracle_record(orc, cfg4, golden4, precision):
    # the oracle's converged solves of this very system (FP64, and the FP32-apply
    # mode for the mixed form), stored by tests/golden/make_oracle_solutions.py
    s, _ = cfg4
    assert s.fingerprint() == golden4["input_sha256"], "regenerated config 4 differs from the stored oracle run"
    rec = golden4["fp64" if precision == "fp64" else "fp32_apply"]
    assert rec["status"] == 0
    g, own = _form(cfg4, precision)
    x, info = g.solve(s.b, 1e-8)
    if own:
        g.close()
    print(f"[cfg4 {precision}] iterations {info.iterations} (oracle {rec['iterations']}) "
          f"rel_res {info.rel_residual:.2e}", flush=True)
    assert info.status == 0
    assert abs(info.iterations - rec["iterations"]) <= 1, (info.iterations, rec["iterations"])
    assert info.level_n == rec["level_n"] and info.level_nnz == rec["level_nnz"]
    x = x.cpu().numpy()
    A = orc.as_csr(s.indptr, s.indices, s.data)
    res = np.linalg.norm(s.b - orc.spmv(A, x)) / np.linalg.norm(s.b)
    assert res <= 1e-8
    if precision != "fp64":
        return
    # matched-iteration mode: exactly the oracle's number of Arnoldi steps, tol = 0;
    # the stored solution is compared through its norm, eight seeded projections
    # (each sees every entry) and 4,096 seeded entries
    from paper_1801_08464_amd.solver import MGRSolver
    gm = MGRSolver(s.indptr, s.indices, s.data, s.labels, max_iter=rec["iterations"], **SOLVER_OPTS)
    xm, im = gm.solve(s.b, 0.0)
    gm.close()
    assert im.iterations == rec["iterations"]
    xm = xm.cpu().numpy()
    xo_norm = rec["x_norm"]
    idx = np.asarray(rec["sample_index"])
    xs = np.asarray(rec["x_sample"])
    err_sample = np.linalg.norm(xm[idx] - xs) / np.linalg.norm(xs)
    err_norm = abs(np.linalg.norm(xm) - xo_norm) / xo_norm
    err_proj = max(abs(float(np.dot(random_vector(s.n, golden4["projection_seed0"] + k), xm)) - p) /
                   (np.sqrt(s.n) * xo_norm) for k, p in enumerate(rec["projections"]))
    print(f"[cfg4 matched] sample {err_sample:.2e} norm {err_norm:.2e} projections {err_proj:.2e}", flush=True)
    assert err_sample <= 1e-8 and err_norm <= 1e-8 and err_proj <= 1e-8


def test_cfg5_adjoint_finite_differences_and_oracle(orc):
    import torch
    from paper_1801_08464_amd.solver import DifferentiableMGR, MGRSolver
    s = make_config(5)
    obs = 3 * s.obs_cells
    prob = DifferentiableMGR(s.indptr, s.indices, s.labels, tol=1e-12, **SOLVER_OPTS)
    vals = torch.tensor(s.data, device="cuda", requires_grad=True)
    b = torch.tensor(s.b, device="cuda", requires_grad=True)
    x = prob(vals, b)
    x[torch.as_tensor(obs, device="cuda")].sum().backward()
    gv, gb = vals.grad.cpu().numpy(), b.grad.cpu().numpy()
    print(f"[cfg5] forward its {prob.last_forward.iterations} adjoint its {prob.last_adjoint.iterations}", flush=True)
    x0 = x.detach()
    # the oracle's adjoint, matched iterations
    A = orc.as_csr(s.indptr, s.indices, s.data)
    gvec = np.zeros(s.n)
    gvec[obs] = 1.0
    lo = orc.adjoint(A, s.labels, gvec, tol=1e-8, **SOLVER_OPTS)
    am = MGRSolver(s.indptr, s.indices, s.data, s.labels, transpose=True, max_iter=lo.iterations, **SOLVER_OPTS)
    lm, _ = am.solve(gvec, 0.0)
    assert np.linalg.norm(lm.cpu().numpy() - lo.x) / np.linalg.norm(lo.x) <= 1e-8
    am.close()

    # Central differences with step 1e-6.  Each perturbed system A' x' = b' is solved
    # as a correction from x0 (A' d = b' - A' x0, x' = x0 + d) so that the solver
    # tolerance applies to the small correction; L(x') - L(x'') = L(d') - L(d'').
    import scipy.sparse as sp
    xh = x0.cpu().numpy()
    Asp = sp.csr_matrix((s.data, s.indices, s.indptr), shape=(s.n, s.n))
    r0 = s.b - Asp @ xh
    rows = np.repeat(np.arange(s.n), np.diff(s.indptr))

    def dloss(v, rhs):
        g = MGRSolver(s.indptr, s.indices, v, s.labels, **SOLVER_OPTS)
        d, info = g.solve(rhs, 1e-10)
        g.close()
        assert info.status == 0
        return float(d.cpu().numpy()[obs].sum())

    rng = np.random.default_rng(18)
    h = 1e-6
    scale_v, scale_b = np.abs(gv).max(), np.abs(gb).max()
    checked = 0
    for p in rng.choice(s.nnz, 32, replace=False):
        i, j = rows[p], s.indices[p]
        vp, vm = s.data.copy(), s.data.copy()
        vp[p] += h
        vm[p] -= h
        rp, rm = r0.copy(), r0.copy()
        rp[i] -= h * xh[j]
        rm[i] += h * xh[j]
        fd = (dloss(vp, rp) - dloss(vm, rm)) / (2 * h)
        assert abs(fd - gv[p]) <= 1e-4 * abs(gv[p]) + 1e-8 * scale_v, (p, fd, gv[p])
        checked += abs(gv[p]) >= 1e-2 * scale_v
    for i in rng.choice(s.n, 32, replace=False):
        rp, rm = r0.copy(), r0.copy()
        rp[i] += h
        rm[i] -= h
        fd = (dloss(s.data, rp) - dloss(s.data, rm)) / (2 * h)
        assert abs(fd - gb[i]) <= 1e-4 * abs(gb[i]) + 1e-8 * scale_b, (i, fd, gb[i])
        checked += abs(gb[i]) >= 1e-2 * scale_b
    print(f"[cfg5] finite differences: 64 entries, {checked} with |g| >= 1e-2 |g|_inf", flush=True)
    prob.close()
