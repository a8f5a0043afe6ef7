"""Full-size checks in the configuration the benchmark times: config 4 (128^3,
6.3M unknowns) with sampled outputs the oracle computes one by one and
properties that hold at any size, and config 5 (48^3) for the differentiable
solve against central finite differences."""
import numpy as np
import pytest

from synth import make_config

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


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cfg4_solve_certified(orc, cfg4, precision):
    s, g0 = cfg4
    if precision == "fp64":
        g = g0
    else:
        from paper_1801_08464_amd.solver import MGRSolver
        g = MGRSolver(s.indptr, s.indices, s.data, s.labels, precision="mixed", **SOLVER_OPTS)
    x, info = g.solve(s.b, 1e-8)
    print(f"[cfg4 {precision}] iterations {info.iterations} rel_res {info.rel_residual:.2e}", flush=True)
    assert info.status == 0
    x = x.cpu().numpy()
    A = orc.as_csr(s.indptr, s.indices, s.data)
    res = np.linalg.norm(s.b - orc.spmv(A, x)) / np.linalg.norm(s.b)
    assert res <= 1e-8
    assert np.linalg.norm(x - s.x_true) / np.linalg.norm(s.x_true) < 1e-3
    if g is not g0:
        g.close()


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
