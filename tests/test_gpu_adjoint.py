"""The differentiable solve: adjoint MGR-GMRES on a hierarchy built on A^T and the
pattern scatter dL/dvals = -lambda x^T, against the oracle's adjoint, the
dot-product identity and central finite differences."""
import numpy as np
import pytest

from gpu_common import gpu_solver, oracle_csr, small_system
from synth import make_system

pytestmark = pytest.mark.gpu


def test_adjoint_matches_oracle_and_dot_identity(orc):
    s = small_system((16, 15, 4), seed=5, sigma=1.5, frac=0.35, region="ball")
    A = oracle_csr(orc, s)
    g = np.random.default_rng(3).standard_normal(s.n)
    lo = orc.adjoint(A, s.labels, g, tol=1e-8)
    adj = gpu_solver(s, transpose=True)
    lam, info = adj.solve(g, 1e-8)
    assert info.status == 0 and abs(info.iterations - lo.iterations) <= 1
    fwd = gpu_solver(s)
    x, _ = fwd.solve(s.b, 1e-12)
    lam2, _ = gpu_solver(s, transpose=True).solve(g, 1e-12)
    lhs = float(np.dot(g, x.cpu().numpy()))
    rhs = float(np.dot(lam2.cpu().numpy(), s.b))
    assert lhs == pytest.approx(rhs, rel=1e-10)
    # matched iterations against the oracle's adjoint
    am = gpu_solver(s, transpose=True, max_iter=lo.iterations)
    lm, _ = am.solve(g, 0.0)
    assert np.linalg.norm(lm.cpu().numpy() - lo.x) / np.linalg.norm(lo.x) <= 1e-8
    # the pattern scatter
    d = adj.pattern_outer(lam2, x).cpu().numpy()
    np.testing.assert_array_equal(d, orc.pattern_outer(A, lam2.cpu().numpy(), x.cpu().numpy()))


def test_autograd_function_against_finite_differences(orc):
    import torch
    from paper_1801_08464_amd.solver import DifferentiableMGR
    s = make_system((10, 9, 3), 1.5, "ball", 0.35, seed=5, n_obs=8)
    obs = torch.as_tensor(3 * s.obs_cells, device="cuda")
    prob = DifferentiableMGR(s.indptr, s.indices, s.labels, tol=1e-13)
    vals = torch.tensor(s.data, device="cuda", requires_grad=True)
    b = torch.tensor(s.b, device="cuda", requires_grad=True)
    x = prob(vals, b)
    loss = x[obs].sum()
    loss.backward()
    gv, gb = vals.grad.cpu().numpy(), b.grad.cpu().numpy()
    # oracle adjoint gives the same gradients
    A = oracle_csr(orc, s)
    gvec = np.zeros(s.n)
    gvec[3 * s.obs_cells] = 1.0
    lam = orc.adjoint(A, s.labels, gvec, tol=1e-13).x
    xo = orc.Oracle(A, s.labels).solve(s.b, 1e-13).x
    np.testing.assert_allclose(gb, lam, rtol=1e-8, atol=1e-10 * np.abs(lam).max())
    np.testing.assert_allclose(gv, orc.pattern_outer(A, lam, xo), rtol=1e-7, atol=1e-10 * np.abs(gv).max())

    def L(v, bb):
        with torch.no_grad():
            return float(prob(torch.tensor(v, device="cuda"), torch.tensor(bb, device="cuda"))[obs].sum())

    rng = np.random.default_rng(0)
    h = 1e-6
    for p in rng.choice(s.nnz, 6, replace=False):
        vp, vm = s.data.copy(), s.data.copy()
        vp[p] += h
        vm[p] -= h
        fd = (L(vp, s.b) - L(vm, s.b)) / (2 * h)
        assert fd == pytest.approx(gv[p], rel=1e-4, abs=1e-6 * np.abs(gv).max())
    for i in rng.choice(s.n, 4, replace=False):
        bp, bm = s.b.copy(), s.b.copy()
        bp[i] += h
        bm[i] -= h
        fd = (L(s.data, bp) - L(s.data, bm)) / (2 * h)
        assert fd == pytest.approx(gb[i], rel=1e-4, abs=1e-6 * np.abs(gb).max())
    prob.close()
