"""Pins of the oracle's semi-smooth Newton outer loop (Section 3.1, algorithm
"Semi-smooth Newton Method") on the synthetic complementarity problem: the
manufactured root, the generalised Jacobian against the generator's matrix, the
well-posedness of the reduced complementarity problem with brute force over all
active sets on a tiny grid, and convergence from several starts (CPU only)."""
import itertools

import numpy as np
import pytest

from oracle import newton as NW
from synth import make_ncp_problem


def _L(orc, pr):
    return orc.as_csr(pr.l_indptr, pr.l_indices, pr.l_data)


@pytest.mark.parametrize("grid", [(7, 6), (5, 4, 3)])
def test_manufactured_solution_is_a_root(orc, grid):
    pr = make_ncp_problem(grid, 1.5, "disk" if len(grid) == 2 else "ball", 0.35, 2)
    R, act = NW.residual(_L(orc, pr), pr.henry, pr.f, pr.u_star)
    assert np.all(R == 0.0)
    np.testing.assert_array_equal(act, pr.active_star)
    # the tie F = G counts as active (A = {F >= G}): at u = 0 every cell is active
    _, act0 = NW.residual(_L(orc, pr), pr.henry, pr.f, np.zeros(pr.n))
    assert act0.all()


@pytest.mark.parametrize("grid", [(7, 6), (5, 4, 3)])
def test_jacobian_is_the_generator_matrix(orc, grid):
    # at the active set of u*, the generalised Jacobian is the seeded Jacobian with
    # the two-phase constraint rows negated (G = rho - H p), and the labels agree
    pr = make_ncp_problem(grid, 1.5, "disk" if len(grid) == 2 else "ball", 0.35, 2)
    s = pr.system
    J = NW.jacobian(_L(orc, pr), pr.henry, pr.active_star)
    np.testing.assert_array_equal(J.indptr, s.indptr)
    np.testing.assert_array_equal(J.indices, s.indices)
    want = s.data.copy()
    two_rows = 3 * np.nonzero(s.two_phase)[0] + 2
    for r in two_rows:
        want[s.indptr[r]:s.indptr[r + 1]] *= -1.0
    np.testing.assert_array_equal(J.data, want)
    np.testing.assert_array_equal(NW.labels(pr.active_star), s.labels)


def test_tiny_problem_has_one_complementary_solution(orc):
    # eliminate p and rho: G = q + M S with M positive definite, so exactly one of
    # the 2^N active sets gives S >= 0 on A, G = 0 on A, S = 0 and G >= 0 on I
    pr = make_ncp_problem((3, 3), 1.0, "disk", 0.4, 4)
    n, N = pr.n, pr.n_cells
    Ld = orc.to_scipy(_L(orc, pr)).toarray()
    pde = np.sort(np.r_[np.arange(0, n, 3), np.arange(1, n, 3)])
    K, B = Ld[np.ix_(pde, pde)], Ld[np.ix_(pde, np.arange(2, n, 3))]
    E = np.zeros((N, pde.size))
    where = {v: i for i, v in enumerate(pde)}
    for c in range(N):
        E[c, where[3 * c]] = -pr.henry[c]
        E[c, where[3 * c + 1]] = 1.0
    M = -E @ np.linalg.solve(K, B)
    assert np.linalg.eigvals(M).real.min() > 0
    feasible = []
    for bits in itertools.product([False, True], repeat=N):
        act = np.array(bits)
        J = orc.to_scipy(NW.jacobian(_L(orc, pr), pr.henry, act)).toarray()
        rhs = pr.f.copy()
        rhs[2::3] = 0.0
        u = np.linalg.solve(J, rhs)
        S, G = u[2::3], u[1::3] - pr.henry * u[0::3]
        tol = 1e-12 * np.abs(u).max()
        if np.all(S[act] >= -tol) and np.all(G[~act] >= -tol):
            feasible.append((act, u))
    assert len(feasible) == 1
    np.testing.assert_array_equal(feasible[0][0], pr.active_star)
    np.testing.assert_allclose(feasible[0][1], pr.u_star, rtol=1e-10, atol=1e-12)


def test_newton_step_solves_the_generalised_system(orc):
    # step (3): the MGR-GMRES correction equals the dense solve of J du = -R
    pr = make_ncp_problem((8, 7), 1.5, "disk", 0.35, 6)
    L = _L(orc, pr)
    u0 = pr.u_star + 0.3 * np.random.default_rng(0).standard_normal(pr.n)
    R, act = NW.residual(L, pr.henry, pr.f, u0)
    J = NW.jacobian(L, pr.henry, act)
    res = orc.Oracle(J, NW.labels(act), frelax_amg_mask=2).solve(-R, 1e-12)
    du = np.linalg.solve(orc.to_scipy(J).toarray(), -R)
    np.testing.assert_allclose(res.x, du, rtol=1e-9, atol=1e-10 * np.abs(du).max())


@pytest.mark.parametrize("grid", [(12, 10), (8, 8, 8)])
@pytest.mark.parametrize("start", ["zero", "perturbed", "previous"])
def test_newton_converges_to_the_manufactured_solution(orc, grid, start):
    reg = "disk" if len(grid) == 2 else "ball"
    pr = make_ncp_problem(grid, 1.5, reg, 0.35, 5)
    u0 = {"zero": None,
          "perturbed": pr.u_star + 0.05 * np.random.default_rng(1).standard_normal(pr.n),
          "previous": make_ncp_problem(grid, 1.5, reg, 0.25, 5).u_star}[start]
    u, hist = NW.newton(_L(orc, pr), pr.henry, pr.f, u0=u0, frelax_amg_mask=2)
    assert len(hist) - 1 <= 8
    assert all(h["lin_status"] == 0 for h in hist)
    assert np.linalg.norm(u - pr.u_star) <= 1e-10 * np.linalg.norm(pr.u_star)
    _, act = NW.residual(_L(orc, pr), pr.henry, pr.f, u)
    np.testing.assert_array_equal(act, pr.active_star)
    # finite termination: the last step keeps the active set
    assert hist[-1]["nactive"] == hist[-2]["nactive"] == int(pr.active_star.sum())
