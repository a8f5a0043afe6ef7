"""Parity of the library's semi-smooth Newton support (mgr_ncp_eval,
mgr_ncp_jacobian) and of the GPU Newton loop against the oracle (Section 3.1,
algorithm "Semi-smooth Newton Method")."""
import ctypes as C

import numpy as np
import pytest

from oracle import newton as NW
from synth import CONFIGS, make_ncp_problem

pytestmark = pytest.mark.gpu


def _gpu(pr):
    from paper_1801_08464_amd.newton import NCPNewton
    return NCPNewton(pr.l_indptr, pr.l_indices, pr.l_data, pr.henry, pr.f)


def _L(orc, pr):
    return orc.as_csr(pr.l_indptr, pr.l_indices, pr.l_data)


@pytest.mark.parametrize("grid", [(9, 7), (6, 5, 4)])
def test_residual_labels_and_update_bitwise(orc, grid):
    import torch
    pr = make_ncp_problem(grid, 1.5, "disk" if len(grid) == 2 else "ball", 0.35, 3)
    print(f"[ncp eval] grid={grid} n={pr.n}", flush=True)
    g = _gpu(pr)
    rng = np.random.default_rng(9)
    u = pr.u_star + 0.2 * rng.standard_normal(pr.n)
    u[2::3][rng.random(pr.n_cells) < 0.2] = 0.0
    du = rng.standard_normal(pr.n)
    ud = torch.as_tensor(u, device="cuda")
    rn, na = g.eval(ud)
    R, act = NW.residual(_L(orc, pr), pr.henry, pr.f, u)
    np.testing.assert_array_equal(g.R.cpu().numpy(), R)
    np.testing.assert_array_equal(g.labels.cpu().numpy(), NW.labels(act))
    assert na == int(act.sum())
    assert abs(rn - np.linalg.norm(R)) <= 1e-12 * np.linalg.norm(R)
    # the update u += alpha du happens before the evaluation
    rn2, na2 = g.eval(ud, torch.as_tensor(du, device="cuda"), -1.0)
    u2 = u + (-1.0) * du
    np.testing.assert_array_equal(ud.cpu().numpy(), u2)
    R2, act2 = NW.residual(_L(orc, pr), pr.henry, pr.f, u2)
    np.testing.assert_array_equal(g.R.cpu().numpy(), R2)
    assert na2 == int(act2.sum())


@pytest.mark.parametrize("grid", [(9, 7), (6, 5, 4)])
def test_jacobian_bitwise(orc, grid):
    import torch
    pr = make_ncp_problem(grid, 1.5, "disk" if len(grid) == 2 else "ball", 0.35, 3)
    g = _gpu(pr)
    for frac in (0.0, 0.3, 1.0):
        act = np.random.default_rng(4).random(pr.n_cells) < frac
        g.labels.copy_(torch.as_tensor(NW.labels(act), device="cuda"))
        rp, ci, v = g.jacobian()
        J = NW.jacobian(_L(orc, pr), pr.henry, act)
        np.testing.assert_array_equal(rp.cpu().numpy().astype(np.int64), J.indptr)
        np.testing.assert_array_equal(ci.cpu().numpy(), J.indices)
        np.testing.assert_array_equal(v.cpu().numpy(), J.data)
    # the generator's Jacobian (two-phase rows negated) at the active set of u*
    g.labels.copy_(torch.as_tensor(pr.system.labels, device="cuda"))
    rp, ci, v = g.jacobian()
    np.testing.assert_array_equal(ci.cpu().numpy(), pr.system.indices)


def test_jacobian_capacity_and_argument_errors(orc):
    import torch
    from paper_1801_08464_amd import binding as B
    pr = make_ncp_problem((5, 4), 1.0, "disk", 0.4, 2)
    g = _gpu(pr)
    g.labels.copy_(torch.as_tensor(pr.system.labels, device="cuda"))
    nnz = C.c_int64()
    stream = torch.cuda.current_stream().cuda_stream
    rc = g.lib.mgr_ncp_jacobian(C.byref(g.csr), g.henry.data_ptr(), g.labels.data_ptr(), g.Jrp.data_ptr(),
                                g.Jci.data_ptr(), g.Jv.data_ptr(), 10, C.byref(nnz), stream)
    assert rc == B.E_INVALID and nnz.value == pr.system.nnz
    assert "capacity" in B.last_error(None)
    bad = B.MgrCsr(7, 0, g.csr.row_ptr, None, None)
    rc = g.lib.mgr_ncp_eval(C.byref(bad), g.henry.data_ptr(), g.f.data_ptr(), g.R.data_ptr(), None, 1.0,
                            g.R.data_ptr(), g.labels.data_ptr(), None, None, None, stream)
    assert rc == B.E_INVALID


@pytest.mark.parametrize("grid,start", [((12, 10), "zero"), ((12, 10), "previous"), ((8, 8, 8), "zero"),
                                        ((8, 8, 8), "perturbed"), ((8, 8, 8), "previous")])
def test_newton_matches_oracle(orc, grid, start):
    reg = "disk" if len(grid) == 2 else "ball"
    pr = make_ncp_problem(grid, 1.5, reg, 0.35, 5)
    u0 = {"zero": None,
          "perturbed": pr.u_star + 0.05 * np.random.default_rng(1).standard_normal(pr.n),
          "previous": make_ncp_problem(grid, 1.5, reg, 0.25, 5).u_star}[start]
    print(f"[newton] grid={grid} start={start}", flush=True)
    uo, ho = NW.newton(_L(orc, pr), pr.henry, pr.f, u0=u0, frelax_amg_mask=2)
    res = _gpu(pr).solve(u0=u0, frelax_amg_mask=2)
    assert res.converged
    # the same active-set sequence and number of steps as the oracle
    assert [s.nactive for s in res.steps] == [h["nactive"] for h in ho]
    for s, h in zip(res.steps[1:], ho[1:]):
        assert s.lin_status == 0 and abs(s.lin_iterations - h["lin_its"]) <= 1
    u = res.u.cpu().numpy()
    assert np.linalg.norm(u - pr.u_star) <= 1e-10 * np.linalg.norm(pr.u_star)
    assert np.linalg.norm(u - uo) <= 1e-10 * np.linalg.norm(uo)


def test_newton_at_benchmark_size():
    # the workload of the benchmark's Newton form: the 64^3 grid of the
    # mixed-precision parity case, started from a smaller two-phase region
    p = CONFIGS[3]
    pr = make_ncp_problem(p["grid"], p["sigma"], p["region"], p["frac"], p["seed"])
    prev = make_ncp_problem(p["grid"], p["sigma"], p["region"], 0.8 * p["frac"], p["seed"])
    print(f"[newton full] n={pr.n}", flush=True)
    res = _gpu(pr).solve(u0=prev.u_star, frelax_amg_mask=2)
    print(f"[newton full] steps={len(res.steps) - 1} values-only updates="
          f"{sum(s.values_only for s in res.steps[1:])}", flush=True)
    assert res.converged and len(res.steps) - 1 <= 10
    u = res.u.cpu().numpy()
    assert np.linalg.norm(u - pr.u_star) <= 1e-9 * np.linalg.norm(pr.u_star)
    # the final active set is the manufactured one
    assert res.steps[-1].nactive == int(pr.active_star.sum())
