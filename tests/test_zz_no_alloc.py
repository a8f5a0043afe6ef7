"""The allocation-free residual evaluation (mgr_ncp_eval_noalloc) against
mgr_ncp_eval, called through the C ABI: two calls in a row, the second on a
smaller system, each with the update u += alpha du, so the static scratch (norm
partials and counters) holds the previous call's contents when the next begins."""
import ctypes as C

import numpy as np
import pytest

from oracle import newton as NW
from synth import make_ncp_problem

pytestmark = pytest.mark.gpu


def _run(entry, g, u, du, alpha, labels0):
    import torch
    ud = torch.as_tensor(u, device="cuda").clone()
    dd = torch.as_tensor(du, device="cuda")
    g.labels.copy_(torch.as_tensor(labels0, device="cuda"))
    g.R.fill_(np.nan)
    rn, na, nch = C.c_double(), C.c_int64(), C.c_int64()
    stream = torch.cuda.current_stream().cuda_stream
    rc = entry(C.byref(g.csr), g.henry.data_ptr(), g.f.data_ptr(), ud.data_ptr(), dd.data_ptr(), float(alpha),
               g.R.data_ptr(), g.labels.data_ptr(), C.byref(rn), C.byref(na), C.byref(nch), stream)
    torch.cuda.synchronize()
    return rc, ud.cpu().numpy(), g.R.cpu().numpy(), g.labels.cpu().numpy(), rn.value, na.value, nch.value


def test_noalloc_eval_matches_allocating_eval(orc):
    from paper_1801_08464_amd import binding as B
    from paper_1801_08464_amd.newton import NCPNewton
    lib = B.load_library()
    # the larger system first, then a smaller one: the second call must not see
    # the first call's partial sums or counts
    for grid, seed in (((40, 36, 20), 3), ((7, 5), 4)):
        pr = make_ncp_problem(grid, 1.5, "ball" if len(grid) == 3 else "disk", 0.35, seed)
        print(f"[noalloc eval] grid={grid} n={pr.n}", flush=True)
        g = NCPNewton(pr.l_indptr, pr.l_indices, pr.l_data, pr.henry, pr.f)
        rng = np.random.default_rng(seed)
        u = pr.u_star + 0.2 * rng.standard_normal(pr.n)
        u[2::3][rng.random(pr.n_cells) < 0.2] = 0.0
        du = rng.standard_normal(pr.n)
        labels0 = NW.labels(rng.random(pr.n_cells) < 0.5)
        ref = _run(lib.mgr_ncp_eval, g, u, du, -0.5, labels0)
        new = _run(lib.mgr_ncp_eval_noalloc, g, u, du, -0.5, labels0)
        assert ref[0] == B.OK and new[0] == B.OK, (ref[0], new[0], B.last_error(None))
        for k, what in ((1, "u"), (2, "R"), (3, "labels")):
            np.testing.assert_array_equal(new[k], ref[k], err_msg=what)
        assert new[4] == ref[4] and new[5] == ref[5] and new[6] == ref[6], (new[4:], ref[4:])
        # and both equal the oracle's residual and active set at u + alpha du
        R, act = NW.residual(orc.as_csr(pr.l_indptr, pr.l_indices, pr.l_data), pr.henry, pr.f, u + (-0.5) * du)
        np.testing.assert_array_equal(new[2], R)
        np.testing.assert_array_equal(new[3], NW.labels(act))
        assert new[5] == int(act.sum())
        assert new[6] == int(np.any((NW.labels(act) != labels0).reshape(-1, 3), axis=1).sum())
        assert abs(new[4] - np.linalg.norm(R)) <= 1e-12 * np.linalg.norm(R)
        # a third call on the same system repeats the counts (they restart at zero)
        again = _run(lib.mgr_ncp_eval_noalloc, g, u, du, -0.5, labels0)
        assert again[4:] == new[4:]


def test_noalloc_eval_rejects_bad_input():
    import torch
    from paper_1801_08464_amd import binding as B
    lib = B.load_library()
    rp = torch.zeros(8, dtype=torch.int32, device="cuda")
    bad = B.MgrCsr(7, 0, rp.data_ptr(), None, None)
    rc = lib.mgr_ncp_eval_noalloc(C.byref(bad), rp.data_ptr(), rp.data_ptr(), rp.data_ptr(), None, 1.0,
                                  rp.data_ptr(), rp.data_ptr(), None, None, None, None)
    assert rc == B.E_INVALID
