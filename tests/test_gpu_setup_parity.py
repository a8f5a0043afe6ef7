"""Setup parity: every hierarchy object built on the GPU is bit-for-bit equal to
the oracle's (C/F splits, patterns and values), on seeded systems that span
several 64-cell slices with a ragged last slice."""
import numpy as np
import pytest

from gpu_common import assert_same_csr, gpu_solver, oracle_csr, small_system
from synth import make_config, make_poisson

pytestmark = pytest.mark.gpu

def long_row_system():
    """A 12^3 system whose first pressure row also couples to the pressure of 300
    other cells (row sum kept): the Galerkin products then hold rows of more
    than 256 entries (up to 506 on AMG level 1), and the SpGEMM count recounts
    with the group of the longest left-operand row."""
    import scipy.sparse as sp
    s = small_system((12, 12, 12), seed=5, sigma=2.0, frac=0.3, region="ball")
    assert s.labels[0] == 3
    A = sp.csr_matrix((s.data, s.indices, s.indptr), shape=(s.n, s.n))
    cells = np.arange(5, 5 + 5 * 300, 5)
    eps = 1e-3 * A[0, 0]
    extra = sp.csr_matrix((np.r_[np.full(300, -eps), [300 * eps]], (np.zeros(301, int), np.r_[3 * cells, [0]])),
                          shape=A.shape)
    A = (A + extra).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return s.__class__(**{**s.__dict__, "indptr": A.indptr.astype(np.int32), "indices": A.indices.astype(np.int32),
                          "data": A.data.astype(np.float64)})


CASES = {
    "cfg1_32x32": lambda: make_config(1),
    "2d_37x29_band": lambda: small_system((37, 29), seed=8, sigma=2.0, frac=0.3, region="band"),
    "3d_13x11x9_ball": lambda: small_system((13, 11, 9), seed=4, sigma=2.0, frac=0.3, region="ball"),
    "3d_12cube_long_row": long_row_system,
}


def compare_hierarchy(orc, s, **opts):
    o = orc.Oracle(oracle_csr(orc, s), s.labels, **opts)
    g = gpu_solver(s, **{k: v for k, v in opts.items() if k != "precision"})
    try:
        check_hierarchy(g, o, **opts)
    finally:
        g.close()
        o.close()


def check_hierarchy(g, o, **opts):
    nm, na = g.levels
    assert (nm, na) == (o.n_mgr_levels, o.n_amg_levels)
    if o.n_mgr_levels > 0 and opts.get("global_relax", 1):
        np.testing.assert_array_equal(g.get_vector(0), o.block_inverses(), err_msg="cell-block inverses")
    for l in range(nm):
        ol = o.mgr_level(l)
        assert_same_csr(g.get_matrix(0, l), ol["A"], f"MGR A_{l}")
        assert_same_csr(g.get_matrix(1, l), ol["P"], f"MGR P_{l}")
        assert_same_csr(g.get_matrix(2, l), ol["R"], f"MGR R_{l}")
        np.testing.assert_array_equal(g.get_vector(1, l), ol["dinv"], err_msg=f"dinv_{l}")
        np.testing.assert_array_equal(g.get_vector(2, l), ol["flist"], err_msg=f"F list {l}")
        np.testing.assert_array_equal(g.get_vector(3, l), ol["clist"], err_msg=f"C list {l}")
    for k in range(na):
        ok = o.amg_level(k)
        assert_same_csr(g.get_matrix(3, k), ok["A"], f"AMG A_{k}")
        if k < na - 1:
            np.testing.assert_array_equal(g.get_vector(4, k), ok["cf"], err_msg=f"AMG C/F split {k}")
            assert_same_csr(g.get_matrix(5, k), ok["S"], f"AMG strength {k}")
            assert_same_csr(g.get_matrix(4, k), ok["P"], f"AMG P_{k}")
            np.testing.assert_array_equal(g.get_vector(5, k), ok["l1"], err_msg=f"AMG l1 {k}")
    lu, perm = o.coarse_lu()
    np.testing.assert_array_equal(g.get_vector(7), perm, err_msg="coarsest LU permutation")
    np.testing.assert_array_equal(g.get_vector(6), lu.ravel(), err_msg="coarsest LU factors")
    for l in range(nm):
        nff = o.n_ff_levels(l)
        for k in range(nff):
            code = (l << 8) | k
            ok = o.ff_level(l, k)
            assert_same_csr(g.get_matrix(6, code), ok["A"], f"F-block AMG A_{k} of level {l}")
            if k < nff - 1:
                assert_same_csr(g.get_matrix(7, code), ok["P"], f"F-block AMG P_{k} of level {l}")
                np.testing.assert_array_equal(g.get_vector(8, code), ok["cf"])
                np.testing.assert_array_equal(g.get_vector(9, code), ok["l1"])
        if nff:
            flu, fperm = o.ff_coarse_lu(l)
            np.testing.assert_array_equal(g.get_vector(11, l << 8), fperm)
            np.testing.assert_array_equal(g.get_vector(10, l << 8), flu.ravel())
        else:
            with pytest.raises(Exception):
                g.get_matrix(6, l << 8)


@pytest.mark.parametrize("case", sorted(CASES))
def test_hierarchy_bitwise(orc, case):
    s = CASES[case]()
    print(f"[setup parity] {case} n={s.n} nnz={s.nnz}", flush=True)
    compare_hierarchy(orc, s)


@pytest.mark.parametrize("opts", [dict(rp_type=1), dict(rp_type=2), dict(global_relax=0),
                                  dict(amg_theta=0.5, pmis_seed=12345), dict(amg_coarse_max=10),
                                  dict(frelax_amg_mask=2), dict(frelax_amg_mask=2, amg_coarse_max=20,
                                                                frelax_amg_pre=2, frelax_amg_post=0)])
def test_hierarchy_bitwise_options(orc, opts):
    s = small_system((19, 17), seed=6)
    print(f"[setup parity] options {opts}", flush=True)
    compare_hierarchy(orc, s, **opts)


def test_hierarchy_bitwise_transpose(orc):
    s = small_system((23, 21), seed=2)
    At = orc.transpose(oracle_csr(orc, s))
    o = orc.Oracle(At, s.labels)
    g = gpu_solver(s, transpose=True)
    try:
        for l in range(o.n_mgr_levels):
            assert_same_csr(g.get_matrix(0, l), o.mgr_level(l)["A"], f"A^T hierarchy level {l}")
        for k in range(o.n_amg_levels):
            assert_same_csr(g.get_matrix(3, k), o.amg_level(k)["A"], f"A^T AMG level {k}")
    finally:
        g.close()


def test_plain_amg_poisson_bitwise(orc):
    ip, ix, dv, _ = make_poisson((45, 39))
    n = ip.shape[0] - 1

    class S:  # minimal system record
        pass
    s = S()
    s.indptr, s.indices, s.data, s.labels = ip, ix, dv, np.zeros(n, np.int32)
    o = orc.Oracle(orc.as_csr(ip, ix, dv), s.labels, block_size=1)
    g = gpu_solver(s, block_size=1)
    try:
        assert g.levels == (0, o.n_amg_levels)
        for k in range(o.n_amg_levels):
            assert_same_csr(g.get_matrix(3, k), o.amg_level(k)["A"], f"AMG A_{k}")
            if k < o.n_amg_levels - 1:
                np.testing.assert_array_equal(g.get_vector(4, k), o.amg_level(k)["cf"])
                assert_same_csr(g.get_matrix(4, k), o.amg_level(k)["P"], f"AMG P_{k}")
    finally:
        g.close()


def test_setup_is_deterministic(orc):
    s = small_system((21, 20, 3), seed=9)
    a, b = gpu_solver(s), gpu_solver(s)
    try:
        for k in range(a.levels[1]):
            ma, mb = a.get_matrix(3, k), b.get_matrix(3, k)
            for x, y in zip(ma[:3], mb[:3]):
                np.testing.assert_array_equal(x, y)
    finally:
        a.close()
        b.close()


def _perturbed(s, seed):
    # the same pattern and labels with every value scaled by a factor in [0.85, 1.15]
    f = 1.0 + 0.3 * (np.random.default_rng(seed).random(s.data.shape[0]) - 0.5)
    return s.__class__(**{**s.__dict__, "data": s.data * f})


def test_update_values_is_bitwise_a_new_setup(orc):
    # values-only update (the Newton step with an unchanged active set): every
    # hierarchy object equals the oracle's on the new values, and two updates
    # in a row (new values, then the first ones back) each equal a fresh setup
    s = small_system((13, 11, 9), seed=4, sigma=2.0, frac=0.3, region="ball")
    s2 = _perturbed(s, 11)
    g = gpu_solver(s, frelax_amg_mask=2)
    try:
        g.update_values(s2.data)
        o = orc.Oracle(oracle_csr(orc, s2), s2.labels, frelax_amg_mask=2)
        try:
            check_hierarchy(g, o, frelax_amg_mask=2)
        finally:
            o.close()
        for sys_ in (s2, s):
            if sys_ is s:
                g.update_values(s.data)
            f = gpu_solver(sys_, frelax_amg_mask=2)
            try:
                xa, ia = g.solve(sys_.b, 1e-10)
                xb, ib = f.solve(sys_.b, 1e-10)
                assert ia.status == ib.status == 0 and ia.iterations == ib.iterations
                np.testing.assert_array_equal(xa.cpu().numpy(), xb.cpu().numpy())
            finally:
                f.close()
    finally:
        g.close()


def test_update_values_long_rows():
    # the value-only Galerkin products size their lane groups from the longest
    # left-operand row they read back; on the long-row system (AMG rows of more
    # than 256 entries) the update must still equal a fresh setup bit for bit
    s = long_row_system()
    s2 = _perturbed(s, 13)
    g = gpu_solver(s, frelax_amg_mask=2)
    f = gpu_solver(s2, frelax_amg_mask=2)
    try:
        g.update_values(s2.data)
        xa, ia = g.solve(s2.b, 1e-9)
        xb, ib = f.solve(s2.b, 1e-9)
        assert ia.status == ib.status == 0 and ia.iterations == ib.iterations
        np.testing.assert_array_equal(xa.cpu().numpy(), xb.cpu().numpy())
        for kind, lvl in [(0, 1), (0, 2)] + [(3, k) for k in range(g.levels[1])]:
            for x, y in zip(g.get_matrix(kind, lvl)[:3], f.get_matrix(kind, lvl)[:3]):
                np.testing.assert_array_equal(x, y)
    finally:
        g.close()
        f.close()


@pytest.mark.parametrize("opts", [dict(precision="mixed"), dict(transpose=True), dict(frelax_amg_mask=6)])
def test_update_values_forms(opts):
    s = small_system((17, 15, 5), seed=6, sigma=1.5, frac=0.35, region="ball")
    s2 = _perturbed(s, 12)
    g = gpu_solver(s, **opts)
    f = gpu_solver(s2, **opts)
    try:
        g.update_values(s2.data)
        xa, ia = g.solve(s2.b, 1e-9)
        xb, ib = f.solve(s2.b, 1e-9)
        assert ia.status == ib.status == 0 and ia.iterations == ib.iterations
        np.testing.assert_array_equal(xa.cpu().numpy(), xb.cpu().numpy())
        for k in range(g.levels[1]):
            for x, y in zip(g.get_matrix(3, k)[:3], f.get_matrix(3, k)[:3]):
                np.testing.assert_array_equal(x, y)
    finally:
        g.close()
        f.close()
