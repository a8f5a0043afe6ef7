"""Pins of the oracle's MGR hierarchy and V-cycle against the paper's identities
(Section 4: ideal interpolation/restriction, eqs. MGR-add/MGR-mul1, RAQ = Q^T A P = 0,
the pre-smoothing propagator eq. MGR-pre) and the closed forms of the three
reductions of Section 5 on the generator's Jacobian (CPU only)."""
import numpy as np
import pytest
import scipy.sparse as sp

from synth import make_system


def dense(orc, M):
    return orc.to_scipy(M).toarray()


def small(grid=(4, 4), seed=11, frac=0.4):
    return make_system(grid, 1.0, "disk", frac, seed)


def test_level0_coarse_operator_is_acc_bitwise(orc):
    # Section 5: the first reduction is exact because C_33 is diagonal.  In the
    # generator the single-phase constraint rows are [0, 0, 1], so A_FC = 0,
    # W_p = 0 and R A P reduces to A_CC exactly.
    s = small((6, 5))
    A = orc.as_csr(s.indptr, s.indices, s.data)
    o = orc.Oracle(A, s.labels)
    lv0, lv1 = o.mgr_level(0), o.mgr_level(1)
    C = lv0["clist"]
    Acc = orc.to_scipy(A)[C][:, C]
    Acc.sort_indices()
    A1 = lv1["A"]
    np.testing.assert_array_equal(A1.indptr, Acc.indptr)
    np.testing.assert_array_equal(A1.indices, Acc.indices)
    np.testing.assert_array_equal(A1.data, Acc.data)
    # F/C lists follow the labels
    np.testing.assert_array_equal(lv0["flist"], np.where(s.labels == 0)[0])
    np.testing.assert_array_equal(C, np.where(s.labels > 0)[0])


def test_level1_and_level2_closed_forms(orc):
    s = make_system((7, 6), 1.5, "disk", 0.45, seed=5)
    A = orc.as_csr(s.indptr, s.indices, s.data)
    D = dense(orc, A)
    for rp_type in (0, 1):
        o = orc.Oracle(A, s.labels, rp_type=rp_type)
        l1, l2 = o.mgr_level(1), o.mgr_level(2)
        glob1 = np.where(s.labels >= 1)[0]
        glob2 = np.where(s.labels >= 2)[0]
        A1 = dense(orc, l1["A"])
        A2 = dense(orc, l2["A"])
        # p rows of A_2 are the p rows of A_1 restricted to C columns (the p row
        # has no rho coupling, so its row of W_r is empty and W_p does not reach it)
        loc1 = {g: i for i, g in enumerate(glob1)}
        keep = [loc1[g] for g in glob2]
        for i2, g in enumerate(glob2):
            if g % 3 == 0:
                np.testing.assert_array_equal(A2[i2], A1[loc1[g], keep])
        # two-phase S diagonal of A_2 = a_{rho S} / a_{rho rho} of the same cell
        for i2, g in enumerate(glob2):
            if g % 3 == 2:
                c = g // 3
                expect = D[3 * c + 1, 3 * c + 2] / D[3 * c + 1, 3 * c + 1]
                assert A2[i2, i2] == pytest.approx(expect, rel=1e-14)


def test_each_level_is_r_a_p(orc):
    s = small((5, 5))
    A = orc.as_csr(s.indptr, s.indices, s.data)
    o = orc.Oracle(A, s.labels)
    for l in range(o.n_mgr_levels):
        lv = o.mgr_level(l)
        An = o.mgr_level(l + 1)["A"] if l + 1 < o.n_mgr_levels else o.amg_level(0)["A"]
        RAP = dense(orc, lv["R"]) @ dense(orc, lv["A"]) @ dense(orc, lv["P"])
        np.testing.assert_allclose(dense(orc, An), RAP, rtol=1e-13, atol=1e-13 * np.abs(RAP).max())
        # P = [W_p; I], R = [W_r, I] on the C points
        P, R = dense(orc, lv["P"]), dense(orc, lv["R"])
        C = lv["clist"]
        np.testing.assert_array_equal(P[C], np.eye(len(C)))
        np.testing.assert_array_equal(R[:, C], np.eye(len(C)))


@pytest.mark.parametrize("transpose", [False, True])
def test_two_level_ideal_operators_are_exact(orc, transpose):
    # With A_FF diagonal, D_FF^{-1} = A_FF^{-1}: P and R are the ideal operators of
    # Section 4, so R A Q = Q^T A P = 0, R A P is the Schur complement, and with an
    # exact coarse solve the two-level method is exact (eq. MGR-mul1): GMRES
    # converges in a single iteration.
    s = small((4, 4))
    A = orc.as_csr(s.indptr, s.indices, s.data)
    if transpose:
        A = orc.transpose(A)
    labels = np.where(s.labels == 0, 0, 1).astype(np.int32)
    o = orc.Oracle(A, labels)
    assert o.n_amg_levels == 1  # coarse grid (<= 64 unknowns) is solved by dense LU
    lv = o.mgr_level(0)
    Ad = dense(orc, A)
    F, C = lv["flist"], lv["clist"]
    Q = np.zeros((Ad.shape[0], len(F)))
    Q[F, np.arange(len(F))] = 1
    P, R = dense(orc, lv["P"]), dense(orc, lv["R"])
    scale = np.abs(Ad).max()
    np.testing.assert_allclose(R @ Ad @ Q, 0, atol=1e-14 * scale)
    np.testing.assert_allclose(Q.T @ Ad @ P, 0, atol=1e-14 * scale)
    Sch = Ad[np.ix_(C, C)] - Ad[np.ix_(C, F)] @ np.linalg.inv(Ad[np.ix_(F, F)]) @ Ad[np.ix_(F, C)]
    np.testing.assert_allclose(dense(orc, o.amg_level(0)["A"]), Sch, rtol=1e-13, atol=1e-13 * scale)
    b = np.random.default_rng(1).standard_normal(Ad.shape[0])
    r = o.solve(b, 1e-10)
    assert r.status == 0 and r.iterations == 1


def _mgr_minv(orc, o, bs_inv, post=False):
    """M^{-1} of the recursive MGR V-cycle from the paper's propagator
    I - M_l^{-1} A_l = (I - P_l M_{l+1}^{-1} R_l A_l)(I - Q_l D_l^{-1} Q_l^T A_l)(I - B^{-1} A_0 at l = 0)
    (eq. MGR-pre), or with post=True eq. MGR-post, the same smoother factor
    I - M_f^{-1} A after the coarse-grid correction:
    (I - Q_l D_l^{-1} Q_l^T A_l)(I - B^{-1} A_0 at l = 0)(I - P_l M_{l+1}^{-1} R_l A_l),
    with AMG V(2,2) (or dense LU) below the last level."""
    L = o.n_mgr_levels
    nl = o.n_amg_levels

    def amg_minv(k):
        lv = o.amg_level(k)
        Ak = dense(orc, lv["A"])
        n = Ak.shape[0]
        if k == nl - 1:
            return np.linalg.inv(Ak)
        P = dense(orc, lv["P"])
        Sm = np.eye(n) - np.diag(1.0 / lv["l1"]) @ Ak
        E = Sm @ Sm @ (np.eye(n) - P @ amg_minv(k + 1) @ P.T @ Ak) @ Sm @ Sm
        return (np.eye(n) - E) @ np.linalg.inv(Ak)

    def mgr_minv(l):
        if l == L:
            return amg_minv(0)
        lv = o.mgr_level(l)
        Al = dense(orc, lv["A"])
        n = Al.shape[0]
        F = lv["flist"]
        Q = np.zeros((n, len(F)))
        Q[F, np.arange(len(F))] = 1
        Ec = np.eye(n) - dense(orc, lv["P"]) @ mgr_minv(l + 1) @ dense(orc, lv["R"]) @ Al
        Ef = np.eye(n) - Q @ np.diag(lv["dinv"]) @ Q.T @ Al
        Eg = np.eye(n) - bs_inv @ Al if l == 0 else np.eye(n)
        # I - M_f^{-1} A = Ef Eg in both forms (global relaxation first, then F-relaxation)
        E = Ef @ Eg @ Ec if post else Ec @ Ef @ Eg
        return (np.eye(n) - E) @ np.linalg.inv(Al)

    return mgr_minv(0)


def _rho_first_labels(s):
    """Labels that eliminate rho first (level 0), then S in every cell (level 1),
    with p as the coarse grid.  The level-0 F rows then couple to other cells, so
    the F-relaxation and the global relaxation do not commute (with the default
    labels they do: the single-phase S rows hold only their own diagonal)."""
    lab = np.empty(s.n, np.int32)
    lab[0::3], lab[1::3], lab[2::3] = 2, 0, 1
    return lab


@pytest.mark.parametrize("grid,post,labels", [((4, 4), False, "default"), ((9, 9), False, "default"),
                                              ((4, 4), True, "default"), ((9, 9), True, "default"),
                                              ((5, 4), False, "rho_first"), ((5, 4), True, "rho_first")])
def test_vcycle_equals_closed_form_propagator(orc, grid, post, labels):
    s = make_system(grid, 1.0, "disk", 0.4, seed=2)
    A = orc.as_csr(s.indptr, s.indices, s.data)
    lab = s.labels if labels == "default" else _rho_first_labels(s)
    o = orc.Oracle(A, lab, cycle_post=int(post))
    binv = o.block_inverses().reshape(-1, 3, 3)
    B = np.zeros((s.n, s.n))
    for c in range(s.n_cells):
        B[3 * c:3 * c + 3, 3 * c:3 * c + 3] = binv[c]
    Minv = _mgr_minv(orc, o, B, post=post)
    cols = np.stack([o.vcycle(e) for e in np.eye(s.n)], axis=1)
    np.testing.assert_allclose(cols, Minv, rtol=1e-9, atol=1e-11 * np.abs(Minv).max())


def _amg_operator(levels, pre, post):
    """Dense M^{-1} of an AMG V(pre, post) cycle (l1-Jacobi, exact LU at the bottom)
    given per-level dicts of dense A, P and l1."""
    def minv(k):
        A = levels[k]["A"]
        n = A.shape[0]
        if k == len(levels) - 1:
            return np.linalg.inv(A)
        P = levels[k]["P"]
        Sm = np.eye(n) - np.diag(1.0 / levels[k]["l1"]) @ A
        E = np.linalg.matrix_power(Sm, post) @ (np.eye(n) - P @ minv(k + 1) @ P.T @ A) @ \
            np.linalg.matrix_power(Sm, pre)
        return (np.eye(n) - E) @ np.linalg.inv(A)
    return minv(0)


def test_vcycle_with_amg_frelaxation_equals_closed_form(orc):
    # level 1 relaxes its F-points with one AMG V(1,1)-cycle on A_FF (the paper's
    # F-relaxation for its phase-transition runs): M_f = I - Q M_FF^{-1} Q^T A
    s = make_system((9, 9), 1.5, "disk", 0.4, seed=2)
    A = orc.as_csr(s.indptr, s.indices, s.data)
    o = orc.Oracle(A, s.labels, frelax_amg_mask=2, amg_coarse_max=20)
    assert o.n_ff_levels(1) >= 2 and o.n_ff_levels(0) == 0
    lv1 = o.mgr_level(1)
    F = lv1["flist"]
    Aff = dense(orc, lv1["A"])[np.ix_(F, F)]
    ffl = [o.ff_level(1, k) for k in range(o.n_ff_levels(1))]
    np.testing.assert_array_equal(dense(orc, ffl[0]["A"]), Aff)
    levels = [dict(A=dense(orc, d["A"]), P=dense(orc, d["P"]) if "P" in d else None, l1=d.get("l1")) for d in ffl]
    Mff = _amg_operator(levels, 1, 1)
    # replace D_FF^{-1} of level 1 by M_FF^{-1} in the recursive propagator
    L, nl = o.n_mgr_levels, o.n_amg_levels

    def amg_minv(k):
        lv = o.amg_level(k)
        Ak = dense(orc, lv["A"])
        n = Ak.shape[0]
        if k == nl - 1:
            return np.linalg.inv(Ak)
        P = dense(orc, lv["P"])
        Sm = np.eye(n) - np.diag(1.0 / lv["l1"]) @ Ak
        E = Sm @ Sm @ (np.eye(n) - P @ amg_minv(k + 1) @ P.T @ Ak) @ Sm @ Sm
        return (np.eye(n) - E) @ np.linalg.inv(Ak)

    binv = o.block_inverses().reshape(-1, 3, 3)
    B = np.zeros((s.n, s.n))
    for c in range(s.n_cells):
        B[3 * c:3 * c + 3, 3 * c:3 * c + 3] = binv[c]

    def mgr_minv(l):
        if l == L:
            return amg_minv(0)
        lv = o.mgr_level(l)
        Al = dense(orc, lv["A"])
        n = Al.shape[0]
        Fl = lv["flist"]
        Q = np.zeros((n, len(Fl)))
        Q[Fl, np.arange(len(Fl))] = 1
        Mf = Mff if l == 1 else np.diag(lv["dinv"])
        E = (np.eye(n) - dense(orc, lv["P"]) @ mgr_minv(l + 1) @ dense(orc, lv["R"]) @ Al) @ \
            (np.eye(n) - Q @ Mf @ Q.T @ Al)
        if l == 0:
            E = E @ (np.eye(n) - B @ Al)
        return (np.eye(n) - E) @ np.linalg.inv(Al)

    Minv = mgr_minv(0)
    cols = np.stack([o.vcycle(e) for e in np.eye(s.n)], axis=1)
    np.testing.assert_allclose(cols, Minv, rtol=1e-9, atol=1e-11 * np.abs(Minv).max())


def test_amg_frelaxation_restores_convergence(orc):
    # sigma = 2 in 3D: one Jacobi sweep on the diffusion-dominated rho block is weak;
    # one AMG V(1,1)-cycle on it brings the iteration count down
    s = make_system((24, 24, 24), 2.0, "ball", 0.3, seed=4)
    A = orc.as_csr(s.indptr, s.indices, s.data)
    rj = orc.Oracle(A, s.labels).solve(s.b, 1e-8)
    ra = orc.Oracle(A, s.labels, frelax_amg_mask=2).solve(s.b, 1e-8)
    assert ra.status == 0 and rj.status == 0
    assert ra.iterations < 0.7 * rj.iterations, (ra.iterations, rj.iterations)


def test_fp32_vcycle_close_to_fp64(orc):
    s = small((8, 8))
    A = orc.as_csr(s.indptr, s.indices, s.data)
    o64 = orc.Oracle(A, s.labels)
    o32 = orc.Oracle(A, s.labels, precision=1)
    r = np.random.default_rng(0).standard_normal(s.n)
    e64, e32 = o64.vcycle(r), o32.vcycle(r)
    assert np.linalg.norm(e32 - e64) / np.linalg.norm(e64) < 1e-4
    assert not np.array_equal(e32, e64)


def test_introspection_of_coarse_and_fblock_hierarchies(orc):
    s = make_system((9, 9), 1.5, "disk", 0.4, seed=2)
    A = orc.as_csr(s.indptr, s.indices, s.data)
    o = orc.Oracle(A, s.labels, frelax_amg_mask=2, amg_coarse_max=20)
    lu, perm = o.coarse_lu()
    Ac = dense(orc, o.amg_level(o.n_amg_levels - 1)["A"])
    L = np.tril(lu, -1) + np.eye(lu.shape[0])
    np.testing.assert_allclose(L @ np.triu(lu), Ac[perm], rtol=1e-12, atol=1e-12 * np.abs(Ac).max())
    flu, fperm = o.ff_coarse_lu(1)
    Af = dense(orc, o.ff_level(1, o.n_ff_levels(1) - 1)["A"])
    L = np.tril(flu, -1) + np.eye(flu.shape[0])
    np.testing.assert_allclose(L @ np.triu(flu), Af[fperm], rtol=1e-12, atol=1e-12 * np.abs(Af).max())
    with pytest.raises(IndexError):
        o.ff_level(0, 0)


def test_level2_fblock_has_no_strong_connections(orc):
    # Section 6.2 relaxes the F-points of every reduction after the first with one
    # AMG V(1,1)-cycle on A_FF.  At the last reduction (S in two-phase cells) of
    # this Jacobian, A_FF has a negative diagonal and only negative off-diagonal
    # entries, so no coupling is strong in the classical (sign-aware) sense: PMIS
    # makes every point F and the F-block "hierarchy" is its coarsest level alone,
    # a direct solve of A_FF.  Below the dense limit that is what the AMG option
    # does (and it takes more GMRES iterations than one Jacobi sweep); above it
    # the setup stops because the coarsening stalls.
    s = make_system((20, 20, 20), 2.0, "ball", 0.3, seed=4)
    A = orc.as_csr(s.indptr, s.indices, s.data)
    o = orc.Oracle(A, s.labels, frelax_amg_mask=2)
    d = o.mgr_level(2)
    M = orc.to_scipy(d["A"]).tocsr()
    F = d["flist"]
    Aff = M[F][:, F].tocsr()
    Aff.sort_indices()
    dg = Aff.diagonal()
    off = Aff - sp.diags(dg)
    off.eliminate_zeros()
    assert np.all(dg < 0) and off.nnz > 0 and np.all(off.data < 0)
    S = orc.strength(orc.from_scipy(Aff))
    assert S.indices.shape[0] == 0
    jac = o.solve(s.b, 1e-8)
    o.close()
    o6 = orc.Oracle(A, s.labels, frelax_amg_mask=6)
    assert o6.n_ff_levels(2) == 1
    amg = o6.solve(s.b, 1e-8)
    o6.close()
    assert jac.status == 0 and amg.status == 0 and amg.iterations > jac.iterations, (jac.iterations, amg.iterations)
    big = make_system((40, 40, 40), 2.0, "ball", 0.3, seed=4)
    with pytest.raises(orc.OracleError, match="stalled"):
        orc.Oracle(orc.as_csr(big.indptr, big.indices, big.data), big.labels, frelax_amg_mask=6)
