"""Pins of the oracle's restarted GMRES, its status codes, the mixed-precision
form and the adjoint (CPU only)."""
import numpy as np
import pytest

from synth import make_config, make_system


def sysA(orc, grid=(6, 5), seed=3, sigma=1.0, frac=0.4):
    s = make_system(grid, sigma, "disk", frac, seed)
    return s, orc.as_csr(s.indptr, s.indices, s.data)


def test_gmres_matches_dense_solve(orc):
    s, A = sysA(orc)
    o = orc.Oracle(A, s.labels)
    r = o.solve(s.b, 1e-13)
    assert r.status == 0
    xd = np.linalg.solve(orc.to_scipy(A).toarray(), s.b)
    np.testing.assert_allclose(r.x, xd, rtol=1e-10, atol=1e-10 * np.abs(xd).max())
    np.testing.assert_allclose(r.x, s.x_true, rtol=1e-9, atol=1e-9)


def test_gmres_residual_history_monotone_across_restarts(orc):
    s, A = sysA(orc, (16, 16), seed=4, sigma=2.0)
    o = orc.Oracle(A, s.labels, restart=5)
    r = o.solve(s.b, 1e-10)
    assert r.status == 0 and r.iterations > 5
    h = r.history
    assert np.all(h[1:] <= h[:-1] * (1 + 1e-6)), h
    # true relative residual recomputed with the oracle's own SpMV
    res = np.linalg.norm(s.b - orc.spmv(A, r.x)) / np.linalg.norm(s.b)
    assert res <= 1e-10 and res == pytest.approx(r.rel_residual, rel=1e-6)


def test_gmres_full_krylov_terminates_within_n(orc):
    s, A = sysA(orc, (3, 3))
    o = orc.Oracle(A, s.labels, restart=s.n, max_iter=s.n, global_relax=0, amg_pre=0, amg_post=0)
    r = o.solve(s.b, 1e-10)
    assert r.status == 0 and r.iterations <= s.n


def test_zero_rhs_and_initial_guess(orc):
    s, A = sysA(orc)
    o = orc.Oracle(A, s.labels)
    r = o.solve(np.zeros(s.n), 1e-8)
    assert r.status == 0 and r.iterations == 0 and not r.x.any()
    o2 = orc.Oracle(A, s.labels, use_x0=1)
    r2 = o2.solve(s.b, 1e-8, x0=s.x_true)
    assert r2.status == 0 and r2.iterations == 0


def test_status_codes(orc):
    s, A = sysA(orc)
    bad = s.labels.copy()
    two = np.where(s.two_phase)[0][0]
    bad[3 * two + 2] = 0  # zero-diagonal constraint row put at level 0
    with pytest.raises(orc.OracleError) as e:
        orc.Oracle(A, bad)
    assert e.value.code == orc.E_ZERO_FDIAG and str(3 * two + 2) in str(e.value)
    with pytest.raises(orc.OracleError) as e:
        orc.Oracle(A, np.full(s.n, -1, np.int32))
    assert e.value.code == orc.E_INVALID
    with pytest.raises(orc.OracleError) as e:
        orc.Oracle(orc.as_csr(A.indptr[:-3], A.indices[:A.indptr[-4]], A.data[:A.indptr[-4]]), s.labels[:-2])
    assert e.value.code == orc.E_INVALID  # n not a multiple of the block size
    unsorted = A.indices.copy()
    unsorted[[0, 1]] = unsorted[[1, 0]]
    with pytest.raises(orc.OracleError) as e:
        orc.Oracle(orc.as_csr(A.indptr, unsorted, A.data), s.labels)
    assert e.value.code == orc.E_INVALID
    sing = A.data.copy()
    c = np.where(~s.two_phase)[0][0]
    for p in range(A.indptr[3 * c], A.indptr[3 * c + 3]):
        if A.indices[p] // 3 == c:
            sing[p] = 0.0
    with pytest.raises(orc.OracleError) as e:
        orc.Oracle(orc.as_csr(A.indptr, A.indices, sing), s.labels)
    assert e.value.code in (orc.E_SINGULAR_BLOCK, orc.E_ZERO_FDIAG)
    o = orc.Oracle(A, s.labels, max_iter=1)
    r = o.solve(s.b, 1e-12)
    assert r.status == orc.NOT_CONVERGED and r.iterations == 1 and np.isfinite(r.x).all()
    o = orc.Oracle(A, s.labels)
    b = s.b.copy()
    b[3] = np.nan
    assert o.solve(b, 1e-8).status == orc.E_BREAKDOWN


def test_mixed_precision_form(orc):
    s = make_config(1)
    A = orc.as_csr(s.indptr, s.indices, s.data)
    r64 = orc.Oracle(A, s.labels).solve(s.b, 1e-8)
    r32 = orc.Oracle(A, s.labels, precision=1).solve(s.b, 1e-8)
    assert r64.status == 0 and r32.status == 0
    assert r32.rel_residual <= 1e-8
    assert abs(r32.iterations - r64.iterations) <= 1


def test_adjoint_dot_product_identity(orc):
    s, A = sysA(orc, (8, 7), seed=9)
    g = np.random.default_rng(2).standard_normal(s.n)
    x = orc.Oracle(A, s.labels).solve(s.b, 1e-13).x
    lam = orc.adjoint(A, s.labels, g, tol=1e-13).x
    assert np.dot(g, x) == pytest.approx(np.dot(lam, s.b), rel=1e-10)


def test_adjoint_hierarchy_is_transpose(orc):
    # non-injective R/P on A^T with the same labels: P' = R^T, R' = P^T, A'_l = A_l^T
    s, A = sysA(orc, (6, 6), seed=1)
    o = orc.Oracle(A, s.labels)
    ot = orc.Oracle(orc.transpose(A), s.labels)
    for l in range(o.n_mgr_levels):
        a, at = o.mgr_level(l), ot.mgr_level(l)
        Al, Alt = orc.to_scipy(a["A"]).toarray(), orc.to_scipy(at["A"]).toarray()
        np.testing.assert_allclose(Alt, Al.T, rtol=1e-14, atol=1e-14 * np.abs(Al).max())
        # equal up to rounding: A_l^T at l >= 1 is itself a rounded product
        np.testing.assert_allclose(orc.to_scipy(at["P"]).toarray(), orc.to_scipy(a["R"]).toarray().T,
                                   rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(orc.to_scipy(at["R"]).toarray(), orc.to_scipy(a["P"]).toarray().T,
                                   rtol=1e-13, atol=1e-15)


def test_adjoint_gradient_against_finite_differences(orc):
    s = make_system((8, 8), 1.5, "disk", 0.35, seed=5, n_obs=6)
    A = orc.as_csr(s.indptr, s.indices, s.data)
    obs = 3 * s.obs_cells  # loss = sum of p over the observation cells
    gvec = np.zeros(s.n)
    gvec[obs] = 1.0

    def loss(vals, b):
        o = orc.Oracle(orc.as_csr(A.indptr, A.indices, vals), s.labels)
        return o.solve(b, 1e-14).x[obs].sum()

    x = orc.Oracle(A, s.labels).solve(s.b, 1e-14).x
    lam = orc.adjoint(A, s.labels, gvec, tol=1e-14).x
    dvals = orc.pattern_outer(A, lam, x)
    rng = np.random.default_rng(0)
    h = 1e-6
    for p in rng.choice(A.indices.shape[0], 8, replace=False):
        vp, vm = A.data.copy(), A.data.copy()
        vp[p] += h
        vm[p] -= h
        fd = (loss(vp, s.b) - loss(vm, s.b)) / (2 * h)
        assert fd == pytest.approx(dvals[p], rel=1e-4, abs=1e-6 * np.abs(dvals).max())
    for i in rng.choice(s.n, 4, replace=False):
        bp, bm = s.b.copy(), s.b.copy()
        bp[i] += h
        bm[i] -= h
        fd = (loss(A.data, bp) - loss(A.data, bm)) / (2 * h)
        assert fd == pytest.approx(lam[i], rel=1e-4, abs=1e-6 * np.abs(lam).max())
