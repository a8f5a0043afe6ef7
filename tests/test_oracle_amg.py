"""Pins of the oracle's AMG pieces: strength, PMIS, classical interpolation,
Galerkin product and the V-cycle, against closed forms and invariants (CPU)."""
import numpy as np
import pytest
import scipy.sparse as sp

from synth import make_poisson


def lap1d(n):
    M = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="csr")
    M.sort_indices()
    return M


def neumann_graph_laplacian(m, seed):
    """2D grid graph Laplacian with random positive anisotropic weights and zero row sums."""
    rng = np.random.default_rng(seed)
    N = m * m
    rows, cols, vals = [], [], []
    for i in range(m):
        for j in range(m):
            c = i + m * j
            for (di, dj, base) in ((1, 0, 1.0), (0, 1, 0.3)):
                if i + di < m and j + dj < m:
                    d = (i + di) + m * (j + dj)
                    w = base * rng.uniform(0.5, 2.0)
                    rows += [c, d]
                    cols += [d, c]
                    vals += [-w, -w]
    W = sp.csr_matrix((vals, (rows, cols)), shape=(N, N))
    A = W - sp.diags(np.asarray(W.sum(axis=1)).ravel())
    A = sp.csr_matrix(A)
    A.sort_indices()
    return A


def test_strength_hand_rows(orc):
    # row 0: positive diagonal; row 1: negative diagonal; row 2: no negative couplings
    D = np.array([[4.0, -1.0, -0.2, 0.5],
                  [1.0, -4.0, 0.2, -0.5],
                  [0.3, 0.1, 2.0, 0.4],
                  [-0.25, -1.0, -0.2, 3.0]])
    A = orc.from_scipy(sp.csr_matrix(D))
    S = orc.strength(A, 0.25)
    rows = [S.indices[S.indptr[i]:S.indptr[i + 1]].tolist() for i in range(4)]
    assert rows == [[1], [0], [], [0, 1]]


def _keys(orc, S, seed):
    ST = orc.transpose(S)
    lam = np.diff(ST.indptr)
    h = np.array([orc.splitmix64(seed ^ i) for i in range(S.shape[0])], dtype=np.uint64)
    return lam, h


def _key_gt(lam, h, i, j):
    return (lam[i], int(h[i]), i) > (lam[j], int(h[j]), j)


@pytest.mark.parametrize("case", ["poisson", "aniso", "random"])
def test_pmis_invariants(orc, case):
    if case == "poisson":
        ip, ix, dv, _ = make_poisson((17, 13))
        A = orc.as_csr(ip, ix, dv)
    elif case == "aniso":
        A = orc.from_scipy(neumann_graph_laplacian(15, 3))
    else:
        rng = np.random.default_rng(4)
        M = sp.random(300, 300, density=0.02, random_state=rng, format="csr")
        M = -(M + M.T) + sp.diags(np.full(300, 10.0))
        M = sp.csr_matrix(M)
        M.sort_indices()
        A = orc.from_scipy(M)
    S = orc.strength(A, 0.25)
    seed = 12345
    cf = orc.pmis(S, seed)
    lam, h = _keys(orc, S, seed)
    n = S.shape[0]
    assert set(np.unique(cf).tolist()) <= {-1, 1}
    Ssets = [set(S.indices[S.indptr[i]:S.indptr[i + 1]].tolist()) for i in range(n)]
    ST = orc.transpose(S)
    STsets = [set(ST.indices[ST.indptr[i]:ST.indptr[i + 1]].tolist()) for i in range(n)]
    for i in range(n):
        if cf[i] == -1:
            # an F point was either never needed (lambda = 0) or depends on a C point
            assert lam[i] == 0 or any(cf[j] == 1 for j in Ssets[i])
        else:
            assert lam[i] > 0
            # a C point i that depends on a C point j was chosen earlier, so its key is larger
            for j in Ssets[i]:
                if cf[j] == 1:
                    assert _key_gt(lam, h, i, j)
        # local key maxima among the points that start undecided are always C
        if lam[i] > 0:
            nb = [j for j in (Ssets[i] | STsets[i]) if lam[j] > 0]
            if all(_key_gt(lam, h, i, j) for j in nb):
                assert cf[i] == 1


def test_pmis_no_strong_connections_all_f(orc):
    A = orc.from_scipy(sp.csr_matrix(sp.diags(np.arange(1.0, 6.0))))
    S = orc.strength(A, 0.25)
    assert S.indices.size == 0
    assert orc.pmis(S, 0).tolist() == [-1] * 5


def test_interp_1d_linear_weights_and_galerkin(orc):
    n = 7
    A = orc.from_scipy(lap1d(n))
    S = orc.strength(A, 0.25)
    cf = np.array([-1, 1, -1, 1, -1, 1, -1], dtype=np.int32)
    P = orc.interp(A, S, cf)
    D = orc.to_scipy(P).toarray()
    expect = np.zeros((7, 3))
    for c, i in enumerate([1, 3, 5]):
        expect[i, c] = 1.0
        expect[i - 1, c] += 0.5
        expect[i + 1, c] += 0.5
    np.testing.assert_array_equal(D, expect)
    Ac = orc.spgemm(orc.transpose(P), orc.spgemm(A, P))
    np.testing.assert_array_equal(orc.to_scipy(Ac).toarray(), 0.5 * lap1d(3).toarray())


def test_interp_distance_two_terms(orc):
    # triangle 0(C)-1(F)-2(F), zero row sums: row 1 gets its F neighbour 2
    # distributed through a_20 -> weight exactly 1.
    D = np.array([[2.0, -1.0, -1.0], [-1.0, 2.0, -1.0], [-1.0, -1.0, 2.0]])
    A = orc.from_scipy(sp.csr_matrix(D))
    S = orc.strength(A, 0.25)
    P = orc.interp(A, S, np.array([1, -1, -1], dtype=np.int32))
    np.testing.assert_array_equal(orc.to_scipy(P).toarray(), np.ones((3, 1)))
    # chain C-F-F-C: the F neighbour shares no C point, so a_12 is lumped into the diagonal
    A = orc.from_scipy(lap1d(4))
    S = orc.strength(A, 0.25)
    P = orc.interp(A, S, np.array([1, -1, -1, 1], dtype=np.int32))
    np.testing.assert_array_equal(orc.to_scipy(P).toarray(), np.array([[1, 0], [1, 0], [0, 1], [0, 1.0]]))


@pytest.mark.parametrize("seed", [0, 1])
def test_interp_preserves_constants_on_zero_row_sums(orc, seed):
    M = neumann_graph_laplacian(14, seed)
    A = orc.from_scipy(M)
    S = orc.strength(A, 0.25)
    cf = orc.pmis(S, 7)
    P = orc.interp(A, S, cf)
    Ps = orc.to_scipy(P)
    rows = np.diff(Ps.indptr)
    ones = Ps @ np.ones(Ps.shape[1])
    ok = rows > 0
    assert ok.mean() > 0.9
    np.testing.assert_allclose(ones[ok], 1.0, rtol=1e-13)
    # Galerkin operator of a zero-row-sum symmetric matrix: symmetric, zero row sums
    Ac = orc.to_scipy(orc.spgemm(orc.transpose(P), orc.spgemm(A, P))).toarray()
    if ok.all():
        np.testing.assert_allclose(Ac.sum(axis=1), 0.0, atol=1e-12 * np.abs(Ac).max())
    np.testing.assert_allclose(Ac, Ac.T, rtol=1e-13, atol=1e-13 * np.abs(Ac).max())


def _amg_propagator(o, A_dense_fn):
    """I - M^{-1} A of the AMG V(pre, post) cycle built from the oracle's
    hierarchy as dense matrices: S^post (I - P M_c^{-1} P^T A) S^pre with
    S = I - D_l1^{-1} A and M_c^{-1} the next level (exact LU at the bottom)."""
    nl = o.n_amg_levels

    def minv(k):
        lv = o.amg_level(k)
        A = A_dense_fn(lv["A"])
        n = A.shape[0]
        if k == nl - 1:
            return np.linalg.inv(A)
        P = A_dense_fn(lv["P"])
        Sm = np.eye(n) - np.diag(1.0 / lv["l1"]) @ A
        Mc = minv(k + 1)
        E = np.linalg.matrix_power(Sm, 2) @ (np.eye(n) - P @ Mc @ P.T @ A) @ np.linalg.matrix_power(Sm, 2)
        return (np.eye(n) - E) @ np.linalg.inv(A)

    return minv(0)


def test_amg_vcycle_equals_closed_form_propagator(orc):
    ip, ix, dv, _ = make_poisson((13, 11))
    A = orc.as_csr(ip, ix, dv)
    n = A.shape[0]
    o = orc.Oracle(A, np.zeros(n, np.int32), block_size=1, amg_coarse_max=10)
    assert o.n_amg_levels >= 3
    dense = lambda M: orc.to_scipy(M).toarray()
    Minv = _amg_propagator(o, dense)
    cols = np.stack([o.vcycle(e) for e in np.eye(n)], axis=1)
    np.testing.assert_allclose(cols, Minv, rtol=1e-10, atol=1e-12 * np.abs(Minv).max())


def test_amg_vcycle_contracts_on_poisson(orc):
    ip, ix, dv, _ = make_poisson((64, 64))
    A = orc.as_csr(ip, ix, dv)
    n = A.shape[0]
    o = orc.Oracle(A, np.zeros(n, np.int32), block_size=1)
    As = orc.to_scipy(A)
    e0 = np.random.default_rng(0).standard_normal(n)
    e = e0.copy()
    for _ in range(15):
        e = e - o.vcycle(As @ e)
    rate = (np.linalg.norm(e) / np.linalg.norm(e0)) ** (1 / 15)
    assert rate < 0.8


def test_amg_gmres_iterations_grow_slowly_with_mesh(orc):
    its = []
    for m in (32, 64, 128, 256, 512):
        ip, ix, dv, b = make_poisson((m, m))
        A = orc.as_csr(ip, ix, dv)
        o = orc.Oracle(A, np.zeros(m * m, np.int32), block_size=1)
        r = o.solve(b, 1e-8)
        assert r.status == 0
        its.append(r.iterations)
    # PMIS with distance-one classical interpolation is not mesh independent
    # (De Sterck, Yang, Heys 2006); growth stays logarithmic in the mesh size:
    # four to five more iterations per halving of the mesh width.  The counts are
    # deterministic and recorded exactly.
    assert its == sorted(its)
    assert max(np.diff(its)) <= 6 and its[-1] <= 32, its
    assert its == [15, 19, 23, 27, 32], its


def _pmis_brute_force(S, lam, h):
    """PMIS written out from its definition with Python sets (tiny graphs only):
    points with lambda = 0 start as F; every round, on the states at its start,
    each undecided point whose key (lambda, hash, index) exceeds the keys of all
    undecided points it is strongly connected to (either direction) becomes C,
    then each undecided point that strongly depends on a C point becomes F."""
    n = S.shape[0]
    dep = [set(S.indices[S.indptr[i]:S.indptr[i + 1]].tolist()) for i in range(n)]
    nbr = [set(d) for d in dep]
    for i in range(n):
        for j in dep[i]:
            nbr[j].add(i)
    key = [(int(lam[i]), int(h[i]), i) for i in range(n)]
    state = [0 if lam[i] > 0 else -1 for i in range(n)]
    while 0 in state:
        und = [i for i in range(n) if state[i] == 0]
        new_c = [i for i in und if all(state[j] != 0 or key[i] > key[j] for j in nbr[i])]
        assert new_c, "a round must select at least the largest undecided key"
        for i in new_c:
            state[i] = 1
        for i in und:
            if state[i] == 0 and any(state[j] == 1 for j in dep[i]):
                state[i] = -1
    return np.array(state)


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4, 5])
def test_pmis_equals_brute_force(orc, seed):
    # random strength graphs of up to 200 points, some directed, some symmetric,
    # with isolated points and points nobody depends on
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(20, 200))
    M = sp.random(n, n, density=float(rng.uniform(0.01, 0.08)), random_state=rng, format="csr")
    if seed % 2:
        M = M + M.T
    M = -abs(M) + sp.diags(np.full(n, 50.0))
    M = sp.csr_matrix(M)
    M.sort_indices()
    A = orc.from_scipy(M)
    S = orc.strength(A, 0.25)
    pmis_seed = int(rng.integers(0, 2**63))
    cf = orc.pmis(S, pmis_seed)
    lam, h = _keys(orc, S, pmis_seed)
    np.testing.assert_array_equal(cf, _pmis_brute_force(S, lam, h))


def _interp_rows(orc, D, strong, cf):
    """Classical interpolation of a small dense matrix with a given strength
    pattern and C/F split; returns P as a dense array."""
    A = orc.from_scipy(sp.csr_matrix(D))
    n = D.shape[0]
    S = orc.as_csr(np.concatenate([[0], np.cumsum([len(s) for s in strong])]),
                   np.array([j for s in strong for j in s], dtype=np.int32), None, (n, n))
    P = orc.interp(A, S, np.asarray(cf, dtype=np.int32))
    return orc.to_scipy(P).toarray()


def test_interp_sign_filter_positive_diagonal_neighbour(orc):
    # F point 0 with strong C neighbours 1, 2, strong F neighbour 3 and a weak
    # coupling to 4.  Row 3 has a_33 = 4 > 0: its coupling a_31 = -1 has the
    # opposite sign (kept in the distance-two sum), a_32 = +1 the same sign
    # (dropped).  Hand computation:
    #   atil = a_00 + a_04 = 4 - 0.2 = 3.8
    #   den  = abar_31 + abar_32 = -1 + 0 = -1
    #   num_1 = a_03 abar_31 / den = (-1)(-1)/(-1) = -1,  num_2 = 0
    #   w_01 = -(a_01 + num_1) / atil = 2 / 3.8,  w_02 = -(a_02) / atil = 1 / 3.8
    # (without the filter den = 0 and a_03 would be lumped into atil: 0.5 / 0.5)
    D = np.array([[4.0, -1.0, -1.0, -1.0, -0.2],
                  [-1.0, 4.0, 0.0, -1.0, 0.0],
                  [-1.0, 0.0, 4.0, 1.0, 0.0],
                  [-1.0, -1.0, 1.0, 4.0, 0.0],
                  [-0.2, 0.0, 0.0, 0.0, 4.0]])
    strong = [[1, 2, 3], [0, 3], [0], [0, 1], []]
    P = _interp_rows(orc, D, strong, [-1, 1, 1, -1, 1])
    assert P[0, 0] == 2.0 / 3.8 and P[0, 1] == 1.0 / 3.8 and P[0, 2] == 0.0
    # C rows are unit rows onto their coarse index
    np.testing.assert_array_equal(P[[1, 2, 4]], np.eye(3))


def test_interp_sign_filter_negative_diagonal_neighbour(orc):
    # as above, but row 3 has a negative diagonal a_33 = -4: now a_31 = +1 has
    # the opposite sign (kept) and a_32 = -1 the same sign (dropped).
    #   atil = 4, den = 1, num_1 = a_03 * 1 / 1 = -2, num_2 = 0
    #   w_01 = -(-1 - 2) / 4 = 3/4,  w_02 = -(-1) / 4 = 1/4
    # A filter on the sign of a_km alone (a_km < 0) would keep a_32 instead and
    # give 1/4, 3/4; no filter gives den = 0 and 1/2, 1/2.
    D = np.array([[4.0, -1.0, -1.0, -2.0],
                  [-1.0, 4.0, 0.0, 1.0],
                  [-1.0, 0.0, 4.0, -1.0],
                  [1.0, 1.0, -1.0, -4.0]])
    strong = [[1, 2, 3], [0], [0], [1]]
    P = _interp_rows(orc, D, strong, [-1, 1, 1, -1])
    assert P[0, 0] == 0.75 and P[0, 1] == 0.25


def test_interp_sign_filter_all_same_sign_lumps_the_f_neighbour(orc):
    # every coupling of the strong F neighbour 3 to C_0 = {1, 2} has the sign of
    # its diagonal (a_33 = 4, a_31 = 1, a_32 = 2): den = 0, so a_03 = -2 joins the
    # diagonal: atil = 4 - 2 = 2, w_01 = -(-1) / 2 = 1/2, w_02 = -(-0.5) / 2 = 1/4.
    D = np.array([[4.0, -1.0, -0.5, -2.0],
                  [-1.0, 4.0, 0.0, 0.0],
                  [-0.5, 0.0, 4.0, 0.0],
                  [-2.0, 1.0, 2.0, 4.0]])
    strong = [[1, 2, 3], [0], [0], [0]]
    P = _interp_rows(orc, D, strong, [-1, 1, 1, -1])
    assert P[0, 0] == 0.5 and P[0, 1] == 0.25


def test_interp_sign_filter_zero_coupling_is_not_kept(orc):
    # a stored zero a_31 = 0 has no sign opposite to a_33: it is dropped like a
    # same-sign entry.  With a_32 = -2 kept: den = -2, num_2 = (-1)(-2)/(-2) = -1,
    # atil = 4, w_01 = -(-1)/4 = 1/4, w_02 = -(-1 - 1)/4 = 1/2.
    D = np.array([[4.0, -1.0, -1.0, -1.0],
                  [-1.0, 4.0, 0.0, 0.0],
                  [-1.0, 0.0, 4.0, 0.0],
                  [-1.0, 0.0, -2.0, 4.0]])
    M = sp.csr_matrix(D)
    # store a_31 = 0 explicitly
    indptr = np.array([0, 4, 6, 8, 12])
    indices = np.array([0, 1, 2, 3, 0, 1, 0, 2, 0, 1, 2, 3], np.int32)
    data = np.array([M[i, j] for i in range(4) for j in indices[indptr[i]:indptr[i + 1]]])
    Ao = orc.as_csr(indptr, indices, data)
    assert Ao.indices[Ao.indptr[3]:Ao.indptr[4]].tolist() == [0, 1, 2, 3]
    S = orc.as_csr([0, 3, 4, 5, 6], np.array([1, 2, 3, 0, 0, 0], np.int32), None, (4, 4))
    P = orc.to_scipy(orc.interp(Ao, S, np.array([-1, 1, 1, -1], np.int32))).toarray()
    assert P[0, 0] == 0.25 and P[0, 1] == 0.5


def test_l1_smoother_diagonal_is_the_absolute_row_sum(orc):
    # mixed-sign rows: the l1 diagonal is sum_j |a_ij| (hand sums below), not
    # |a_ii| and not the signed row sum
    D = np.array([[4.0, -1.0, 0.5, 0.0, 0.0, 0.0],
                  [-1.0, 5.0, -2.0, 0.25, 0.0, 0.0],
                  [0.5, -2.0, -6.0, 1.0, 0.0, 0.0],
                  [0.0, 0.25, 1.0, 3.0, -1.5, 0.0],
                  [0.0, 0.0, 0.0, -1.5, 4.0, -1.0],
                  [0.0, 0.0, 0.0, 0.0, -1.0, 2.0]])
    expect = np.array([5.5, 8.25, 9.5, 5.75, 6.5, 3.0])
    A = orc.from_scipy(sp.csr_matrix(D))
    o = orc.Oracle(A, np.zeros(6, np.int32), block_size=1, amg_coarse_max=2)
    assert o.n_amg_levels >= 2
    np.testing.assert_array_equal(o.amg_level(0)["l1"], expect)
