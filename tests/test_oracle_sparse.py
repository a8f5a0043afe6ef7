"""Pins of the oracle's sparse building blocks against dense linear algebra and
closed forms (CPU only)."""
import os

import numpy as np
import pytest
import scipy.sparse as sp

from synth import make_system

HERE = os.path.dirname(os.path.abspath(__file__))


def rand_csr(orc, m, n, density, seed, allow_empty_rows=True):
    rng = np.random.default_rng(seed)
    M = sp.random(m, n, density=density, random_state=rng, format="csr")
    M.data = rng.standard_normal(M.nnz)
    M.sort_indices()
    return orc.from_scipy(M)


def test_spmv_matches_dense(orc):
    s = make_system((4, 3), 1.0, "disk", 0.4, seed=7)
    A = orc.as_csr(s.indptr, s.indices, s.data)
    D = orc.to_scipy(A).toarray()
    x = np.random.default_rng(0).standard_normal(s.n)
    np.testing.assert_allclose(orc.spmv(A, x), D @ x, rtol=1e-14, atol=1e-13)
    # the generator's b was made from x_true
    np.testing.assert_allclose(orc.spmv(A, s.x_true), s.b, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_transpose_is_stable_and_exact(orc, seed):
    A = rand_csr(orc, 37, 23, 0.15, seed)
    AT = orc.transpose(A)
    np.testing.assert_array_equal(orc.to_scipy(AT).toarray(), orc.to_scipy(A).toarray().T)
    for j in range(AT.shape[0]):
        row = AT.indices[AT.indptr[j]:AT.indptr[j + 1]]
        assert np.all(np.diff(row) > 0), "transpose rows must list source rows in ascending order"
    ATT = orc.transpose(AT)
    np.testing.assert_array_equal(ATT.indptr, A.indptr)
    np.testing.assert_array_equal(ATT.indices, A.indices)
    np.testing.assert_array_equal(ATT.data, A.data)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_spgemm_matches_dense_product(orc, seed):
    A = rand_csr(orc, 29, 31, 0.2, seed)
    B = rand_csr(orc, 31, 17, 0.2, seed + 100)
    Cm = orc.spgemm(A, B)
    Da, Db = orc.to_scipy(A).toarray(), orc.to_scipy(B).toarray()
    np.testing.assert_allclose(orc.to_scipy(Cm).toarray(), Da @ Db, rtol=1e-13, atol=1e-13)
    # the pattern is the symbolic product: (i,j) present iff some k has A_ik, B_kj stored
    sym = (np.abs(Da) > 0).astype(int) @ (np.abs(Db) > 0).astype(int) > 0
    pat = np.zeros_like(sym)
    for i in range(Cm.shape[0]):
        pat[i, Cm.indices[Cm.indptr[i]:Cm.indptr[i + 1]]] = True
    np.testing.assert_array_equal(pat, sym)
    for i in range(Cm.shape[0]):
        assert np.all(np.diff(Cm.indices[Cm.indptr[i]:Cm.indptr[i + 1]]) > 0)


def test_spgemm_keeps_exact_cancellation(orc):
    A = orc.as_csr([0, 2], [0, 1], [1.0, 1.0], (1, 2))
    B = orc.as_csr([0, 1, 2], [0, 0], [1.0, -1.0], (2, 1))
    Cm = orc.spgemm(A, B)
    assert Cm.indices.tolist() == [0] and Cm.data.tolist() == [0.0]


def test_spgemm_ascending_order_summation(orc):
    # (1e16 + 1) - 1e16 in ascending k is 0 in double; any other order gives 1 or 2
    A = orc.as_csr([0, 3], [0, 1, 2], [1.0, 1.0, 1.0], (1, 3))
    B = orc.as_csr([0, 1, 2, 3], [0, 0, 0], [1e16, 1.0, -1e16], (3, 1))
    Cm = orc.spgemm(A, B)
    assert Cm.data[0] == ((1e16 + 1.0) + -1e16)


def test_block_inverse(orc):
    s = make_system((5, 4), 1.5, "disk", 0.4, seed=3)
    A = orc.as_csr(s.indptr, s.indices, s.data)
    binv = orc.block_inverse(A, 3).reshape(-1, 3, 3)
    D = orc.to_scipy(A).toarray()
    for c in range(s.n_cells):
        B = D[3 * c:3 * c + 3, 3 * c:3 * c + 3]
        np.testing.assert_allclose(B @ binv[c], np.eye(3), atol=1e-13)
        np.testing.assert_allclose(binv[c], np.linalg.inv(B), rtol=1e-12, atol=1e-14)


def test_block_inverse_closed_form_single_phase(orc):
    # single-phase cell block [[P, 0, a], [q, d, -c], [0, 0, 1]] has det = P d
    A = orc.as_csr([0, 2, 5, 6], [0, 2, 0, 1, 2, 2], [4.0, 0.5, 0.25, 2.0, -0.75, 1.0])
    binv = orc.block_inverse(A, 3).reshape(3, 3)
    P, a, q, d, c = 4.0, 0.5, 0.25, 2.0, 0.75
    exact = np.array([[1 / P, 0, -a / P], [-q / (P * d), 1 / d, (c + q * a / P) / d], [0, 0, 1]])
    np.testing.assert_allclose(binv, exact, rtol=1e-15, atol=1e-16)


def test_block_inverse_singular(orc):
    A = orc.as_csr([0, 1, 2, 2], [0, 1], [1.0, 1.0])
    with pytest.raises(np.linalg.LinAlgError):
        orc.block_inverse(A, 3)


@pytest.mark.parametrize("n", [1, 5, 33, 64])
def test_dense_lu_solve(orc, n):
    rng = np.random.default_rng(n)
    a = rng.standard_normal((n, n)) + n * np.eye(n) * 0.1
    b = rng.standard_normal(n)
    lu, perm = orc.dense_lu(a)
    x = orc.dense_lu_solve(lu, perm, b)
    np.testing.assert_allclose(x, np.linalg.solve(a, b), rtol=1e-9, atol=1e-10)
    L = np.tril(lu, -1) + np.eye(n)
    U = np.triu(lu)
    np.testing.assert_allclose(L @ U, a[perm], rtol=1e-12, atol=1e-12)


def test_dense_lu_pivot_ties_pick_lowest_row(orc):
    a = np.array([[1.0, 2.0], [-1.0, 3.0]])  # |1| == |-1|: row 0 stays
    _, perm = orc.dense_lu(a)
    assert perm.tolist() == [0, 1]
    a = np.array([[0.5, 2.0], [-1.0, 3.0], [1.0, 1.0]])[:2]
    _, perm = orc.dense_lu(a)
    assert perm.tolist() == [1, 0]


def test_splitmix64_published_vectors(orc):
    vals = [int(l) for l in open(os.path.join(HERE, "golden", "splitmix64_seed1234567.txt"))
            if l.strip() and not l.startswith("#")]
    golden_ratio = 0x9E3779B97F4A7C15
    got = [orc.splitmix64((1234567 + k * golden_ratio) % 2**64) for k in range(len(vals))]
    assert got == vals


def test_pattern_outer(orc):
    A = rand_csr(orc, 6, 6, 0.4, 5)
    lam = np.arange(6, dtype=float) + 1
    x = np.arange(6, dtype=float) * 0.5 - 1
    d = orc.pattern_outer(A, lam, x)
    full = -np.outer(lam, x)
    for i in range(6):
        for p in range(A.indptr[i], A.indptr[i + 1]):
            assert d[p] == full[i, A.indices[p]]
