"""ctypes view of the plain-C oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It never touches the GPU library.

Matrices cross the boundary as ``CSR`` tuples of numpy arrays
(indptr int64, indices int32, data float64 or None, shape).
"""
from __future__ import annotations

import ctypes as C
import os
from collections import namedtuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

CSR = namedtuple("CSR", ["indptr", "indices", "data", "shape"])

OK, NOT_CONVERGED, E_INVALID, E_ZERO_FDIAG, E_SINGULAR_BLOCK, E_BREAKDOWN = 0, 1, -1, -2, -3, -4


class _Mat(C.Structure):
    _fields_ = [("nrows", C.c_int64), ("ncols", C.c_int64), ("nnz", C.c_int64),
                ("rp", C.POINTER(C.c_int64)), ("ci", C.POINTER(C.c_int32)), ("v", C.POINTER(C.c_double))]


class _Opts(C.Structure):
    _fields_ = [("restart", C.c_int), ("max_iter", C.c_int), ("rp_type", C.c_int), ("global_relax", C.c_int),
                ("f_sweeps", C.c_int), ("amg_theta", C.c_double), ("amg_pre", C.c_int), ("amg_post", C.c_int),
                ("amg_max_levels", C.c_int), ("amg_coarse_max", C.c_int), ("dense_max", C.c_int),
                ("pmis_seed", C.c_uint64), ("precision", C.c_int), ("use_x0", C.c_int),
                ("frelax_amg_mask", C.c_int), ("frelax_amg_pre", C.c_int), ("frelax_amg_post", C.c_int),
                ("cycle_post", C.c_int)]


class _Stats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("status", C.c_int), ("rel_residual", C.c_double),
                ("setup_ms", C.c_double), ("solve_ms", C.c_double), ("n_levels", C.c_int),
                ("level_n", C.c_int64 * 64), ("level_nnz", C.c_int64 * 64),
                ("res_history", C.POINTER(C.c_double)), ("res_history_cap", C.c_int),
                ("res_history_len", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b  # type: ignore
            _b.build()
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        L.orc_default_opts.argtypes = [P(_Opts)]
        L.orc_mat_free.argtypes = [P(_Mat)]
        L.orc_spmv.argtypes = [P(_Mat), C.c_void_p, C.c_void_p]
        L.orc_transpose.argtypes = [P(_Mat), P(_Mat)]
        L.orc_spgemm.argtypes = [P(_Mat), P(_Mat), P(_Mat)]
        L.orc_strength.argtypes = [P(_Mat), C.c_double, P(_Mat)]
        L.orc_pmis.argtypes = [P(_Mat), C.c_uint64, C.c_void_p]
        L.orc_interp.argtypes = [P(_Mat), P(_Mat), C.c_void_p, P(_Mat)]
        L.orc_splitmix64.argtypes = [C.c_uint64]
        L.orc_splitmix64.restype = C.c_uint64
        L.orc_block_inverse.argtypes = [C.c_int64, C.c_int, P(_Mat), C.c_void_p]
        L.orc_dense_lu.argtypes = [C.c_int, C.c_void_p, C.c_void_p]
        L.orc_dense_lu_solve.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_setup.argtypes = [P(_Mat), C.c_int, C.c_void_p, P(_Opts), P(C.c_void_p), C.c_char_p, C.c_int]
        L.orc_solve.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, P(_Stats)]
        L.orc_vcycle.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_pattern_outer.argtypes = [P(_Mat), C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_num_mgr_levels.argtypes = [C.c_void_p]
        L.orc_num_amg_levels.argtypes = [C.c_void_p]
        L.orc_num_ff_levels.argtypes = [C.c_void_p, C.c_int]
        L.orc_get_mat.argtypes = [C.c_void_p, C.c_int, C.c_int, P(_Mat)]
        L.orc_get_vec_len.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.orc_get_vec_len.restype = C.c_int64
        L.orc_get_vec.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p]
        _lib = L
    return _lib


def as_csr(indptr, indices, data, shape=None) -> CSR:
    indptr = np.ascontiguousarray(indptr, dtype=np.int64)
    indices = np.ascontiguousarray(indices, dtype=np.int32)
    data = None if data is None else np.ascontiguousarray(data, dtype=np.float64)
    n = indptr.shape[0] - 1
    if shape is None:
        shape = (n, n)
    return CSR(indptr, indices, data, tuple(int(s) for s in shape))


def from_scipy(M) -> CSR:
    M = M.tocsr()
    return as_csr(M.indptr, M.indices, M.data, M.shape)


def to_scipy(M: CSR):
    import scipy.sparse as sp
    data = M.data if M.data is not None else np.ones(M.indices.shape[0])
    return sp.csr_matrix((data, M.indices, M.indptr), shape=M.shape)


def _mat(M: CSR) -> _Mat:
    m = _Mat()
    m.nrows, m.ncols = M.shape
    m.nnz = M.indices.shape[0]
    m.rp = M.indptr.ctypes.data_as(C.POINTER(C.c_int64))
    m.ci = M.indices.ctypes.data_as(C.POINTER(C.c_int32))
    m.v = M.data.ctypes.data_as(C.POINTER(C.c_double)) if M.data is not None else C.POINTER(C.c_double)()
    return m


def _copy_out(m: _Mat) -> CSR:
    nr, nnz = m.nrows, m.nnz
    indptr = np.ctypeslib.as_array(m.rp, shape=(nr + 1,)).copy() if nr >= 0 else np.zeros(1, np.int64)
    indices = np.ctypeslib.as_array(m.ci, shape=(nnz,)).copy() if nnz > 0 else np.zeros(0, np.int32)
    data = None
    if bool(m.v):
        data = np.ctypeslib.as_array(m.v, shape=(nnz,)).copy() if nnz > 0 else np.zeros(0)
    return CSR(indptr, indices, data, (int(m.nrows), int(m.ncols)))


def _owned(m: _Mat) -> CSR:
    out = _copy_out(m)
    lib().orc_mat_free(C.byref(m))
    return out


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


# ---------------- building blocks ----------------

def spmv(A: CSR, x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(A.shape[0])
    lib().orc_spmv(C.byref(_mat(A)), _p(x), _p(y))
    return y


def transpose(A: CSR) -> CSR:
    out = _Mat()
    lib().orc_transpose(C.byref(_mat(A)), C.byref(out))
    return _owned(out)


def spgemm(A: CSR, B: CSR) -> CSR:
    out = _Mat()
    rc = lib().orc_spgemm(C.byref(_mat(A)), C.byref(_mat(B)), C.byref(out))
    if rc != OK:
        raise ValueError("spgemm: shape mismatch")
    return _owned(out)


def strength(A: CSR, theta=0.25) -> CSR:
    out = _Mat()
    lib().orc_strength(C.byref(_mat(A)), float(theta), C.byref(out))
    return _owned(out)


def pmis(S: CSR, seed=0):
    cf = np.empty(S.shape[0], dtype=np.int32)
    rc = lib().orc_pmis(C.byref(_mat(S)), C.c_uint64(seed), _p(cf))
    if rc != OK:
        raise RuntimeError("pmis failed")
    return cf


def interp(A: CSR, S: CSR, cf) -> CSR:
    cf = np.ascontiguousarray(cf, dtype=np.int32)
    out = _Mat()
    lib().orc_interp(C.byref(_mat(A)), C.byref(_mat(S)), _p(cf), C.byref(out))
    return _owned(out)


def splitmix64(x: int) -> int:
    return int(lib().orc_splitmix64(C.c_uint64(x)))


def block_inverse(A: CSR, bs=3):
    ncell = A.shape[0] // bs
    out = np.empty(ncell * bs * bs)
    rc = lib().orc_block_inverse(ncell, bs, C.byref(_mat(A)), _p(out))
    if rc != OK:
        raise np.linalg.LinAlgError("singular cell block")
    return out


def dense_lu(a):
    a = np.ascontiguousarray(a, dtype=np.float64).copy()
    n = a.shape[0]
    perm = np.empty(n, dtype=np.int32)
    rc = lib().orc_dense_lu(n, _p(a), _p(perm))
    if rc != OK:
        raise np.linalg.LinAlgError("singular")
    return a, perm


def dense_lu_solve(lu, perm, b):
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.empty_like(b)
    lib().orc_dense_lu_solve(lu.shape[0], _p(np.ascontiguousarray(lu)), _p(np.ascontiguousarray(perm, np.int32)),
                             _p(b), _p(x))
    return x


def pattern_outer(A: CSR, lam, x):
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty(A.indices.shape[0])
    lib().orc_pattern_outer(C.byref(_mat(A)), _p(lam), _p(x), _p(out))
    return out


# ---------------- the solver ----------------

DEFAULTS = dict(restart=30, max_iter=400, rp_type=0, global_relax=1, f_sweeps=1, amg_theta=0.25, amg_pre=2,
                amg_post=2, amg_max_levels=25, amg_coarse_max=64, dense_max=4096, pmis_seed=0, precision=0,
                use_x0=0, frelax_amg_mask=0, frelax_amg_pre=1, frelax_amg_post=1, cycle_post=0)


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle status {code}: {msg}")
        self.code = code


class Result(namedtuple("Result", ["x", "status", "iterations", "rel_residual", "history", "setup_ms",
                                   "solve_ms", "level_n", "level_nnz"])):
    pass


class Oracle:
    """MGR-preconditioned GMRES on the host (FP64; precision=1 applies the
    hierarchy in FP32 inside the same FP64 Krylov loop)."""

    def __init__(self, A: CSR, labels, block_size=3, **opts):
        self.A = A
        self.labels = np.ascontiguousarray(labels, dtype=np.int32)
        o = _Opts()
        lib().orc_default_opts(C.byref(o))
        for k, v in opts.items():
            if k not in DEFAULTS:
                raise TypeError(f"unknown option {k}")
            setattr(o, k, v)
        self.opts = o
        h = C.c_void_p()
        err = C.create_string_buffer(256)
        self._mat = _mat(A)
        rc = lib().orc_setup(C.byref(self._mat), block_size, _p(self.labels), C.byref(o), C.byref(h), err, 256)
        if rc != OK:
            raise OracleError(rc, err.value.decode())
        self.h = h
        self.n = A.shape[0]

    def close(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    __del__ = close

    def solve(self, b, tol=1e-8, x0=None) -> Result:
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros(self.n) if x0 is None else np.ascontiguousarray(x0, dtype=np.float64).copy()
        hist = np.zeros(max(self.opts.max_iter, 1) + 1)
        st = _Stats()
        st.res_history = hist.ctypes.data_as(C.POINTER(C.c_double))
        st.res_history_cap = hist.shape[0]
        rc = lib().orc_solve(self.h, _p(b), _p(x), float(tol), C.byref(st))
        nl = st.n_levels
        return Result(x, rc, st.iterations, st.rel_residual, hist[: st.res_history_len].copy(), st.setup_ms,
                      st.solve_ms, list(st.level_n[:nl]), list(st.level_nnz[:nl]))

    def vcycle(self, r):
        r = np.ascontiguousarray(r, dtype=np.float64)
        e = np.empty(self.n)
        lib().orc_vcycle(self.h, _p(r), _p(e))
        return e

    @property
    def n_mgr_levels(self):
        return lib().orc_num_mgr_levels(self.h)

    @property
    def n_amg_levels(self):
        return lib().orc_num_amg_levels(self.h)

    def _mat_view(self, kind, level) -> CSR:
        m = _Mat()
        rc = lib().orc_get_mat(self.h, kind, level, C.byref(m))
        if rc != OK:
            raise IndexError((kind, level))
        return _copy_out(m)

    def _vec(self, kind, level, dtype):
        n = lib().orc_get_vec_len(self.h, kind, level)
        if n < 0:
            raise IndexError((kind, level))
        out = np.empty(n, dtype=dtype)
        lib().orc_get_vec(self.h, kind, level, _p(out))
        return out

    def mgr_level(self, l):
        return dict(A=self._mat_view(0, l), P=self._mat_view(1, l), R=self._mat_view(2, l),
                    dinv=self._vec(1, l, np.float64), flist=self._vec(2, l, np.int32),
                    clist=self._vec(3, l, np.int32))

    def amg_level(self, k):
        d = dict(A=self._mat_view(3, k))
        if k < self.n_amg_levels - 1:
            d.update(P=self._mat_view(4, k), S=self._mat_view(5, k), cf=self._vec(4, k, np.int32),
                     l1=self._vec(5, k, np.float64))
        return d

    def n_ff_levels(self, l):
        return lib().orc_num_ff_levels(self.h, l)

    def ff_level(self, l, k):
        """F-relaxation AMG hierarchy of MGR level l, level k."""
        code = (l << 8) | k
        d = dict(A=self._mat_view(6, code))
        if k < self.n_ff_levels(l) - 1:
            d.update(P=self._mat_view(7, code), cf=self._vec(8, code, np.int32), l1=self._vec(9, code, np.float64))
        return d

    def ff_coarse_lu(self, l):
        n = self.ff_level(l, self.n_ff_levels(l) - 1)["A"].shape[0]
        return self._vec(10, l << 8, np.float64).reshape(n, n), self._vec(11, l << 8, np.int32)

    def block_inverses(self):
        return self._vec(0, 0, np.float64)

    def coarse_lu(self):
        n = self.amg_level(self.n_amg_levels - 1)["A"].shape[0]
        return self._vec(6, 0, np.float64).reshape(n, n), self._vec(7, 0, np.int32)


def adjoint(A: CSR, labels, g, tol=1e-8, block_size=3, **opts):
    """lambda = A^{-T} g with a hierarchy built on A^T (same labels)."""
    AT = transpose(A)
    o = Oracle(AT, labels, block_size, **opts)
    try:
        return o.solve(g, tol)
    finally:
        o.close()
