"""Helpers shared by the GPU tests: build the same seeded system for the HIP
library and the oracle, and pull hierarchy data out of both."""
import numpy as np

from synth import make_system


def oracle_csr(orc, s):
    return orc.as_csr(s.indptr, s.indices, s.data)


def gpu_solver(s, **kw):
    from paper_1801_08464_amd.solver import MGRSolver
    return MGRSolver(s.indptr, s.indices, s.data, s.labels, **kw)


def assert_same_csr(gpu_mat, orc_mat, what):
    rp, ci, v, shape = gpu_mat
    assert tuple(shape) == tuple(orc_mat.shape), (what, shape, orc_mat.shape)
    np.testing.assert_array_equal(rp.astype(np.int64), orc_mat.indptr, err_msg=f"{what}: row pointers")
    np.testing.assert_array_equal(ci, orc_mat.indices, err_msg=f"{what}: columns")
    if v is not None and orc_mat.data is not None:
        np.testing.assert_array_equal(v, orc_mat.data, err_msg=f"{what}: values (bitwise)")


def small_system(grid=(7, 5), seed=3, sigma=1.5, frac=0.4, region="disk"):
    return make_system(grid, sigma, region, frac, seed)
