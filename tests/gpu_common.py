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


# Element-wise V-cycle parity (HIP path against the oracle on the same input r).
# FP64: the two sides differ by rounding order only (tree-reduced row sums on
# the small AMG levels, sequential ones in the oracle), a few ulps per entry
# carried through the levels.  FP32 (mixed form, against the oracle's FP32-apply
# mode on the same once-rounded values): the same rounding-order differences at
# unit roundoff 6e-8 instead of 1.1e-16.
VCYCLE_TOL = {"fp64": (1e-10, 1e-12), "mixed": (2e-4, 2e-6)}


def assert_vcycle_close(z, ze, precision, what=""):
    rtol, atol = VCYCLE_TOL[precision]
    scale = float(np.abs(ze).max())
    d = np.abs(z - ze)
    worst = float((d / (rtol * np.abs(ze) + atol * scale)).max()) if ze.size else 0.0
    print(f"[vcycle {what} {precision}] max |dz| / max |z| = {d.max() / scale:.2e}, "
          f"worst entry at {worst:.2e} of the bound", flush=True)
    np.testing.assert_allclose(z, ze, rtol=rtol, atol=atol * scale, err_msg=what)
