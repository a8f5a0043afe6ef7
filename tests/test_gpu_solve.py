"""Solve-phase parity of the HIP path against the oracle: the fine SpMV, one
V-cycle, full MGR-GMRES (iteration count within 1, matched-iteration solution
error), the mixed-precision form, status codes and edge cases."""
import numpy as np
import pytest

from gpu_common import assert_vcycle_close, gpu_solver, oracle_csr, small_system
from synth import make_config, make_poisson, random_vector

pytestmark = pytest.mark.gpu


def test_fine_spmv_bitwise(orc):
    for s in (make_config(1), small_system((13, 11, 9), seed=4, sigma=2.0, frac=0.3, region="ball")):
        print(f"[spmv] n={s.n}", flush=True)
        A = oracle_csr(orc, s)
        g = gpu_solver(s)
        x = random_vector(s.n, 5)
        y = g.spmv(x).cpu().numpy()
        np.testing.assert_array_equal(y, orc.spmv(A, x))
        g.close()


VCYCLE_CASES = [dict(), dict(cycle_post=1), dict(global_relax=0), dict(rp_type=1), dict(rp_type=2),
                dict(f_sweeps=2), dict(frelax_amg_mask=2), dict(frelax_amg_mask=3, global_relax=0),
                dict(cycle_post=1, frelax_amg_mask=2, f_sweeps=2)]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("opts", VCYCLE_CASES)
def test_vcycle_matches_oracle(orc, precision, opts):
    # every reachable path of the cycle: the residual over A's F columns only
    # (global_relax 0), the scatter-add prolongation (W_p = 0), injective R,
    # several F-sweeps, the F-block AMG and the post-smoothing form
    s = small_system((29, 23), seed=12, sigma=2.0, frac=0.35)
    o = orc.Oracle(oracle_csr(orc, s), s.labels, precision=1 if precision == "mixed" else 0, **opts)
    g = gpu_solver(s, precision=precision, **opts)
    r = random_vector(s.n, 1)
    z = g.apply_preconditioner(r).cpu().numpy()
    ze = o.vcycle(r)
    assert_vcycle_close(z, ze, precision, str(opts))
    g.close()
    o.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_vcycle_with_stream_amg_levels_matches_oracle(orc, precision):
    # 52^3 cells: the coarse-grid matrix has 140,608 rows of ~23 entries, so its
    # sweeps and residuals run in the jagged stream kernel over its row-block
    # jagged copy, and the next AMG levels in the stream kernel with 64- and
    # 128-row blocks (the V-cycle tests above only reach the small-level kernels)
    s = small_system((52, 52, 52), seed=6, sigma=2.0, frac=0.3, region="ball")
    print(f"[vcycle stream levels] n={s.n} {precision}", flush=True)
    o = orc.Oracle(oracle_csr(orc, s), s.labels, precision=1 if precision == "mixed" else 0, frelax_amg_mask=2)
    g = gpu_solver(s, precision=precision, frelax_amg_mask=2)
    rp3 = g.get_matrix(3, 0)[0]
    n3 = rp3.shape[0] - 1
    assert n3 >= 131072 and rp3[-1] >= 12 * n3
    r = random_vector(s.n, 2)
    z = g.apply_preconditioner(r).cpu().numpy()
    ze = o.vcycle(r)
    assert_vcycle_close(z, ze, precision, "52^3")
    # the same input twice gives the same bits
    z2 = g.apply_preconditioner(r).cpu().numpy()
    np.testing.assert_array_equal(z, z2)
    o.close()
    g.close()


@pytest.mark.parametrize("cfg", [1, "3d"])
def test_solve_matches_oracle(orc, cfg):
    s = make_config(1) if cfg == 1 else small_system((24, 24, 24), seed=3, sigma=1.5, frac=0.35, region="ball")
    print(f"[solve] cfg={cfg} n={s.n}", flush=True)
    A = oracle_csr(orc, s)
    ro = orc.Oracle(A, s.labels).solve(s.b, 1e-8)
    assert ro.status == 0
    g = gpu_solver(s)
    x, info = g.solve(s.b, 1e-8)
    x = x.cpu().numpy()
    assert info.status == 0
    assert abs(info.iterations - ro.iterations) <= 1, (info.iterations, ro.iterations)
    res = np.linalg.norm(s.b - orc.spmv(A, x)) / np.linalg.norm(s.b)
    assert res <= 1e-8 and info.rel_residual <= 1e-8
    assert info.level_n == ro.level_n and info.level_nnz == ro.level_nnz
    g.close()
    # matched-iteration mode: the same number of Arnoldi steps with tol = 0
    gm = gpu_solver(s, max_iter=ro.iterations)
    xm, im = gm.solve(s.b, 0.0)
    assert im.iterations == ro.iterations
    err = np.linalg.norm(xm.cpu().numpy() - ro.x) / np.linalg.norm(ro.x)
    assert err <= 1e-8, err
    gm.close()


@pytest.mark.parametrize("cfg", [1, "3d"])
def test_mixed_precision_solve(orc, cfg):
    s = make_config(1) if cfg == 1 else small_system((24, 24, 24), seed=3, sigma=1.5, frac=0.35, region="ball")
    A = oracle_csr(orc, s)
    ro = orc.Oracle(A, s.labels, precision=1).solve(s.b, 1e-8)
    g = gpu_solver(s, precision="mixed")
    x, info = g.solve(s.b, 1e-8)
    assert info.status == 0
    assert abs(info.iterations - ro.iterations) <= 1, (info.iterations, ro.iterations)
    res = np.linalg.norm(s.b - orc.spmv(A, x.cpu().numpy())) / np.linalg.norm(s.b)
    assert res <= 1e-8
    g.close()


def test_residual_history_monotone():
    s = small_system((32, 32), seed=4, sigma=2.0)
    g = gpu_solver(s, restart=5)
    x, info = g.solve(s.b, 1e-10)
    h = info.history
    assert info.status == 0 and len(h) == info.iterations
    assert np.all(h[1:] <= h[:-1] * (1 + 1e-6))
    g.close()


@pytest.mark.parametrize("opts", [dict(rp_type=1), dict(rp_type=2), dict(global_relax=0), dict(f_sweeps=0),
                                  dict(f_sweeps=2), dict(amg_pre=1, amg_post=3), dict(amg_pre=0, amg_post=1),
                                  dict(restart=1, max_iter=2000), dict(restart=64), dict(frelax_amg_mask=2),
                                  dict(frelax_amg_mask=2, f_sweeps=2, global_relax=0),
                                  dict(frelax_amg_mask=3, precision="mixed"), dict(cycle_post=1),
                                  dict(cycle_post=1, frelax_amg_mask=2, f_sweeps=2),
                                  dict(cycle_post=1, rp_type=1, precision="mixed")])
def test_option_variants_match_oracle(orc, opts):
    s = small_system((19, 17), seed=6)
    A = oracle_csr(orc, s)
    oopts = {k: (1 if v == "mixed" else v) for k, v in opts.items()}
    ro = orc.Oracle(A, s.labels, **oopts).solve(s.b, 1e-8)
    g = gpu_solver(s, **opts)
    x, info = g.solve(s.b, 1e-8)
    assert info.status == ro.status
    if ro.status == 0:
        assert abs(info.iterations - ro.iterations) <= 1, (opts, info.iterations, ro.iterations)
    g.close()
    # matched-iteration mode: exactly the oracle's number of Arnoldi steps with tol = 0
    gm = gpu_solver(s, **(opts | dict(max_iter=ro.iterations)))
    xm, im = gm.solve(s.b, 0.0)
    assert im.iterations == ro.iterations
    err = np.linalg.norm(xm.cpu().numpy() - ro.x) / np.linalg.norm(ro.x)
    print(f"[variant {opts}] iterations {ro.iterations}, matched-iteration error {err:.2e}", flush=True)
    # FP64: the relative solution error bound of the FP64 runs; mixed (against the
    # oracle's FP32-apply mode): the V-cycles agree to FP32 rounding order only,
    # and flexible GMRES carries those differences into the iterates
    assert err <= (1e-8 if opts.get("precision") != "mixed" else 1e-5), (opts, err)
    gm.close()


def test_plain_amg_and_block_size_one(orc):
    ip, ix, dv, b = make_poisson((40, 33))
    n = ip.shape[0] - 1
    from paper_1801_08464_amd.solver import MGRSolver
    ro = orc.Oracle(orc.as_csr(ip, ix, dv), np.zeros(n, np.int32), block_size=1).solve(b, 1e-8)
    g = MGRSolver(ip, ix, dv, np.zeros(n, np.int32), block_size=1)
    x, info = g.solve(b, 1e-8)
    assert info.status == 0 and abs(info.iterations - ro.iterations) <= 1
    g.close()


def test_tiny_systems(orc):
    # one cell (coarse grid of one unknown), and a grid whose whole hierarchy is a dense LU
    for grid in ((1, 1), (2, 1), (3, 3)):
        s = small_system(grid, seed=1, frac=0.5)
        A = oracle_csr(orc, s)
        ro = orc.Oracle(A, s.labels).solve(s.b, 1e-10)
        g = gpu_solver(s)
        x, info = g.solve(s.b, 1e-10)
        assert info.status == 0 and abs(info.iterations - ro.iterations) <= 1
        np.testing.assert_allclose(x.cpu().numpy(), s.x_true, rtol=1e-7, atol=1e-7)
        g.close()


@pytest.mark.parametrize("opts", [dict(), dict(restart=64), dict(restart=2), dict(precision="mixed")])
def test_exhausted_krylov_space_with_zero_tolerance(opts):
    # one cell (n = 3) and tol = 0: the Krylov space is exhausted after at most
    # three steps and the iteration continues on rounding noise until max_iter.
    # The lagged re-orthogonalisation (restart <= 32) detects a vector inside the
    # span of the basis and ends the cycle; every path must stay finite and keep
    # the exact solution.
    s = small_system((1, 1), seed=1, frac=0.5)
    g = gpu_solver(s, max_iter=12, **opts)
    x, info = g.solve(s.b, 0.0)
    xv = x.cpu().numpy()
    assert info.status in (0, 1) and info.iterations <= 12
    assert np.all(np.isfinite(xv)) and np.isfinite(info.rel_residual)
    np.testing.assert_allclose(xv, s.x_true, rtol=1e-9, atol=1e-9)
    assert info.rel_residual <= 1e-12
    g.close()


def test_zero_rhs_and_initial_guess():
    s = small_system()
    g = gpu_solver(s, use_x0=1)
    x, info = g.solve(np.zeros(s.n), 1e-8, x0=np.ones(s.n))
    assert info.status == 0 and info.iterations == 0 and not x.cpu().numpy().any()
    x, info = g.solve(s.b, 1e-8, x0=s.x_true)
    assert info.status == 0 and info.iterations == 0
    g.close()


def test_status_codes_through_the_abi():
    from paper_1801_08464_amd import binding as B
    s = small_system()
    bad = s.labels.copy()
    two = np.where(s.two_phase)[0][0]
    bad[3 * two + 2] = 0
    with pytest.raises(B.MGRError) as e:
        gpu_solver(s.__class__(**{**s.__dict__, "labels": bad}))
    assert e.value.code == B.E_ZERO_FDIAG and str(3 * two + 2) in str(e.value)
    with pytest.raises(B.MGRError) as e:
        gpu_solver(s.__class__(**{**s.__dict__, "labels": np.full(s.n, 40, np.int32)}))
    assert e.value.code == B.E_INVALID
    unsorted = s.indices.copy()
    unsorted[[0, 1]] = unsorted[[1, 0]]
    with pytest.raises(B.MGRError) as e:
        gpu_solver(s.__class__(**{**s.__dict__, "indices": unsorted}))
    assert e.value.code == B.E_INVALID
    with pytest.raises(B.MGRError) as e:
        gpu_solver(s, restart=0)
    assert e.value.code == B.E_INVALID
    g = gpu_solver(s, max_iter=1)
    x, info = g.solve(s.b, 1e-12)
    assert info.status == B.NOT_CONVERGED and info.iterations == 1 and np.isfinite(x.cpu().numpy()).all()
    g.close()
    g = gpu_solver(s)
    b = s.b.copy()
    b[3] = np.nan
    x, info = g.solve(b, 1e-8)
    assert info.status == B.E_BREAKDOWN
    g.close()


def test_validation_covers_every_row_of_a_large_input():
    # more rows than the validation kernel has threads (1024 workgroups of 256):
    # a bad entry or label in the last rows is still caught
    from paper_1801_08464_amd import binding as B
    s = small_system((48, 48, 48), seed=2, region="ball")
    assert s.n > 1024 * 256
    print(f"[validation] n={s.n}", flush=True)
    unsorted = s.indices.copy()
    last = np.nonzero(np.diff(s.indptr) >= 2)[0][-1]  # the last row with two entries
    assert last > 1024 * 256
    a = s.indptr[last]
    unsorted[[a, a + 1]] = unsorted[[a + 1, a]]
    with pytest.raises(B.MGRError) as e:
        gpu_solver(s.__class__(**{**s.__dict__, "indices": unsorted}))
    assert e.value.code == B.E_INVALID
    bad = s.labels.copy()
    bad[-1] = 32
    with pytest.raises(B.MGRError) as e:
        gpu_solver(s.__class__(**{**s.__dict__, "labels": bad}))
    assert e.value.code == B.E_INVALID


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_index16_falls_back_where_a_slot_spans_too_far(precision):
    # a 29^3 system (73,167 rows) in which the pressure row of cell 24,256 (the
    # first cell of a full 64-cell slice) also couples to the pressure of cell 0:
    # that slice's first pressure slot then holds column 0 beside columns above
    # 70,000, a span no 16-bit offset reaches, so the fine operator keeps 32-bit
    # columns (the same bytes per launch as with index16 = 0) and every result is
    # bitwise that of the 32-bit form
    import dataclasses
    import scipy.sparse as sp
    s = small_system((29, 29, 29), seed=9, sigma=1.5, frac=0.3, region="ball")
    # the unmodified system packs 16-bit columns
    g = gpu_solver(s, precision=precision, index16=1)
    g.set_kernel_timing(True)
    g.spmv(random_vector(s.n, 17))
    _, n_plain, b_plain = g.kernel_time(0)
    g.close()
    i = 3 * 24256
    A = sp.csr_matrix((s.data, s.indices, s.indptr), shape=(s.n, s.n))
    assert A.indices[A.indptr[i]] > 65535 + 3 * 64
    eps = 1e-3 * A[i, i]
    A = (A + sp.csr_matrix(([-eps, eps], ([i, i], [0, i])), shape=A.shape)).tocsr()
    A.sort_indices()
    assert A.indices[A.indptr[i]] == 0
    s = dataclasses.replace(s, indptr=A.indptr.astype(np.int32), indices=A.indices.astype(np.int32),
                            data=np.ascontiguousarray(A.data, dtype=np.float64))
    r = random_vector(s.n, 17)
    out = {}
    for c16 in (1, 0):
        print(f"[index16 fallback] {precision} index16={c16} n={s.n}", flush=True)
        g = gpu_solver(s, precision=precision, index16=c16)
        g.set_kernel_timing(True)
        z = g.apply_preconditioner(r).cpu().numpy()
        _, nz, bz = g.kernel_time(0)
        y = g.spmv(r).cpu().numpy()
        _, ny, by = g.kernel_time(0)
        g.close()
        assert nz > 0 and ny == 1
        out[c16] = (z, y, bz / nz, by)
    assert n_plain == 1 and b_plain < out[0][3] - 1.5 * len(s.data), (b_plain, out[0][3])
    assert out[1][2:] == out[0][2:], (out[1][2:], out[0][2:])
    assert np.array_equal(out[1][0], out[0][0])
    assert np.array_equal(out[1][1], out[0][1])


def test_empty_system_is_rejected():
    # n = 0: the setup refuses it (no partial handle is returned)
    from paper_1801_08464_amd import binding as B
    from paper_1801_08464_amd.solver import MGRSolver
    with pytest.raises(B.MGRError) as e:
        MGRSolver(np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0), np.zeros(0, np.int32))
    assert e.value.code == B.E_INVALID


def test_amg_frelaxation_solve_matched_iterations(orc):
    s = small_system((20, 20, 20), seed=4, sigma=2.0, frac=0.3, region="ball")
    A = oracle_csr(orc, s)
    ro = orc.Oracle(A, s.labels, frelax_amg_mask=2).solve(s.b, 1e-8)
    g = gpu_solver(s, frelax_amg_mask=2)
    x, info = g.solve(s.b, 1e-8)
    assert info.status == 0 and abs(info.iterations - ro.iterations) <= 1
    g.close()
    gm = gpu_solver(s, frelax_amg_mask=2, max_iter=ro.iterations)
    xm, _ = gm.solve(s.b, 0.0)
    assert np.linalg.norm(xm.cpu().numpy() - ro.x) / np.linalg.norm(ro.x) <= 1e-8
    gm.close()


def test_kernel_timing_counts_and_bytes():
    # kernel 0: every level-0 sliced-ELL launch; kernel 1: every preconditioner
    # application; kernel 2: the sweeps on the coarse-grid matrix, launched on
    # their own when it is larger than the single-workgroup tail takes (1,600
    # rows here; the levels below it run in the tail kernel)
    # (32-bit columns in the sliced ELL: the byte model below; the 16-bit form is
    # checked at the end)
    s = small_system((40, 40), seed=5, sigma=1.0, frac=0.4)
    g = gpu_solver(s, index16=0)
    g.set_kernel_timing(True)
    x, info = g.solve(s.b, 1e-8)
    ms0, n0, b0 = g.kernel_time(0)
    ms1, n1, b1 = g.kernel_time(1)
    assert n1 == info.iterations
    # per Arnoldi step one product w = A z and one level-0 residual inside the V-cycle,
    # plus one true residual per restart cycle
    cycles = -(-info.iterations // 30)
    assert n0 == 2 * info.iterations + cycles + 1
    assert ms0 > 0 and ms1 > 0
    nnz, n = len(s.data), s.n
    per0 = b0 / n0
    assert 12 * nnz + 4 * (n + 1) + 16 * n <= per0 <= 12 * nnz + 4 * (n + 1) + 24 * n
    # a V-cycle reads the level-0 matrix at least once
    assert b1 / n1 > 12 * nnz
    # the coarse-grid sweeps: V(2,2) from zero is one sweep after the division, then two
    ms2, n2, b2 = g.kernel_time(2)
    assert n2 == 3 * info.iterations and ms2 > 0
    A3 = g.get_matrix(3, 0)
    n3, nnz3 = A3[3][0], len(A3[1])
    assert b2 / n2 == 12 * nnz3 + 4 * (n3 + 1) + 8 * n3 + 3 * 8 * n3
    # counters reset after reading
    assert g.kernel_time(1)[1] == 0
    with pytest.raises(Exception):
        g.kernel_time(3)
    g.close()
    # 16-bit columns in the sliced ELL: 2 bytes less per entry, 4 more per slot
    # of 64 (a slot's base)
    g = gpu_solver(s, index16=1)
    g.set_kernel_timing(True)
    g.solve(s.b, 1e-8)
    _, n16, b16 = g.kernel_time(0)
    g.close()
    assert n16 == n0
    assert 1.5 * nnz < per0 - b16 / n16 <= 2 * nnz, (per0, b16 / n16, nnz)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_kernel_timing_on_the_mid_size_stream_kernel(precision):
    # config 3 (64^3): the coarse-grid matrix (262,144 rows) runs in the mid-size
    # stream kernel, whose timed launches record their own events; the sweeps
    # lie inside the V-cycles, so their summed time is below the V-cycles'
    s = make_config(3)
    g = gpu_solver(s, precision=precision)
    g.set_kernel_timing(True)
    x, info = g.solve(s.b, 1e-8)
    assert info.status == 0
    ms1, n1, _ = g.kernel_time(1)
    ms2, n2, b2 = g.kernel_time(2)
    ms0, n0, _ = g.kernel_time(0)
    A3 = g.get_matrix(3, 0)
    n3, nnz3 = A3[3][0], len(A3[1])
    g.close()
    assert n3 == 64 ** 3 and n1 == info.iterations and n2 == 3 * info.iterations
    S = 8 if precision == "fp64" else 4
    assert b2 / n2 == (S + 4) * nnz3 + 4 * (n3 + 1) + S * n3 + 3 * S * n3
    assert 0 < ms2 < ms1 and ms0 > 0
    print(f"[timing cfg3 {precision}] sweep {1e3 * ms2 / n2:.1f} us, V-cycle {1e3 * ms1 / n1:.1f} us, "
          f"fine {1e3 * ms0 / n0:.1f} us", flush=True)


def test_reused_device_blocks_give_the_same_bits():
    # a destroyed handle's device blocks are reused by the next handle (with the
    # old contents in them): the results must not depend on that
    s = small_system((21, 17, 6), seed=13, sigma=2.0, frac=0.3, region="ball")
    outs = []
    for precision in ("fp64", "fp64", "mixed", "mixed"):
        g = gpu_solver(s, precision=precision, frelax_amg_mask=2)
        x, info = g.solve(s.b, 1e-10)
        outs.append((precision, info.iterations, x.cpu().numpy()))
        g.close()
    for a, b in ((0, 1), (2, 3)):
        assert outs[a][1] == outs[b][1]
        np.testing.assert_array_equal(outs[a][2], outs[b][2])
