/*
 * mgr.h — C ABI of libmgr: GMRES preconditioned by multigrid reduction (MGR)
 * for block-structured, indefinite Jacobians, on one AMD Instinct MI355X
 * (gfx950).  Method: Bui, Wang, Osei-Kuffuor, "Algebraic Multigrid
 * Preconditioners for Multiphase Flow in Porous Media with Phase Transitions"
 * (arXiv:1801.08464).
 *
 * The linear problem (paper Section 3.2, eq. linear_system, and its split form
 * eq. 2p2c_matrix): solve A u = f with A of size n = block_size * N,
 * non-symmetric and indefinite, where some constraint rows have a zero
 * diagonal so that plain AMG does not apply.  The preconditioner is the MGR
 * V-cycle of Section 4 (algorithm "MGR preconditioner with presmoothing":
 * global block relaxation, F-relaxation, coarse-grid correction with
 * P = [W_p; I], R = [W_r, I] of eq. RPoperator1 and the choices of eqs.
 * injective_rp / non_injective_rp), recursed over the reduction levels of
 * Section 5, with a classical AMG V-cycle on the last (pressure-like) level.
 *
 * Conventions for every entry point:
 *  - Array arguments are DEVICE pointers unless the comment says "host".
 *  - Work is enqueued on mgr_options.stream (a hipStream_t; NULL = the null
 *    stream).  Entry points that return sizes or status synchronise it.
 *  - Matrices are CSR with int32 row pointers and column indices, columns
 *    strictly ascending within each row, no duplicates, FP64 values.  An
 *    absent entry is a structural zero (the zero diagonal of a constraint row
 *    is absent).
 *  - Unknowns of one cell are contiguous: u = block_size * c + v.
 *  - Return value: MGR_OK (0), MGR_NOT_CONVERGED (1) or a negative error code.
 *    The detail of the last error of a handle (offending row, level) is in
 *    mgr_last_error(); errors raised before a handle exists are in
 *    mgr_last_error(NULL) (per thread).
 *  - A handle is not thread safe; distinct handles are independent.
 */
#ifndef MGR_H
#define MGR_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MGR_OK = 0,
    MGR_NOT_CONVERGED = 1,    /* max_iter reached; x holds the last iterate, stats are valid */
    MGR_E_INVALID = -1,       /* bad sizes, block size, labels, pattern or option */
    MGR_E_ZERO_FDIAG = -2,    /* an F-point has a zero/absent diagonal at its level */
    MGR_E_SINGULAR_BLOCK = -3,/* singular cell block, empty AMG row or singular coarsest matrix */
    MGR_E_BREAKDOWN = -4,     /* NaN/Inf in the right-hand side or in the Krylov recurrence */
    MGR_E_HIP = -5,           /* a HIP runtime call failed */
    MGR_E_OOM = -6            /* device allocation failed */
};

typedef struct mgr_handle mgr_handle;

/* CSR matrix view (device pointers, not copied until mgr_setup). */
typedef struct {
    int64_t n;                /* rows = columns */
    int64_t nnz;
    const int32_t *row_ptr;   /* n + 1 */
    const int32_t *col_idx;   /* nnz */
    const double *values;     /* nnz */
} mgr_csr;

typedef struct {
    void *stream;             /* hipStream_t */
    int precision;            /* 0: FP64 hierarchy; 1: mixed (FP32 hierarchy inside FP64 flexible GMRES) */
    int restart;              /* GMRES restart length m (1..64), default 30 */
    int max_iter;             /* total Arnoldi steps, default 400 */
    int rp_type;              /* 0 non-injective W_r = -A_CF D_FF^{-1} (default), 1 injective W_r = 0,
                                 2 block factorization W_p = 0 (paper Section 4, last paragraph) */
    int global_relax;         /* 1: level-0 block-Jacobi with the block_size x block_size cell blocks */
    int f_sweeps;             /* Jacobi F-relaxation sweeps per MGR level (0..8), default 1 */
    double amg_theta;         /* strength threshold, default 0.25 */
    int amg_pre, amg_post;    /* l1-Jacobi sweeps, default 2, 2 */
    int amg_max_levels;       /* default 25 (max 32) */
    int amg_coarse_max;       /* stop coarsening at n <= this, default 64 */
    int dense_max;            /* largest coarsest level solved by dense LU, default and max 4096 */
    uint64_t pmis_seed;       /* hash seed of the PMIS tie-breaking keys, default 0 */
    int transpose;            /* 1: build the hierarchy on A^T (adjoint solves) */
    int use_x0;               /* 1: mgr_solve starts from the x passed in */
    int frelax_amg_mask;      /* bit l set: MGR level l relaxes its F-points with one AMG V-cycle on A_FF
                                 (the paper's F-relaxation of its phase-transition runs, Section 6.2)
                                 instead of Jacobi; default 0 */
    int frelax_amg_pre, frelax_amg_post;  /* smoothing sweeps of that V-cycle, default 1, 1 */
    int cycle_post;           /* 0: pre-smoothing form eq. MGR-pre (Section 4 algorithm "MGR preconditioner
                                 with presmoothing", default); 1: post-smoothing form eq. MGR-post: the
                                 coarse-grid correction from e = 0 first, then the same smoother M_f as
                                 the pre-smoothing form: (level 0) the global relaxation, then F-relaxation */
    int index16;              /* column storage of the solve-phase copies (no effect on results, which are
                                 bitwise the same either way): 1 (default) 16-bit column offsets from a 32-bit
                                 base per slot where every offset of the matrix fits (else 32-bit columns),
                                 in the level-0 operator's sliced ELL and in the long-row level-0 matrix of
                                 each mixed-precision AMG hierarchy; 0 32-bit columns everywhere */
} mgr_options;

typedef struct {
    int iterations;           /* Arnoldi steps = preconditioner applications */
    double rel_residual;      /* ||b - A x||_2 / ||b||_2 at exit (true residual) */
    double setup_ms, solve_ms;
    int n_levels;             /* MGR levels + AMG levels */
    int64_t level_n[64], level_nnz[64];
    double *res_history;      /* host buffer (may be NULL): |g_{j+1}| / ||b|| per iteration */
    int res_history_cap;
    int res_history_len;
} mgr_stats;

/* Fill *opts with the defaults listed above (stream = NULL). */
void mgr_default_options(mgr_options *opts);

/*
 * Build the hierarchy (all on the GPU).
 *  A          : the n x n matrix (device CSR).  Copied; the caller may free it
 *               once the stream has passed this call.
 *  block_size : 1 or 3 (unknowns per cell; 3 = (p, rho, S) of the paper's
 *               two-phase two-component model).  n % block_size == 0.
 *  cf_labels  : device int32[n].  cf_labels[u] = l means u is an F-point of
 *               reduction level l and is eliminated there (paper Section 5:
 *               level 0 the constraint rows with a nonzero diagonal, C_33;
 *               level 1 the second PDE variable; level 2 the remaining
 *               constraints).  L = max label is the final coarse grid, solved
 *               by AMG; L = 0 gives plain AMG on A.  0 <= label <= 31.
 *  out        : receives the handle, or NULL on failure.
 * Errors: MGR_E_INVALID, MGR_E_ZERO_FDIAG (mgr_last_error names the level,
 * level-local row and global unknown), MGR_E_SINGULAR_BLOCK, MGR_E_HIP, MGR_E_OOM.
 */
int mgr_setup(const mgr_csr *A, int block_size, const int32_t *cf_labels, const mgr_options *opts,
              mgr_handle **out);

/*
 * New values on the handle's matrix, with the pattern and cf_labels of its
 * setup unchanged (the semi-smooth Newton iteration of Section 3.1 between
 * steps whose active set, and so the Jacobian's pattern, did not change).
 * Only the values are redone: D_FF^{-1}, W_p and W_r, the reduced operators
 * A_{l+1} = R_l A_l P_l written over their arrays, the cell-block inverses, and
 * the AMG hierarchies, rebuilt because their coarsening depends on the values.
 * The pattern checks, level maps, sparsity patterns and Krylov workspace of the
 * setup are kept.  The result is bitwise the one a new mgr_setup with these
 * values would give.
 *  values : device double[nnz] in the order of the setup's col_idx (copied).
 * Errors: MGR_E_INVALID, MGR_E_ZERO_FDIAG, MGR_E_SINGULAR_BLOCK, MGR_E_HIP,
 * MGR_E_OOM.  After an error the handle's hierarchy is incomplete: destroy it.
 * The caller keeps the pattern unchanged; nothing checks it.
 */
int mgr_update_values(mgr_handle *h, const double *values);

/*
 * Solve A x = b (or A^T x = b for a transpose handle) to
 * ||b - A x|| <= tol ||b|| with restarted GMRES(m) right-preconditioned by the
 * MGR V-cycle: the linear solve of each semi-smooth Newton step (Section 3.1),
 * with the tolerance relative to the right-hand side and the iteration cap of
 * the experiments of Section 6 (the paper uses the simulator's GMRES, the method
 * its introduction cites; here the preconditioned directions are kept, x += Z y,
 * which also serves the mixed-precision form as flexible GMRES).
 * b: device double[n] (read only).  x: device double[n] (output; also the
 * initial guess when use_x0).  stats may be NULL.
 * Returns MGR_OK, MGR_NOT_CONVERGED or MGR_E_BREAKDOWN.  ||b|| = 0 gives x = 0.
 */
int mgr_solve(mgr_handle *h, const double *b, double *x, double tol, mgr_stats *stats);

/*
 * Gradient of a loss L(x), x = A^{-1} b (the linear system of Section 3.2), with
 * respect to the stored values of the matrix given to mgr_setup (the adjoint
 * form of the solve): dvals[k] = -lambda[row(k)] * x[col(k)] for
 * each stored entry k, where lambda = A^{-T} dL/dx (from a transpose handle).
 * lambda, x: device double[n]; dvals: device double[nnz].  The pattern is the
 * one passed to mgr_setup of this handle (before any transposition).
 */
int mgr_pattern_outer(mgr_handle *h, const double *lambda, const double *x, double *dvals);

/* One application of the preconditioner, z = M^{-1} r (device double[n]).
 * Mixed precision handles round r to FP32 and return the FP32 result widened. */
int mgr_apply_preconditioner(mgr_handle *h, const double *r, double *z);

/* y = A x with the level-0 operator of the handle (A^T for a transpose handle). */
int mgr_spmv(mgr_handle *h, const double *x, double *y);

void mgr_destroy(mgr_handle *h);
const char *mgr_status_string(int code);
const char *mgr_last_error(const mgr_handle *h);

/* ---- introspection (tests, diagnostics; synchronises the stream) ---- */
int mgr_num_levels(mgr_handle *h, int *n_mgr_levels, int *n_amg_levels);

/*
 * Copy one hierarchy matrix to HOST memory.  kind: 0 MGR A_l, 1 MGR P_l,
 * 2 MGR R_l, 3 AMG A_k, 4 AMG P_k, 5 AMG strength pattern S_k (values unset),
 * 6 / 7: A_k / P_k of the F-relaxation AMG of MGR level l, with level = (l << 8) | k.
 * Call with row_ptr == NULL to get the sizes only.  Host arrays: row_ptr
 * int32[nrows + 1], col_idx int32[nnz], values double[nnz] (may be NULL).
 */
int mgr_get_matrix(mgr_handle *h, int kind, int level, int64_t *nrows, int64_t *ncols, int64_t *nnz,
                   int32_t *row_ptr, int32_t *col_idx, double *values);

/*
 * Copy one hierarchy vector to HOST memory.  kind: 0 cell-block inverses
 * (double, 9 per cell, row-major), 1 MGR dinv_l (double), 2 MGR F list_l
 * (int32, level-local indices), 3 MGR C list_l (int32), 4 AMG C/F marker_k
 * (int32, +1 C / -1 F), 5 AMG l1 row norms_k (double), 6 coarsest LU factors
 * (double n*n row-major, unit-lower L below the diagonal), 7 coarsest LU row
 * permutation (int32); 8..11: kinds 4..7 for the F-relaxation AMG of MGR level
 * l, with level = (l << 8) | k.  out == NULL returns the length only in *len.
 */
int mgr_get_vector(mgr_handle *h, int kind, int level, void *out, int64_t *len);

/*
 * Kernel timing: when on, every launch of the level-0 sliced-ELL SpMV /
 * residual kernel, every l1-Jacobi sweep on the coarse-grid matrix (level 0 of
 * the coarse AMG hierarchy), and every whole preconditioner application (the MGR
 * V-cycle of Section 4, algorithm "MGR preconditioner with presmoothing", inside mgr_solve or
 * mgr_apply_preconditioner), is timed by HIP events on the handle's stream: the
 * two kernels' launches record their own start and end events
 * (hipExtLaunchKernelGGL), so each interval is the kernel's execution alone;
 * an application is bracketed by events recorded before and after it.
 * mgr_kernel_time (synchronises) returns the summed event time, the number of
 * launches and the summed algorithmic bytes of those launches, then resets the
 * counters.  kernel: 0 = the level-0 kernel (bytes: stored values and column
 * indices of the true nonzeros, row pointers, x, y and r when read); 1 = the
 * V-cycle (bytes: the sum over its launches of every array each reads or
 * writes, counted once per launch, with gathered vectors at their length);
 * 2 = the coarse-grid sweeps (bytes: stored values and column indices, row
 * pointers, the gathered x, and r, d and y).  Returns MGR_E_INVALID for another
 * kernel id.
 */
int mgr_set_kernel_timing(mgr_handle *h, int on);
int mgr_kernel_time(mgr_handle *h, int kernel, double *total_ms, int64_t *launches, double *bytes_total);

/*
 * Semi-smooth Newton support (Section 3.1, algorithm "Semi-smooth Newton Method")
 * for the complementarity system with block_size 3: unknowns u = (p, rho, S) per
 * cell, u[3c + v].  L (device CSR, n = 3 N rows, int32 indices, FP64 values) holds
 * the two PDE rows of each cell (the residual H(u) = L u - f is linear in u);
 * entries of L in the S rows are ignored.  henry: N values H_c.  The constraint of
 * cell c is Theta_c = min(F_c, G_c), F_c = S_c, G_c = rho_c - H_c p_c.
 *
 * mgr_ncp_eval: if du != NULL, first u += alpha du (step 4); then R = [L u - f on
 * the PDE rows; min(F, G) on the S rows] (step 1's residual) and labels for
 * mgr_setup: 3 for p, 1 for rho, and for S 2 on the active set A = {F >= G}
 * (the gas-present rows, zero diagonal) and 0 off it (the three-stage reduction of
 * Section 5).  *rnorm = ||R||_2, *nactive = |A|, *nchanged = the number of cells
 * whose labels differ from what the labels array held before the call (0: the
 * Jacobian keeps its pattern, and mgr_update_values may replace a new setup);
 * host outputs, each may be NULL.  All
 * arrays are caller-owned device memory of length n (henry: N); ordered on stream
 * (a hipStream_t); synchronises before returning.  Errors: MGR_E_INVALID (bad CSR
 * or null array), MGR_E_BREAKDOWN (non-finite residual), MGR_E_HIP, MGR_E_OOM.
 *
 * mgr_ncp_jacobian: the generalised Jacobian of step 2 for the given labels: the
 * rows of L, and per cell the constraint row [-H_c, 1] at (p, rho) if its S label
 * is 2, [1] at S otherwise, columns ascending.  Writes row_ptr (n + 1, device),
 * col_idx / values (device, capacity entries) and *nnz (host).  If the Jacobian
 * needs more than capacity entries, returns MGR_E_INVALID with *nnz set and
 * row_ptr written, col_idx / values untouched; capacity nnz(L) + 2 N always
 * suffices.  Ordered on stream; synchronises before returning.
 */
int mgr_ncp_eval(const mgr_csr *L, const double *henry, const double *f, double *u, const double *du, double alpha,
                 double *R, int32_t *labels, double *rnorm, int64_t *nactive, int64_t *nchanged, void *stream);
int mgr_ncp_jacobian(const mgr_csr *L, const double *henry, const int32_t *labels, int32_t *row_ptr,
                     int32_t *col_idx, double *values, int64_t capacity, int64_t *nnz, void *stream);

/*
 * mgr_ncp_eval_noalloc: mgr_ncp_eval for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and errors as mgr_ncp_eval; it
 * calls no hipMalloc, hipFree or allocating library routine.  Its device scratch
 * (the residual norm's partial sums, the norm and the two cell counters) is a
 * file-scope device array of 16 KiB that each GPU the library runs on holds
 * until the process ends; the need is (blocks of the norm reduction + 1)
 * doubles and two ints (at most 8,208 bytes with the library's reduction grid,
 * whatever n), and a call that would need more returns MGR_E_INVALID with the
 * sizes in mgr_last_error(NULL).  The counters are cleared by a kernel on every
 * call.  All calls on one GPU share that array: calls that overlap on one GPU
 * (different streams, or threads) race and must be serialised by the caller.
 */
int mgr_ncp_eval_noalloc(const mgr_csr *L, const double *henry, const double *f, double *u, const double *du,
                         double alpha, double *R, int32_t *labels, double *rnorm, int64_t *nactive,
                         int64_t *nchanged, void *stream);

#ifdef __cplusplus
}
#endif
#endif
