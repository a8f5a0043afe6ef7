/*
 * Plain CPU oracle for MGR-preconditioned GMRES (Bui, Wang, Osei-Kuffuor,
 * "Algebraic Multigrid Preconditioners for Multiphase Flow in Porous Media
 * with Phase Transitions", arXiv:1801.08464).
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It shares
 * no source, header or helper with the GPU library.
 *
 * Everything is FP64 host arithmetic, single threaded, compiled with
 * -ffp-contract=off so that every product and sum is rounded once.
 * Setup sums run in ascending index order (the canonical order the GPU setup
 * must reproduce bit for bit).
 *
 * Status codes mirror the library's C ABI.
 */
#ifndef MGR_ORACLE_H
#define MGR_ORACLE_H
#include <stdint.h>

#define ORC_OK 0
#define ORC_NOT_CONVERGED 1
#define ORC_E_INVALID (-1)
#define ORC_E_ZERO_FDIAG (-2)
#define ORC_E_SINGULAR_BLOCK (-3)
#define ORC_E_BREAKDOWN (-4)

/* Compressed sparse row matrix; columns sorted within a row, no duplicates.
 * v may be NULL for a pattern-only matrix (strength graph). */
typedef struct {
    int64_t nrows, ncols, nnz;
    int64_t *rp;   /* nrows + 1 */
    int32_t *ci;   /* nnz */
    double *v;     /* nnz or NULL */
} orc_mat;

typedef struct {
    int restart, max_iter;
    int rp_type;          /* 0 non-injective, 1 injective, 2 block factorization (W_p = 0) */
    int global_relax;     /* 1: level-0 block-Jacobi with the cell blocks */
    int f_sweeps;         /* F-relaxation Jacobi sweeps per level */
    double amg_theta;
    int amg_pre, amg_post, amg_max_levels, amg_coarse_max;
    int dense_max;        /* largest coarsest AMG level factored densely */
    uint64_t pmis_seed;
    int precision;        /* 0 FP64 preconditioner, 1 FP32 preconditioner */
    int use_x0;
    int frelax_amg_mask;  /* bit l set: F-relaxation of MGR level l by one AMG V-cycle on A_FF */
    int frelax_amg_pre, frelax_amg_post;
    int cycle_post;       /* 1: post-smoothing form eq. MGR-post (coarse correction, then smoothing) */
} orc_opts;

typedef struct {
    int iterations;
    int status;
    double rel_residual;
    double setup_ms, solve_ms;
    int n_levels;             /* MGR levels + AMG levels */
    int64_t level_n[64], level_nnz[64];
    double *res_history;      /* caller buffer, may be NULL */
    int res_history_cap;
    int res_history_len;
} orc_stats;

typedef struct orc_handle orc_handle;

void orc_default_opts(orc_opts *o);
void orc_mat_free(orc_mat *m);

/* --- sparse building blocks (each pinned by its own tests) --- */
int orc_spmv(const orc_mat *A, const double *x, double *y);
int orc_transpose(const orc_mat *A, orc_mat *AT);
int orc_spgemm(const orc_mat *A, const orc_mat *B, orc_mat *C);
int orc_strength(const orc_mat *A, double theta, orc_mat *S);
int orc_pmis(const orc_mat *S, uint64_t seed, int32_t *cf);
int orc_interp(const orc_mat *A, const orc_mat *S, const int32_t *cf, orc_mat *P);
uint64_t orc_splitmix64(uint64_t x);
int orc_block_inverse(int64_t ncell, int bs, const orc_mat *A, double *binv);
int orc_dense_lu(int n, double *a, int32_t *perm);
void orc_dense_lu_solve(int n, const double *lu, const int32_t *perm, const double *b, double *x);

/* --- the preconditioned solver --- */
int orc_setup(const orc_mat *A, int block_size, const int32_t *labels, const orc_opts *o,
              orc_handle **out, char *err, int errlen);
int orc_solve(orc_handle *h, const double *b, double *x, double tol, orc_stats *st);
int orc_vcycle(orc_handle *h, const double *r, double *e);
int orc_destroy(orc_handle *h);
int orc_pattern_outer(const orc_mat *A, const double *lambda, const double *x, double *dvals);

/* --- introspection of a built hierarchy --- */
int orc_num_mgr_levels(orc_handle *h);
int orc_num_amg_levels(orc_handle *h);
int orc_num_ff_levels(orc_handle *h, int l);
/* kind: 0 MGR A_l, 1 MGR P_l, 2 MGR R_l, 3 AMG A_k, 4 AMG P_k, 5 AMG strength S_k,
 *       6 F-block AMG A_k of MGR level l, 7 its P_k (level argument (l << 8) | k) */
int orc_get_mat(orc_handle *h, int kind, int level, orc_mat *out_view);
/* kind: 0 block inverses (9 per cell), 1 MGR dinv_l, 2 MGR F list_l, 3 MGR C list_l,
 *       4 AMG C/F marker_k (+1 C, -1 F), 5 AMG l1 diagonal_k, 6 coarsest LU (n*n),
 *       7 coarsest LU row permutation; 8..11 the same as 4..7 for the F-block AMG of
 *       MGR level l (level argument (l << 8) | k) */
int64_t orc_get_vec_len(orc_handle *h, int kind, int level);
int orc_get_vec(orc_handle *h, int kind, int level, void *out);

#endif
