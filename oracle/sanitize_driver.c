/*
 * Standalone driver of the oracle for the host sanitizers (AddressSanitizer and
 * UndefinedBehaviorSanitizer).  TEST INFRASTRUCTURE ONLY: it exercises every
 * oracle entry point on one system read from a file and is built and run by
 * the CPU test suite with -fsanitize=address,undefined.
 *
 * Input file (little endian): int64 n, int64 nnz, int32 block_size, then
 * rp[n+1] (int64), ci[nnz] (int32), v[nnz] (float64), labels[n] (int32),
 * b[n] (float64).
 *
 * For each option set it builds the hierarchy, solves, applies one V-cycle,
 * reads every matrix and vector the introspection calls expose and destroys
 * the handle; it also runs the sparse building blocks on the fine matrix.
 * Exit status 0 when every call returned what it should.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            exit(2);                                                      \
        }                                                                 \
    } while (0)

static void *read_all(FILE *f, size_t bytes) {
    void *p = malloc(bytes ? bytes : 1);
    CHECK(p && fread(p, 1, bytes, f) == bytes);
    return p;
}

static void touch_hierarchy(orc_handle *h) {
    int L = orc_num_mgr_levels(h), K = orc_num_amg_levels(h);
    orc_mat m;
    for (int l = 0; l < L; l++) {
        for (int kind = 0; kind < 3; kind++) CHECK(orc_get_mat(h, kind, l, &m) == ORC_OK);
        int nff = orc_num_ff_levels(h, l);
        for (int k = 0; k < nff; k++) {
            CHECK(orc_get_mat(h, 6, (l << 8) | k, &m) == ORC_OK);
            if (k < nff - 1) CHECK(orc_get_mat(h, 7, (l << 8) | k, &m) == ORC_OK);
        }
    }
    CHECK(orc_get_mat(h, 0, L, &m) == ORC_E_INVALID);
    for (int k = 0; k < K; k++) {
        CHECK(orc_get_mat(h, 3, k, &m) == ORC_OK);
        if (k < K - 1) {
            CHECK(orc_get_mat(h, 4, k, &m) == ORC_OK);
            CHECK(orc_get_mat(h, 5, k, &m) == ORC_OK);
        }
    }
    for (int kind = 0; kind < 12; kind++) {
        int hi = kind <= 3 ? L : 8;
        for (int l = 0; l < hi; l++) {
            int nsub = kind >= 8 ? orc_num_ff_levels(h, l) : (kind >= 4 ? K : 1);
            for (int k = 0; k < nsub; k++) {
                int level = kind >= 8 ? ((l << 8) | k) : (kind >= 4 ? k : l);
                int64_t len = orc_get_vec_len(h, kind, level);
                if (len <= 0) continue;
                size_t elem = (kind == 2 || kind == 3 || kind == 4 || kind == 7 || kind == 8 || kind == 11)
                                  ? sizeof(int32_t) : sizeof(double);
                void *buf = malloc((size_t)len * elem);
                CHECK(buf && orc_get_vec(h, kind, level, buf) == ORC_OK);
                free(buf);
            }
            if (kind >= 4 && kind < 8) break;
        }
    }
}

static void building_blocks(const orc_mat *A, const double *b) {
    double *y = malloc((size_t)A->nrows * sizeof(double));
    CHECK(y && orc_spmv(A, b, y) == ORC_OK);
    orc_mat AT = {0}, AA = {0}, S = {0}, P = {0};
    CHECK(orc_transpose(A, &AT) == ORC_OK);
    CHECK(orc_spgemm(A, &AT, &AA) == ORC_OK);
    CHECK(orc_strength(A, 0.25, &S) == ORC_OK);
    int32_t *cf = malloc((size_t)A->nrows * sizeof(int32_t));
    CHECK(cf && orc_pmis(&S, 7, cf) == ORC_OK);
    CHECK(orc_interp(A, &S, cf, &P) == ORC_OK);
    enum { N = 5 };
    double lu[N * N], x[N], rhs[N];
    int32_t perm[N];
    for (int i = 0; i < N; i++) {
        rhs[i] = i + 1;
        for (int j = 0; j < N; j++) lu[i * N + j] = (i == j) ? 4.0 : 1.0 / (1 + i + 2 * j);
    }
    CHECK(orc_dense_lu(N, lu, perm) == ORC_OK);
    orc_dense_lu_solve(N, lu, perm, rhs, x);
    free(cf); free(y);
    orc_mat_free(&AT); orc_mat_free(&AA); orc_mat_free(&S); orc_mat_free(&P);
}

int main(int argc, char **argv) {
    CHECK(argc == 2);
    FILE *f = fopen(argv[1], "rb");
    CHECK(f);
    int64_t n, nnz;
    int32_t bs;
    CHECK(fread(&n, 8, 1, f) == 1 && fread(&nnz, 8, 1, f) == 1 && fread(&bs, 4, 1, f) == 1);
    CHECK(n > 0 && nnz > 0 && n % bs == 0);
    orc_mat A = {n, n, nnz, NULL, NULL, NULL};
    A.rp = read_all(f, (size_t)(n + 1) * 8);
    A.ci = read_all(f, (size_t)nnz * 4);
    A.v = read_all(f, (size_t)nnz * 8);
    int32_t *labels = read_all(f, (size_t)n * 4);
    double *b = read_all(f, (size_t)n * 8);
    fclose(f);

    building_blocks(&A, b);

    /* option sets: defaults, each interpolation/restriction form, the FP32
     * hierarchy, F-relaxation by AMG on every level with the post-smoothing
     * cycle, and a deep AMG hierarchy with a one-row dense coarse solve */
    enum { NSETS = 6 };
    double *x = malloc((size_t)n * sizeof(double)), *e = malloc((size_t)n * sizeof(double));
    double hist[64];
    CHECK(x && e);
    for (int s = 0; s < NSETS; s++) {
        orc_opts o;
        orc_default_opts(&o);
        o.max_iter = 60;
        if (s == 1) o.rp_type = 1;
        if (s == 2) o.rp_type = 2;
        if (s == 3) o.precision = 1;
        if (s == 4) { o.frelax_amg_mask = 7; o.cycle_post = 1; o.use_x0 = 1; }
        if (s == 5) { o.amg_coarse_max = 1; o.restart = 5; o.global_relax = 0; }
        orc_handle *h = NULL;
        char err[256];
        int rc = orc_setup(&A, bs, labels, &o, &h, err, sizeof err);
        if (rc != ORC_OK) {
            fprintf(stderr, "set %d: setup %d (%s)\n", s, rc, err);
            return 3;
        }
        touch_hierarchy(h);
        for (int64_t i = 0; i < n; i++) x[i] = s == 4 ? 0.5 : 0.0;
        orc_stats st;
        memset(&st, 0, sizeof st);
        st.res_history = hist;
        st.res_history_cap = 64;
        rc = orc_solve(h, b, x, 1e-8, &st);
        fprintf(stderr, "set %d: status %d, %d iterations, rel %.3e, %d levels\n", s, rc, st.iterations,
                st.rel_residual, st.n_levels);
        CHECK(rc == ORC_OK || rc == ORC_NOT_CONVERGED);
        CHECK(orc_vcycle(h, b, e) == ORC_OK);
        CHECK(orc_destroy(h) == ORC_OK);
    }
    /* a negative label is rejected */
    labels[0] = -1;
    orc_opts o;
    orc_default_opts(&o);
    orc_handle *h = NULL;
    char err[256];
    CHECK(orc_setup(&A, bs, labels, &o, &h, err, sizeof err) != ORC_OK && h == NULL);

    free(x); free(e); free(labels); free(b);
    free(A.rp); free(A.ci); free(A.v);
    return 0;
}
