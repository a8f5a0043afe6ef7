/*
 * Oracle sparse building blocks: SpMV, stable transpose and Gustavson SpGEMM.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Canonical evaluation order (the paper builds every coarse operator as the
 * product R (A P), Section 4, eq. RPoperator1 and the Schur complements of
 * Section 5): every output entry C_ij = sum_k A_ik B_kj is accumulated from
 * 0.0 in ascending k, each product rounded once, and no entry is ever
 * dropped, so the output pattern depends on the input patterns only.
 */
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

void orc_mat_free(orc_mat *m) {
    if (!m) return;
    free(m->rp);
    free(m->ci);
    free(m->v);
    m->rp = NULL;
    m->ci = NULL;
    m->v = NULL;
    m->nrows = m->ncols = m->nnz = 0;
}

/* y = A x, each row summed left to right in ascending column order. */
int orc_spmv(const orc_mat *A, const double *x, double *y) {
    for (int64_t i = 0; i < A->nrows; ++i) {
        double s = 0.0;
        for (int64_t p = A->rp[i]; p < A->rp[i + 1]; ++p) s += A->v[p] * x[A->ci[p]];
        y[i] = s;
    }
    return ORC_OK;
}

/* A^T with each output row listing the source rows in ascending order. */
int orc_transpose(const orc_mat *A, orc_mat *AT) {
    AT->nrows = A->ncols;
    AT->ncols = A->nrows;
    AT->nnz = A->nnz;
    AT->rp = (int64_t *)calloc((size_t)AT->nrows + 1, sizeof(int64_t));
    AT->ci = (int32_t *)malloc((size_t)(A->nnz > 0 ? A->nnz : 1) * sizeof(int32_t));
    AT->v = A->v ? (double *)malloc((size_t)(A->nnz > 0 ? A->nnz : 1) * sizeof(double)) : NULL;
    for (int64_t p = 0; p < A->nnz; ++p) AT->rp[A->ci[p] + 1]++;
    for (int64_t j = 0; j < AT->nrows; ++j) AT->rp[j + 1] += AT->rp[j];
    int64_t *next = (int64_t *)malloc((size_t)(AT->nrows > 0 ? AT->nrows : 1) * sizeof(int64_t));
    for (int64_t j = 0; j < AT->nrows; ++j) next[j] = AT->rp[j];
    for (int64_t i = 0; i < A->nrows; ++i) {
        for (int64_t p = A->rp[i]; p < A->rp[i + 1]; ++p) {
            int64_t q = next[A->ci[p]]++;
            AT->ci[q] = (int32_t)i;
            if (A->v) AT->v[q] = A->v[p];
        }
    }
    free(next);
    return ORC_OK;
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* C = A B (Gustavson, row by row, dense accumulator). */
int orc_spgemm(const orc_mat *A, const orc_mat *B, orc_mat *C) {
    if (A->ncols != B->nrows) return ORC_E_INVALID;
    int64_t m = A->nrows, ncol = B->ncols;
    int64_t *mark = (int64_t *)malloc((size_t)(ncol > 0 ? ncol : 1) * sizeof(int64_t));
    double *acc = (double *)malloc((size_t)(ncol > 0 ? ncol : 1) * sizeof(double));
    int32_t *cols = (int32_t *)malloc((size_t)(ncol > 0 ? ncol : 1) * sizeof(int32_t));
    for (int64_t j = 0; j < ncol; ++j) mark[j] = -1;

    /* symbolic pass: row lengths */
    C->nrows = m;
    C->ncols = ncol;
    C->rp = (int64_t *)calloc((size_t)m + 1, sizeof(int64_t));
    for (int64_t i = 0; i < m; ++i) {
        int64_t cnt = 0;
        for (int64_t p = A->rp[i]; p < A->rp[i + 1]; ++p) {
            int32_t k = A->ci[p];
            for (int64_t q = B->rp[k]; q < B->rp[k + 1]; ++q) {
                int32_t j = B->ci[q];
                if (mark[j] != i) {
                    mark[j] = i;
                    cnt++;
                }
            }
        }
        C->rp[i + 1] = C->rp[i] + cnt;
    }
    C->nnz = C->rp[m];
    C->ci = (int32_t *)malloc((size_t)(C->nnz > 0 ? C->nnz : 1) * sizeof(int32_t));
    C->v = (double *)malloc((size_t)(C->nnz > 0 ? C->nnz : 1) * sizeof(double));
    for (int64_t j = 0; j < ncol; ++j) mark[j] = -1;

    /* numeric pass: ascending k, acc starts at 0.0 */
    for (int64_t i = 0; i < m; ++i) {
        int64_t cnt = 0;
        for (int64_t p = A->rp[i]; p < A->rp[i + 1]; ++p) {
            int32_t k = A->ci[p];
            double a = A->v[p];
            for (int64_t q = B->rp[k]; q < B->rp[k + 1]; ++q) {
                int32_t j = B->ci[q];
                if (mark[j] != i) {
                    mark[j] = i;
                    acc[j] = 0.0;
                    cols[cnt++] = j;
                }
                double prod = a * B->v[q];
                acc[j] = acc[j] + prod;
            }
        }
        qsort(cols, (size_t)cnt, sizeof(int32_t), cmp_i32);
        int64_t base = C->rp[i];
        for (int64_t t = 0; t < cnt; ++t) {
            C->ci[base + t] = cols[t];
            C->v[base + t] = acc[cols[t]];
        }
    }
    free(mark);
    free(acc);
    free(cols);
    return ORC_OK;
}

/* dL/dvals_k = -lambda_row(k) * x_col(k): the gradient of L(x) with x = A^{-1} b
 * with respect to the stored values of A, given lambda = A^{-T} dL/dx. */
int orc_pattern_outer(const orc_mat *A, const double *lambda, const double *x, double *dvals) {
    for (int64_t i = 0; i < A->nrows; ++i)
        for (int64_t p = A->rp[i]; p < A->rp[i + 1]; ++p) dvals[p] = -(lambda[i] * x[A->ci[p]]);
    return ORC_OK;
}
