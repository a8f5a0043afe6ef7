/*
 * Oracle pieces of the classical AMG used as the coarse-grid solver M_c^{-1}
 * (the paper's Section 4, step (3) of the MGR algorithm with presmoothing, and
 * Section 6: BoomerAMG with classical Ruge-Stueben interpolation).  CLJP
 * coarsening is replaced by PMIS (De Sterck, Yang, Heys 2006) with hashed
 * tie-breaking keys, and the hybrid Gauss-Seidel smoother by l1-Jacobi
 * (Baker, Falgout, Kolev, Yang 2011); both are readings recorded with the
 * method's definition.  Also the 3x3 cell-block inverse of the global
 * relaxation (step (1) of the same algorithm, M = blockdiag(A)) and the dense
 * LU of the coarsest level.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

/* SplitMix64 output function (Steele, Lea, Flood 2014). */
uint64_t orc_splitmix64(uint64_t x) {
    uint64_t z = x + 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static double diag_of(const orc_mat *A, int64_t i) {
    for (int64_t p = A->rp[i]; p < A->rp[i + 1]; ++p)
        if (A->ci[p] == i) return A->v[p];
    return 0.0;
}

/* Classical strength of connection with the sign of the diagonal:
 * j in S_i  iff  j != i, m_i > 0 and -s_i a_ij >= theta m_i,
 * where s_i = +1 if a_ii >= 0 else -1 and m_i = max_{j != i} (-s_i a_ij). */
int orc_strength(const orc_mat *A, double theta, orc_mat *S) {
    int64_t n = A->nrows;
    S->nrows = n;
    S->ncols = A->ncols;
    S->rp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    S->ci = (int32_t *)malloc((size_t)(A->nnz > 0 ? A->nnz : 1) * sizeof(int32_t));
    S->v = NULL;
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i) {
        double d = diag_of(A, i);
        int pos = d >= 0.0;
        double m = -INFINITY;
        for (int64_t p = A->rp[i]; p < A->rp[i + 1]; ++p) {
            if (A->ci[p] == i) continue;
            double t = pos ? -A->v[p] : A->v[p];
            if (t > m) m = t;
        }
        if (m > 0.0) {
            double thr = theta * m;
            for (int64_t p = A->rp[i]; p < A->rp[i + 1]; ++p) {
                if (A->ci[p] == i) continue;
                double t = pos ? -A->v[p] : A->v[p];
                if (t >= thr) S->ci[cnt++] = A->ci[p];
            }
        }
        S->rp[i + 1] = cnt;
    }
    S->nnz = cnt;
    return ORC_OK;
}

/* PMIS key order: (lambda, hash, index) compared lexicographically. */
static int key_greater(int64_t i, int64_t j, const int64_t *lam, const uint64_t *h) {
    if (lam[i] != lam[j]) return lam[i] > lam[j];
    if (h[i] != h[j]) return h[i] > h[j];
    return i > j;
}

/* Parallel modified independent set coarsening in synchronous rounds.
 * cf[i] = +1 (C) or -1 (F). */
int orc_pmis(const orc_mat *S, uint64_t seed, int32_t *cf) {
    int64_t n = S->nrows;
    orc_mat ST;
    orc_transpose(S, &ST);
    int64_t *lam = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    uint64_t *h = (uint64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint64_t));
    char *newc = (char *)malloc((size_t)(n > 0 ? n : 1));
    int64_t undecided = 0;
    for (int64_t i = 0; i < n; ++i) {
        lam[i] = ST.rp[i + 1] - ST.rp[i];      /* |{j : i in S_j}| */
        h[i] = orc_splitmix64(seed ^ (uint64_t)i);
        cf[i] = lam[i] == 0 ? -1 : 0;
        if (cf[i] == 0) undecided++;
    }
    while (undecided > 0) {
        int64_t made = 0;
        for (int64_t i = 0; i < n; ++i) {
            newc[i] = 0;
            if (cf[i] != 0) continue;
            int ok = 1;
            for (int64_t p = S->rp[i]; p < S->rp[i + 1] && ok; ++p) {
                int64_t j = S->ci[p];
                if (cf[j] == 0 && !key_greater(i, j, lam, h)) ok = 0;
            }
            for (int64_t p = ST.rp[i]; p < ST.rp[i + 1] && ok; ++p) {
                int64_t j = ST.ci[p];
                if (cf[j] == 0 && !key_greater(i, j, lam, h)) ok = 0;
            }
            newc[i] = (char)ok;
        }
        for (int64_t i = 0; i < n; ++i)
            if (newc[i]) {
                cf[i] = 1;
                made++;
            }
        for (int64_t j = 0; j < n; ++j) {
            if (cf[j] != 0) continue;
            for (int64_t p = S->rp[j]; p < S->rp[j + 1]; ++p)
                if (newc[S->ci[p]]) {
                    cf[j] = -1;
                    break;
                }
        }
        undecided = 0;
        for (int64_t i = 0; i < n; ++i)
            if (cf[i] == 0) undecided++;
        if (made == 0) { /* cannot happen: the largest undecided key always wins */
            free(lam); free(h); free(newc); orc_mat_free(&ST);
            return ORC_E_INVALID;
        }
    }
    free(lam);
    free(h);
    free(newc);
    orc_mat_free(&ST);
    return ORC_OK;
}

/* Classical (Ruge-Stueben) interpolation with the sign-filtered distance-two
 * terms and weak connections lumped into the diagonal.  For F-point i:
 *   C_i = S_i cap C, F_i = S_i cap F, W_i = other off-diagonal entries;
 *   atil = a_ii + sum_{n in W_i} a_in;
 *   for k in F_i ascending: den = sum_{m in C_i} abar_km
 *     (abar_km = a_km if a_km * a_kk < 0, else 0);
 *     den == 0 -> atil += a_ik, else num_j += (a_ik * abar_kj) / den;
 *   w_ij = -((a_ij + num_j) / atil)  (all zero if atil == 0).
 * C rows are unit rows; coarse points are numbered in ascending fine index. */
int orc_interp(const orc_mat *A, const orc_mat *S, const int32_t *cf, orc_mat *P) {
    int64_t n = A->nrows;
    int64_t *cmap = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t nc = 0;
    for (int64_t i = 0; i < n; ++i) cmap[i] = cf[i] == 1 ? nc++ : -1;
    /* strong flag per entry of A */
    char *strong = (char *)calloc((size_t)(A->nnz > 0 ? A->nnz : 1), 1);
    for (int64_t i = 0; i < n; ++i) {
        int64_t q = S->rp[i];
        for (int64_t p = A->rp[i]; p < A->rp[i + 1]; ++p) {
            while (q < S->rp[i + 1] && S->ci[q] < A->ci[p]) q++;
            if (q < S->rp[i + 1] && S->ci[q] == A->ci[p]) strong[p] = 1;
        }
    }
    P->nrows = n;
    P->ncols = nc;
    P->rp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
        int64_t cnt = 0;
        if (cf[i] == 1) cnt = 1;
        else
            for (int64_t p = A->rp[i]; p < A->rp[i + 1]; ++p)
                if (strong[p] && cf[A->ci[p]] == 1) cnt++;
        P->rp[i + 1] = P->rp[i] + cnt;
    }
    P->nnz = P->rp[n];
    P->ci = (int32_t *)malloc((size_t)(P->nnz > 0 ? P->nnz : 1) * sizeof(int32_t));
    P->v = (double *)malloc((size_t)(P->nnz > 0 ? P->nnz : 1) * sizeof(double));
    /* marker: position of column j inside the current row's C_i, or -1 */
    int64_t *pos = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    for (int64_t j = 0; j < n; ++j) pos[j] = -1;
    for (int64_t i = 0; i < n; ++i) {
        int64_t base = P->rp[i];
        if (cf[i] == 1) {
            P->ci[base] = (int32_t)cmap[i];
            P->v[base] = 1.0;
            continue;
        }
        int64_t nci = P->rp[i + 1] - base;
        if (nci == 0) continue;
        double *num = P->v + base;
        int64_t t = 0;
        for (int64_t p = A->rp[i]; p < A->rp[i + 1]; ++p) {
            int32_t j = A->ci[p];
            if (strong[p] && cf[j] == 1) {
                pos[j] = t;
                P->ci[base + t] = (int32_t)cmap[j];
                num[t] = 0.0;
                t++;
            }
        }
        double atil = diag_of(A, i);
        for (int64_t p = A->rp[i]; p < A->rp[i + 1]; ++p) {
            if (A->ci[p] == i) continue;
            if (!strong[p]) atil = atil + A->v[p];
        }
        for (int64_t p = A->rp[i]; p < A->rp[i + 1]; ++p) {
            int32_t k = A->ci[p];
            if (k == i || !strong[p] || cf[k] != -1) continue;
            double aik = A->v[p];
            double akk = diag_of(A, k);
            double den = 0.0;
            for (int64_t q = A->rp[k]; q < A->rp[k + 1]; ++q) {
                int32_t m = A->ci[q];
                if (pos[m] < 0) continue;
                double akm = A->v[q];
                double abar = (akm * akk < 0.0) ? akm : 0.0;
                den = den + abar;
            }
            if (den == 0.0) {
                atil = atil + aik;
            } else {
                for (int64_t q = A->rp[k]; q < A->rp[k + 1]; ++q) {
                    int32_t m = A->ci[q];
                    if (pos[m] < 0) continue;
                    double akm = A->v[q];
                    double abar = (akm * akk < 0.0) ? akm : 0.0;
                    double prod = aik * abar;
                    num[pos[m]] = num[pos[m]] + prod / den;
                }
            }
        }
        t = 0;
        for (int64_t p = A->rp[i]; p < A->rp[i + 1]; ++p) {
            int32_t j = A->ci[p];
            if (!(strong[p] && cf[j] == 1)) continue;
            double s = A->v[p] + num[t];
            num[t] = (atil == 0.0) ? 0.0 : -(s / atil);
            pos[j] = -1;
            t++;
        }
    }
    free(pos);
    free(strong);
    free(cmap);
    return ORC_OK;
}

/* Inverse of each bs x bs diagonal cell block B_c = A[bs c : bs c + bs, same]
 * (structural zeros included).  bs = 3: determinant by cofactor expansion
 * along row 0, inv_ij = cof_ji * (1 / det).  Output: 9 values per cell,
 * row-major.  bs = 1: 1 / a_ii. */
int orc_block_inverse(int64_t ncell, int bs, const orc_mat *A, double *binv) {
    for (int64_t c = 0; c < ncell; ++c) {
        double a[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        for (int r = 0; r < bs; ++r) {
            int64_t i = (int64_t)bs * c + r;
            for (int64_t p = A->rp[i]; p < A->rp[i + 1]; ++p) {
                int64_t j = A->ci[p];
                if (j >= (int64_t)bs * c && j < (int64_t)bs * c + bs) a[r][j - (int64_t)bs * c] = A->v[p];
            }
        }
        if (bs == 1) {
            if (a[0][0] == 0.0) return ORC_E_SINGULAR_BLOCK;
            binv[c] = 1.0 / a[0][0];
            continue;
        }
        double c00 = a[1][1] * a[2][2] - a[1][2] * a[2][1];
        double c01 = -(a[1][0] * a[2][2] - a[1][2] * a[2][0]);
        double c02 = a[1][0] * a[2][1] - a[1][1] * a[2][0];
        double c10 = -(a[0][1] * a[2][2] - a[0][2] * a[2][1]);
        double c11 = a[0][0] * a[2][2] - a[0][2] * a[2][0];
        double c12 = -(a[0][0] * a[2][1] - a[0][1] * a[2][0]);
        double c20 = a[0][1] * a[1][2] - a[0][2] * a[1][1];
        double c21 = -(a[0][0] * a[1][2] - a[0][2] * a[1][0]);
        double c22 = a[0][0] * a[1][1] - a[0][1] * a[1][0];
        double det = a[0][0] * c00 + a[0][1] * c01 + a[0][2] * c02;
        if (det == 0.0 || !isfinite(det)) return ORC_E_SINGULAR_BLOCK;
        double id = 1.0 / det;
        double *o = binv + 9 * c;
        o[0] = c00 * id; o[1] = c10 * id; o[2] = c20 * id;
        o[3] = c01 * id; o[4] = c11 * id; o[5] = c21 * id;
        o[6] = c02 * id; o[7] = c12 * id; o[8] = c22 * id;
    }
    return ORC_OK;
}

/* In-place LU with partial pivoting (first row of largest |a_ik| wins ties). */
int orc_dense_lu(int n, double *a, int32_t *perm) {
    for (int i = 0; i < n; ++i) perm[i] = i;
    for (int k = 0; k < n; ++k) {
        int piv = k;
        double best = fabs(a[(size_t)k * n + k]);
        for (int i = k + 1; i < n; ++i) {
            double t = fabs(a[(size_t)i * n + k]);
            if (t > best) {
                best = t;
                piv = i;
            }
        }
        if (!(best > 0.0)) return ORC_E_SINGULAR_BLOCK;
        if (piv != k) {
            for (int j = 0; j < n; ++j) {
                double t = a[(size_t)k * n + j];
                a[(size_t)k * n + j] = a[(size_t)piv * n + j];
                a[(size_t)piv * n + j] = t;
            }
            int32_t t = perm[k];
            perm[k] = perm[piv];
            perm[piv] = t;
        }
        for (int i = k + 1; i < n; ++i) {
            double l = a[(size_t)i * n + k] / a[(size_t)k * n + k];
            a[(size_t)i * n + k] = l;
            for (int j = k + 1; j < n; ++j) a[(size_t)i * n + j] = a[(size_t)i * n + j] - l * a[(size_t)k * n + j];
        }
    }
    return ORC_OK;
}

void orc_dense_lu_solve(int n, const double *lu, const int32_t *perm, const double *b, double *x) {
    for (int i = 0; i < n; ++i) {
        double s = b[perm[i]];
        for (int j = 0; j < i; ++j) s = s - lu[(size_t)i * n + j] * x[j];
        x[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = x[i];
        for (int j = i + 1; j < n; ++j) s = s - lu[(size_t)i * n + j] * x[j];
        x[i] = s / lu[(size_t)i * n + i];
    }
}
