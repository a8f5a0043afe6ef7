/*
 * Oracle MGR hierarchy, V-cycle and restarted GMRES.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Setup of reduction level l (paper Section 4, eqs. RPoperator1,
 * injective_rp, non_injective_rp; the three reductions of Section 5):
 *   U_l = {u : label(u) >= l} in ascending global index,
 *   F_l = {label == l}, C_l = {label > l};
 *   dinv_i = 1 / a_ii for i in F (a missing or zero diagonal is an error);
 *   W_p[i,j] = -(a_ij * dinv_i)  (i in F, j in C)   [empty for block factorization]
 *   W_r[i,j] = -(a_ij * dinv_j)  (i in C, j in F)   [empty for injective]
 *   P = [W_p; I_C] (rows U_l), R = [W_r, I_C] (columns U_l),
 *   A_{l+1} = R (A_l P), each product by the canonical Gustavson SpGEMM.
 * The last level A_L is handed to classical AMG (amg.c).  A level may instead
 * relax its F-points with one AMG V-cycle on A_FF (the paper's F-relaxation
 * for the saturation-like blocks of its phase-transition runs, Section 6.2):
 * A_FF = rows and columns F of A_l, numbered in ascending level-local index.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#include "oracle.h"

typedef struct {
    orc_mat A, P, PT, S;
    int32_t *cf;
    double *l1;
    float *Af, *Pf, *PTf, *l1f;
} amg_lev;

/* one classical AMG hierarchy (coarse-grid solver or an F-block solver) */
typedef struct {
    amg_lev *lev;
    int nlev;
    double *lu;
    int32_t *perm;
    int pre, post;
} amg_hier;

typedef struct {
    orc_mat A, P, R;
    int64_t nF, nC;
    int32_t *flist, *clist; /* U-local indices of F and C points */
    int32_t *glob;          /* U-local -> global unknown */
    int32_t *lab;           /* labels of U_l */
    double *dinv;
    float *Af, *Pf, *Rf, *dinvf;
    amg_hier *ff;           /* AMG on A_FF for the F-relaxation, or NULL (Jacobi) */
} mgr_lev;

struct orc_handle {
    int64_t n, ncell;
    int bs, L;
    orc_opts o;
    orc_mat A0;
    double *binv;
    float *binvf;
    mgr_lev *lev;
    amg_hier cg;            /* coarse-grid AMG on A_L */
    double setup_ms;
};

void orc_default_opts(orc_opts *o) {
    o->restart = 30;
    o->max_iter = 400;
    o->rp_type = 0;
    o->global_relax = 1;
    o->f_sweeps = 1;
    o->amg_theta = 0.25;
    o->amg_pre = 2;
    o->amg_post = 2;
    o->amg_max_levels = 25;
    o->amg_coarse_max = 64;
    o->dense_max = 4096;
    o->pmis_seed = 0;
    o->precision = 0;
    o->use_x0 = 0;
    o->frelax_amg_mask = 0;
    o->frelax_amg_pre = 1;
    o->frelax_amg_post = 1;
    o->cycle_post = 0;
}

static double now_ms(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return ts.tv_sec * 1e3 + ts.tv_nsec * 1e-6;
}

static void seterr(char *err, int len, const char *msg) {
    if (err && len > 0) {
        strncpy(err, msg, (size_t)len - 1);
        err[len - 1] = 0;
    }
}

static int copy_mat(const orc_mat *src, orc_mat *dst) {
    dst->nrows = src->nrows;
    dst->ncols = src->ncols;
    dst->nnz = src->nnz;
    dst->rp = (int64_t *)malloc(((size_t)src->nrows + 1) * sizeof(int64_t));
    dst->ci = (int32_t *)malloc((size_t)(src->nnz > 0 ? src->nnz : 1) * sizeof(int32_t));
    dst->v = (double *)malloc((size_t)(src->nnz > 0 ? src->nnz : 1) * sizeof(double));
    memcpy(dst->rp, src->rp, ((size_t)src->nrows + 1) * sizeof(int64_t));
    memcpy(dst->ci, src->ci, (size_t)src->nnz * sizeof(int32_t));
    memcpy(dst->v, src->v, (size_t)src->nnz * sizeof(double));
    return ORC_OK;
}

static float *to_f32(const double *v, int64_t n) {
    float *f = (float *)malloc((size_t)(n > 0 ? n : 1) * sizeof(float));
    for (int64_t i = 0; i < n; ++i) f[i] = (float)v[i];
    return f;
}

static int validate_csr(const orc_mat *A) {
    if (A->nrows < 0 || A->ncols < 0 || A->rp[0] != 0 || A->rp[A->nrows] != A->nnz) return 0;
    for (int64_t i = 0; i < A->nrows; ++i) {
        if (A->rp[i + 1] < A->rp[i]) return 0;
        for (int64_t p = A->rp[i]; p < A->rp[i + 1]; ++p) {
            if (A->ci[p] < 0 || A->ci[p] >= A->ncols) return 0;
            if (p > A->rp[i] && A->ci[p] <= A->ci[p - 1]) return 0;
        }
    }
    return 1;
}

/* ---------------- classical AMG hierarchy ---------------- */

/* Build the hierarchy on a copy of A: strength -> PMIS -> classical
 * interpolation -> Galerkin P^T (A P), until n <= coarse_max, the level cap,
 * an empty or too large (> 0.9 n) coarse set; dense LU on the last level. */
static int amg_build(amg_hier *H, const orc_mat *A, const orc_opts *o, int pre, int post, char *err, int errlen) {
    int cap = o->amg_max_levels > 0 ? o->amg_max_levels : 1;
    if (cap > 64) cap = 64;
    H->lev = (amg_lev *)calloc(64, sizeof(amg_lev));
    H->pre = pre;
    H->post = post;
    copy_mat(A, &H->lev[0].A);
    int k = 0;
    for (;;) {
        amg_lev *lv = &H->lev[k];
        int64_t n = lv->A.nrows;
        int coarsest = (n <= o->amg_coarse_max) || (k == cap - 1);
        if (!coarsest) {
            orc_strength(&lv->A, o->amg_theta, &lv->S);
            lv->cf = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
            orc_pmis(&lv->S, o->pmis_seed, lv->cf);
            int64_t nc = 0;
            for (int64_t i = 0; i < n; ++i) nc += lv->cf[i] == 1;
            if (nc == 0 || nc == n || (double)nc > 0.9 * (double)n) {
                coarsest = 1;
            } else {
                orc_interp(&lv->A, &lv->S, lv->cf, &lv->P);
                orc_transpose(&lv->P, &lv->PT);
                orc_mat T;
                orc_spgemm(&lv->A, &lv->P, &T);
                orc_spgemm(&lv->PT, &T, &H->lev[k + 1].A);
                orc_mat_free(&T);
                lv->l1 = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
                for (int64_t i = 0; i < n; ++i) {
                    double s = 0.0;
                    for (int64_t p = lv->A.rp[i]; p < lv->A.rp[i + 1]; ++p) s = s + fabs(lv->A.v[p]);
                    if (s == 0.0) {
                        seterr(err, errlen, "AMG: empty row (zero l1 norm)");
                        H->nlev = k + 1;
                        return ORC_E_SINGULAR_BLOCK;
                    }
                    lv->l1[i] = s;
                }
                k++;
                continue;
            }
        }
        /* coarsest level: dense LU */
        H->nlev = k + 1;
        if (n > o->dense_max) {
            seterr(err, errlen, "AMG coarsening stalled above the dense coarse-solve limit");
            return ORC_E_INVALID;
        }
        H->lu = (double *)calloc((size_t)(n > 0 ? n * n : 1), sizeof(double));
        H->perm = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
        for (int64_t i = 0; i < n; ++i)
            for (int64_t p = lv->A.rp[i]; p < lv->A.rp[i + 1]; ++p) H->lu[i * n + lv->A.ci[p]] = lv->A.v[p];
        if (orc_dense_lu((int)n, H->lu, H->perm) != ORC_OK) {
            seterr(err, errlen, "AMG: coarsest matrix is singular");
            return ORC_E_SINGULAR_BLOCK;
        }
        return ORC_OK;
    }
}

static void amg_to_f32(amg_hier *H) {
    for (int k = 0; k + 1 < H->nlev; ++k) {
        amg_lev *lv = &H->lev[k];
        lv->Af = to_f32(lv->A.v, lv->A.nnz);
        lv->Pf = to_f32(lv->P.v, lv->P.nnz);
        lv->PTf = to_f32(lv->PT.v, lv->PT.nnz);
        lv->l1f = to_f32(lv->l1, lv->A.nrows);
    }
}

static void amg_free(amg_hier *H) {
    if (!H->lev) return;
    for (int k = 0; k < 64; ++k) {
        amg_lev *lv = &H->lev[k];
        orc_mat_free(&lv->A);
        orc_mat_free(&lv->P);
        orc_mat_free(&lv->PT);
        orc_mat_free(&lv->S);
        free(lv->cf); free(lv->l1); free(lv->Af); free(lv->Pf); free(lv->PTf); free(lv->l1f);
    }
    free(H->lev);
    free(H->lu);
    free(H->perm);
    H->lev = NULL;
}

/* ---------------- MGR levels ---------------- */

/* rows and columns F of A (F = flist, ascending), renumbered 0..nF-1 */
static void extract_ff(const orc_mat *A, const int64_t *fmap, const int32_t *flist, int64_t nF, orc_mat *Aff) {
    Aff->nrows = Aff->ncols = nF;
    Aff->rp = (int64_t *)calloc((size_t)nF + 1, sizeof(int64_t));
    for (int64_t f = 0; f < nF; ++f) {
        int64_t i = flist[f], c = 0;
        for (int64_t p = A->rp[i]; p < A->rp[i + 1]; ++p) c += fmap[A->ci[p]] >= 0;
        Aff->rp[f + 1] = Aff->rp[f] + c;
    }
    Aff->nnz = Aff->rp[nF];
    Aff->ci = (int32_t *)malloc((size_t)(Aff->nnz > 0 ? Aff->nnz : 1) * sizeof(int32_t));
    Aff->v = (double *)malloc((size_t)(Aff->nnz > 0 ? Aff->nnz : 1) * sizeof(double));
    for (int64_t f = 0; f < nF; ++f) {
        int64_t i = flist[f], q = Aff->rp[f];
        for (int64_t p = A->rp[i]; p < A->rp[i + 1]; ++p) {
            int64_t j = fmap[A->ci[p]];
            if (j < 0) continue;
            Aff->ci[q] = (int32_t)j;
            Aff->v[q] = A->v[p];
            q++;
        }
    }
}

static int setup_mgr_level(orc_handle *h, int l, char *err, int errlen) {
    mgr_lev *lv = &h->lev[l];
    const orc_mat *A = &lv->A;
    int64_t nU = A->nrows;
    int64_t *fmap = (int64_t *)malloc((size_t)(nU > 0 ? nU : 1) * sizeof(int64_t));
    int64_t *cmap = (int64_t *)malloc((size_t)(nU > 0 ? nU : 1) * sizeof(int64_t));
    lv->nF = lv->nC = 0;
    for (int64_t u = 0; u < nU; ++u) {
        fmap[u] = cmap[u] = -1;
        if (lv->lab[u] == l) fmap[u] = lv->nF++;
        else cmap[u] = lv->nC++;
    }
    lv->flist = (int32_t *)malloc((size_t)(lv->nF > 0 ? lv->nF : 1) * sizeof(int32_t));
    lv->clist = (int32_t *)malloc((size_t)(lv->nC > 0 ? lv->nC : 1) * sizeof(int32_t));
    for (int64_t u = 0; u < nU; ++u) {
        if (fmap[u] >= 0) lv->flist[fmap[u]] = (int32_t)u;
        else lv->clist[cmap[u]] = (int32_t)u;
    }
    /* D_FF^{-1} */
    lv->dinv = (double *)malloc((size_t)(lv->nF > 0 ? lv->nF : 1) * sizeof(double));
    for (int64_t f = 0; f < lv->nF; ++f) {
        int64_t i = lv->flist[f];
        double d = 0.0;
        for (int64_t p = A->rp[i]; p < A->rp[i + 1]; ++p)
            if (A->ci[p] == i) d = A->v[p];
        if (d == 0.0) {
            char msg[160];
            snprintf(msg, sizeof msg, "MGR level %d: zero diagonal at F row %lld (global unknown %d)", l,
                     (long long)i, lv->glob[i]);
            seterr(err, errlen, msg);
            free(fmap);
            free(cmap);
            return ORC_E_ZERO_FDIAG;
        }
        lv->dinv[f] = 1.0 / d;
    }
    /* optional AMG on A_FF for the F-relaxation */
    if ((h->o.frelax_amg_mask >> l) & 1) {
        if (lv->nF > 0) {
            orc_mat Aff;
            extract_ff(A, fmap, lv->flist, lv->nF, &Aff);
            lv->ff = (amg_hier *)calloc(1, sizeof(amg_hier));
            int rc = amg_build(lv->ff, &Aff, &h->o, h->o.frelax_amg_pre, h->o.frelax_amg_post, err, errlen);
            orc_mat_free(&Aff);
            if (rc != ORC_OK) {
                free(fmap);
                free(cmap);
                return rc;
            }
        }
    }
    /* P = [W_p; I_C] */
    orc_mat *P = &lv->P;
    P->nrows = nU;
    P->ncols = lv->nC;
    P->rp = (int64_t *)calloc((size_t)nU + 1, sizeof(int64_t));
    for (int64_t u = 0; u < nU; ++u) {
        int64_t cnt = 0;
        if (cmap[u] >= 0) cnt = 1;
        else if (h->o.rp_type != 2)
            for (int64_t p = A->rp[u]; p < A->rp[u + 1]; ++p)
                if (cmap[A->ci[p]] >= 0) cnt++;
        P->rp[u + 1] = P->rp[u] + cnt;
    }
    P->nnz = P->rp[nU];
    P->ci = (int32_t *)malloc((size_t)(P->nnz > 0 ? P->nnz : 1) * sizeof(int32_t));
    P->v = (double *)malloc((size_t)(P->nnz > 0 ? P->nnz : 1) * sizeof(double));
    for (int64_t u = 0; u < nU; ++u) {
        int64_t q = P->rp[u];
        if (cmap[u] >= 0) {
            P->ci[q] = (int32_t)cmap[u];
            P->v[q] = 1.0;
        } else if (h->o.rp_type != 2) {
            double di = lv->dinv[fmap[u]];
            for (int64_t p = A->rp[u]; p < A->rp[u + 1]; ++p) {
                int32_t j = A->ci[p];
                if (cmap[j] < 0) continue;
                P->ci[q] = (int32_t)cmap[j];
                P->v[q] = -(A->v[p] * di);
                q++;
            }
        }
    }
    /* R = [W_r, I_C] with columns in U-local numbering */
    orc_mat *R = &lv->R;
    R->nrows = lv->nC;
    R->ncols = nU;
    R->rp = (int64_t *)calloc((size_t)lv->nC + 1, sizeof(int64_t));
    for (int64_t c = 0; c < lv->nC; ++c) {
        int64_t u = lv->clist[c];
        int64_t cnt = 1;
        if (h->o.rp_type != 1)
            for (int64_t p = A->rp[u]; p < A->rp[u + 1]; ++p)
                if (fmap[A->ci[p]] >= 0) cnt++;
        R->rp[c + 1] = R->rp[c] + cnt;
    }
    R->nnz = R->rp[lv->nC];
    R->ci = (int32_t *)malloc((size_t)(R->nnz > 0 ? R->nnz : 1) * sizeof(int32_t));
    R->v = (double *)malloc((size_t)(R->nnz > 0 ? R->nnz : 1) * sizeof(double));
    for (int64_t c = 0; c < lv->nC; ++c) {
        int64_t u = lv->clist[c];
        int64_t q = R->rp[c];
        int placed = 0;
        if (h->o.rp_type != 1) {
            for (int64_t p = A->rp[u]; p < A->rp[u + 1]; ++p) {
                int32_t j = A->ci[p];
                if (!placed && j > u) {
                    R->ci[q] = (int32_t)u;
                    R->v[q] = 1.0;
                    q++;
                    placed = 1;
                }
                if (fmap[j] < 0) continue;
                R->ci[q] = j;
                R->v[q] = -(A->v[p] * lv->dinv[fmap[j]]);
                q++;
            }
        }
        if (!placed) {
            R->ci[q] = (int32_t)u;
            R->v[q] = 1.0;
        }
    }
    /* A_{l+1} = R (A P) */
    orc_mat T;
    orc_spgemm(A, P, &T);
    orc_mat An;
    orc_spgemm(R, &T, &An);
    orc_mat_free(&T);
    if (l + 1 < h->L) {
        mgr_lev *nx = &h->lev[l + 1];
        nx->A = An;
        nx->lab = (int32_t *)malloc((size_t)(lv->nC > 0 ? lv->nC : 1) * sizeof(int32_t));
        nx->glob = (int32_t *)malloc((size_t)(lv->nC > 0 ? lv->nC : 1) * sizeof(int32_t));
        for (int64_t c = 0; c < lv->nC; ++c) {
            nx->lab[c] = lv->lab[lv->clist[c]];
            nx->glob[c] = lv->glob[lv->clist[c]];
        }
    } else {
        /* the last reduction's coarse operator goes to the coarse-grid AMG */
        int rc = amg_build(&h->cg, &An, &h->o, h->o.amg_pre, h->o.amg_post, err, errlen);
        orc_mat_free(&An);
        if (rc != ORC_OK) {
            free(fmap);
            free(cmap);
            return rc;
        }
    }
    free(fmap);
    free(cmap);
    return ORC_OK;
}

int orc_setup(const orc_mat *A, int bs, const int32_t *labels, const orc_opts *o, orc_handle **out,
              char *err, int errlen) {
    double t0 = now_ms();
    *out = NULL;
    if (!A || A->nrows <= 0 || A->nrows != A->ncols || (bs != 1 && bs != 3) || A->nrows % bs != 0 ||
        !validate_csr(A)) {
        seterr(err, errlen, "invalid matrix or block size");
        return ORC_E_INVALID;
    }
    int L = 0;
    for (int64_t i = 0; i < A->nrows; ++i) {
        if (labels[i] < 0 || labels[i] > 31) {
            seterr(err, errlen, "label out of range [0, 31]");
            return ORC_E_INVALID;
        }
        if (labels[i] > L) L = labels[i];
    }
    orc_handle *h = (orc_handle *)calloc(1, sizeof(orc_handle));
    h->n = A->nrows;
    h->bs = bs;
    h->ncell = A->nrows / bs;
    h->L = L;
    h->o = *o;
    copy_mat(A, &h->A0);
    h->lev = (mgr_lev *)calloc((size_t)(L > 0 ? L : 1), sizeof(mgr_lev));
    int rc = ORC_OK;
    if (o->global_relax && L > 0) {
        h->binv = (double *)malloc((size_t)h->ncell * bs * bs * sizeof(double));
        if (orc_block_inverse(h->ncell, bs, A, h->binv) != ORC_OK) {
            seterr(err, errlen, "singular diagonal cell block");
            rc = ORC_E_SINGULAR_BLOCK;
        }
    }
    if (rc == ORC_OK && L > 0) {
        copy_mat(A, &h->lev[0].A);
        h->lev[0].lab = (int32_t *)malloc((size_t)h->n * sizeof(int32_t));
        h->lev[0].glob = (int32_t *)malloc((size_t)h->n * sizeof(int32_t));
        for (int64_t i = 0; i < h->n; ++i) {
            h->lev[0].lab[i] = labels[i];
            h->lev[0].glob[i] = (int32_t)i;
        }
        for (int l = 0; l < L && rc == ORC_OK; ++l) rc = setup_mgr_level(h, l, err, errlen);
    } else if (rc == ORC_OK) {
        rc = amg_build(&h->cg, A, &h->o, h->o.amg_pre, h->o.amg_post, err, errlen);
    }
    if (rc == ORC_OK && o->precision == 1) {
        for (int l = 0; l < L; ++l) {
            mgr_lev *lv = &h->lev[l];
            lv->Af = to_f32(lv->A.v, lv->A.nnz);
            lv->Pf = to_f32(lv->P.v, lv->P.nnz);
            lv->Rf = to_f32(lv->R.v, lv->R.nnz);
            lv->dinvf = to_f32(lv->dinv, lv->nF);
            if (lv->ff) amg_to_f32(lv->ff);
        }
        amg_to_f32(&h->cg);
        if (h->binv) h->binvf = to_f32(h->binv, h->ncell * bs * bs);
    }
    if (rc != ORC_OK) {
        orc_destroy(h);
        return rc;
    }
    h->setup_ms = now_ms() - t0;
    *out = h;
    return ORC_OK;
}

int orc_destroy(orc_handle *h) {
    if (!h) return ORC_OK;
    orc_mat_free(&h->A0);
    for (int l = 0; l < h->L; ++l) {
        mgr_lev *lv = &h->lev[l];
        orc_mat_free(&lv->A);
        orc_mat_free(&lv->P);
        orc_mat_free(&lv->R);
        free(lv->flist); free(lv->clist); free(lv->glob); free(lv->lab); free(lv->dinv);
        free(lv->Af); free(lv->Pf); free(lv->Rf); free(lv->dinvf);
        if (lv->ff) {
            amg_free(lv->ff);
            free(lv->ff);
        }
    }
    amg_free(&h->cg);
    free(h->lev);
    free(h->binv);
    free(h->binvf);
    free(h);
    return ORC_OK;
}

/* ---- V-cycle, FP64 and FP32 instantiations ---- */
#define REAL double
#define FN(name) name##_d
#define VALS(m, f) ((m).v)
#define VALS2(d, f) (d)
#include "vcycle_impl.h"
#undef REAL
#undef FN
#undef VALS
#undef VALS2
#define REAL float
#define FN(name) name##_f
#define VALS(m, f) (f)
#define VALS2(d, f) (f)
#include "vcycle_impl.h"
#undef REAL
#undef FN
#undef VALS
#undef VALS2

/* z = M^{-1} r (one V-cycle), in the handle's precision */
static void apply_prec(orc_handle *h, const double *r, double *z) {
    if (h->o.precision == 1) {
        float *rf = (float *)malloc((size_t)h->n * sizeof(float));
        float *zf = (float *)malloc((size_t)h->n * sizeof(float));
        for (int64_t i = 0; i < h->n; ++i) rf[i] = (float)r[i];
        mgr_cycle_f(h, 0, rf, zf);
        for (int64_t i = 0; i < h->n; ++i) z[i] = (double)zf[i];
        free(rf);
        free(zf);
    } else {
        mgr_cycle_d(h, 0, r, z);
    }
}

int orc_vcycle(orc_handle *h, const double *r, double *e) {
    apply_prec(h, r, e);
    return ORC_OK;
}

static double dot(int64_t n, const double *a, const double *b) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Restarted GMRES(m) with right preconditioning (Saad and Schultz 1986), modified
 * Gram-Schmidt and Givens rotations.  The preconditioned directions z_j = M^{-1} v_j
 * are kept, so the update is x += Z y (the flexible form, equal to M^{-1} V y for a
 * fixed preconditioner).  Iterations = Arnoldi steps = preconditioner applications.
 * A cycle ends when |g_{j+1}| <= tol ||b||, on a happy breakdown or at max_iter;
 * convergence is decided on the true residual ||b - A x|| <= tol ||b||. */
int orc_solve(orc_handle *h, const double *b, double *x, double tol, orc_stats *st) {
    double t0 = now_ms();
    int64_t n = h->n;
    int m = h->o.restart > 0 ? h->o.restart : 30;
    int maxit = h->o.max_iter;
    st->iterations = 0;
    st->res_history_len = 0;
    st->setup_ms = h->setup_ms;
    st->n_levels = h->L + h->cg.nlev;
    for (int l = 0; l < h->L && l < 64; ++l) {
        st->level_n[l] = h->lev[l].A.nrows;
        st->level_nnz[l] = h->lev[l].A.nnz;
    }
    for (int k = 0; k < h->cg.nlev && h->L + k < 64; ++k) {
        st->level_n[h->L + k] = h->cg.lev[k].A.nrows;
        st->level_nnz[h->L + k] = h->cg.lev[k].A.nnz;
    }
    double bnorm = sqrt(dot(n, b, b));
    if (!isfinite(bnorm)) {
        st->status = ORC_E_BREAKDOWN;
        return ORC_E_BREAKDOWN;
    }
    if (!h->o.use_x0)
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        st->rel_residual = 0.0;
        st->status = ORC_OK;
        st->solve_ms = now_ms() - t0;
        return ORC_OK;
    }
    double *V = (double *)malloc((size_t)(m + 1) * n * sizeof(double));
    double *Z = (double *)malloc((size_t)m * n * sizeof(double));
    double *w = (double *)malloc((size_t)n * sizeof(double));
    double *r = (double *)malloc((size_t)n * sizeof(double));
    double *H = (double *)calloc((size_t)(m + 1) * m, sizeof(double)); /* H[i*m + j] */
    double *cs = (double *)malloc((size_t)m * sizeof(double));
    double *sn = (double *)malloc((size_t)m * sizeof(double));
    double *g = (double *)malloc((size_t)(m + 1) * sizeof(double));
    double *y = (double *)malloc((size_t)m * sizeof(double));
    int its = 0, status = ORC_NOT_CONVERGED;
    double rel = 0.0;
    for (;;) {
        orc_spmv(&h->A0, x, r);
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
        double beta = sqrt(dot(n, r, r));
        rel = beta / bnorm;
        if (!isfinite(beta)) { status = ORC_E_BREAKDOWN; break; }
        if (beta <= tol * bnorm) { status = ORC_OK; break; }
        if (its >= maxit) { status = ORC_NOT_CONVERGED; break; }
        for (int64_t i = 0; i < n; ++i) V[i] = r[i] / beta;
        for (int i = 0; i <= m; ++i) g[i] = 0.0;
        g[0] = beta;
        int k = 0;
        int broke = 0;
        for (int j = 0; j < m; ++j) {
            double *vj = V + (size_t)j * n, *zj = Z + (size_t)j * n;
            apply_prec(h, vj, zj);
            orc_spmv(&h->A0, zj, w);
            for (int i = 0; i <= j; ++i) {
                double *vi = V + (size_t)i * n;
                double hij = dot(n, w, vi);
                H[i * m + j] = hij;
                for (int64_t q = 0; q < n; ++q) w[q] = w[q] - hij * vi[q];
            }
            double hn = sqrt(dot(n, w, w));
            for (int i = 0; i < j; ++i) {
                double a = H[i * m + j], bb = H[(i + 1) * m + j];
                H[i * m + j] = cs[i] * a + sn[i] * bb;
                H[(i + 1) * m + j] = -sn[i] * a + cs[i] * bb;
            }
            double a = H[j * m + j];
            double den = sqrt(a * a + hn * hn);
            if (den == 0.0) { cs[j] = 1.0; sn[j] = 0.0; }
            else { cs[j] = a / den; sn[j] = hn / den; }
            H[j * m + j] = cs[j] * a + sn[j] * hn;
            H[(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            its++;
            k = j + 1;
            if (st->res_history && st->res_history_len < st->res_history_cap)
                st->res_history[st->res_history_len++] = fabs(g[j + 1]) / bnorm;
            if (!isfinite(hn) || !isfinite(g[j + 1])) { broke = 1; break; }
            if (fabs(g[j + 1]) <= tol * bnorm || hn == 0.0 || its >= maxit) break;
            double *vn = V + (size_t)(j + 1) * n;
            for (int64_t q = 0; q < n; ++q) vn[q] = w[q] / hn;
        }
        if (broke) { status = ORC_E_BREAKDOWN; break; }
        for (int i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int q = i + 1; q < k; ++q) s = s - H[i * m + q] * y[q];
            y[i] = s / H[i * m + i];
        }
        for (int i = 0; i < k; ++i) {
            double *zi = Z + (size_t)i * n;
            for (int64_t q = 0; q < n; ++q) x[q] = x[q] + y[i] * zi[q];
        }
    }
    st->iterations = its;
    st->rel_residual = rel;
    st->status = status;
    free(V); free(Z); free(w); free(r); free(H); free(cs); free(sn); free(g); free(y);
    st->solve_ms = now_ms() - t0;
    return status;
}

/* ---- introspection ----
 * For the F-relaxation AMG of MGR level l, the level argument is (l << 8) | k. */
int orc_num_mgr_levels(orc_handle *h) { return h->L; }
int orc_num_amg_levels(orc_handle *h) { return h->cg.nlev; }
int orc_num_ff_levels(orc_handle *h, int l) {
    if (l < 0 || l >= h->L || !h->lev[l].ff) return 0;
    return h->lev[l].ff->nlev;
}

static amg_hier *hier_of(orc_handle *h, int ff_kind, int *level) {
    if (ff_kind) {
        int l = *level >> 8;
        *level &= 0xff;
        if (l < 0 || l >= h->L || !h->lev[l].ff) return NULL;
        return h->lev[l].ff;
    }
    return &h->cg;
}

int orc_get_mat(orc_handle *h, int kind, int level, orc_mat *out) {
    const orc_mat *m = NULL;
    if (kind <= 2) {
        if (level < 0 || level >= h->L) return ORC_E_INVALID;
        m = kind == 0 ? &h->lev[level].A : kind == 1 ? &h->lev[level].P : &h->lev[level].R;
    } else {
        amg_hier *H = hier_of(h, kind >= 6, &level);
        if (!H || level < 0 || level >= H->nlev) return ORC_E_INVALID;
        if (kind == 3 || kind == 6) m = &H->lev[level].A;
        else if (level >= H->nlev - 1) return ORC_E_INVALID;
        else if (kind == 4 || kind == 7) m = &H->lev[level].P;
        else if (kind == 5) m = &H->lev[level].S;
        else return ORC_E_INVALID;
    }
    *out = *m; /* a view: the handle keeps ownership */
    return ORC_OK;
}

int64_t orc_get_vec_len(orc_handle *h, int kind, int level) {
    if (kind == 0) return h->binv ? h->ncell * h->bs * h->bs : 0;
    if (kind >= 1 && kind <= 3) {
        if (level < 0 || level >= h->L) return -1;
        return kind == 3 ? h->lev[level].nC : h->lev[level].nF;
    }
    int base = (kind >= 8) ? kind - 4 : kind; /* 8..11 mirror 4..7 for an F-block AMG */
    amg_hier *H = hier_of(h, kind >= 8, &level);
    if (!H) return -1;
    switch (base) {
    case 4: case 5: return (level >= 0 && level < H->nlev - 1) ? H->lev[level].A.nrows : -1;
    case 6: { int64_t n = H->lev[H->nlev - 1].A.nrows; return n * n; }
    case 7: return H->lev[H->nlev - 1].A.nrows;
    }
    return -1;
}

int orc_get_vec(orc_handle *h, int kind, int level, void *out) {
    int64_t len = orc_get_vec_len(h, kind, level);
    if (len < 0) return ORC_E_INVALID;
    if (kind == 0) { memcpy(out, h->binv, (size_t)len * sizeof(double)); return ORC_OK; }
    if (kind == 1) { memcpy(out, h->lev[level].dinv, (size_t)len * sizeof(double)); return ORC_OK; }
    if (kind == 2) { memcpy(out, h->lev[level].flist, (size_t)len * sizeof(int32_t)); return ORC_OK; }
    if (kind == 3) { memcpy(out, h->lev[level].clist, (size_t)len * sizeof(int32_t)); return ORC_OK; }
    int base = (kind >= 8) ? kind - 4 : kind;
    amg_hier *H = hier_of(h, kind >= 8, &level);
    switch (base) {
    case 4: memcpy(out, H->lev[level].cf, (size_t)len * sizeof(int32_t)); break;
    case 5: memcpy(out, H->lev[level].l1, (size_t)len * sizeof(double)); break;
    case 6: memcpy(out, H->lu, (size_t)len * sizeof(double)); break;
    case 7: memcpy(out, H->perm, (size_t)len * sizeof(int32_t)); break;
    }
    return ORC_OK;
}
