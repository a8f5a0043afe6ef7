/*
 * Oracle MGR V-cycle, written once and instantiated twice by mgr.c:
 * REAL = double (FP64 preconditioner) and REAL = float (the FP32 hierarchy of
 * the mixed-precision form).  The coarsest dense solves are FP64 in both.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * MGR(l, r) follows the paper's algorithm "MGR preconditioner with
 * presmoothing" (Section 4) applied recursively over the reduction levels of
 * Section 5, i.e. the error propagator of eq. MGR-pre,
 *   I - M^{-1} A = (I - P M_c^{-1} R A)(I - M_f^{-1} A),
 * with M_f = global block relaxation (level 0 only) followed by F-relaxation
 * (Jacobi with diag(A_FF), or one AMG V-cycle on A_FF), and M_c = the next
 * level (AMG V-cycle at the last level).
 */

/* y = r - M x over rows [0, nrows), values taken from vals */
static void FN(residual)(const orc_mat *M, const REAL *vals, const REAL *r, const REAL *x, REAL *y) {
    for (int64_t i = 0; i < M->nrows; ++i) {
        REAL s = 0;
        for (int64_t p = M->rp[i]; p < M->rp[i + 1]; ++p) s += vals[p] * x[M->ci[p]];
        y[i] = r[i] - s;
    }
}

/* y = M x */
static void FN(spmv)(const orc_mat *M, const REAL *vals, const REAL *x, REAL *y) {
    for (int64_t i = 0; i < M->nrows; ++i) {
        REAL s = 0;
        for (int64_t p = M->rp[i]; p < M->rp[i + 1]; ++p) s += vals[p] * x[M->ci[p]];
        y[i] = s;
    }
}

/* y += M x */
static void FN(spmv_add)(const orc_mat *M, const REAL *vals, const REAL *x, REAL *y) {
    for (int64_t i = 0; i < M->nrows; ++i) {
        REAL s = 0;
        for (int64_t p = M->rp[i]; p < M->rp[i + 1]; ++p) s += vals[p] * x[M->ci[p]];
        y[i] += s;
    }
}

/* classical AMG V(pre, post) cycle from x = 0 with l1-Jacobi smoothing */
static void FN(amg_cycle)(const amg_hier *H, int k, const REAL *r, REAL *x) {
    const amg_lev *lv = &H->lev[k];
    int64_t n = lv->A.nrows;
    if (k == H->nlev - 1) {
        double *rd = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
        double *xd = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
        for (int64_t i = 0; i < n; ++i) rd[i] = (double)r[i];
        orc_dense_lu_solve((int)n, H->lu, H->perm, rd, xd);
        for (int64_t i = 0; i < n; ++i) x[i] = (REAL)xd[i];
        free(rd);
        free(xd);
        return;
    }
    const REAL *Av = VALS(lv->A, lv->Af);
    const REAL *l1 = VALS2(lv->l1, lv->l1f);
    REAL *t = (REAL *)malloc((size_t)n * sizeof(REAL));
    int64_t nc = lv->P.ncols;
    REAL *rc = (REAL *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(REAL));
    REAL *ec = (REAL *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(REAL));
    for (int64_t i = 0; i < n; ++i) x[i] = 0;
    /* pre-smoothing: l1-Jacobi, x += (r - A x) / d_l1 */
    for (int s = 0; s < H->pre; ++s) {
        FN(residual)(&lv->A, Av, r, x, t);
        for (int64_t i = 0; i < n; ++i) x[i] = x[i] + t[i] / l1[i];
    }
    /* coarse-grid correction x += P M_c^{-1} P^T (r - A x) */
    FN(residual)(&lv->A, Av, r, x, t);
    FN(spmv)(&lv->PT, VALS(lv->PT, lv->PTf), t, rc);
    FN(amg_cycle)(H, k + 1, rc, ec);
    FN(spmv_add)(&lv->P, VALS(lv->P, lv->Pf), ec, x);
    /* post-smoothing */
    for (int s = 0; s < H->post; ++s) {
        FN(residual)(&lv->A, Av, r, x, t);
        for (int64_t i = 0; i < n; ++i) x[i] = x[i] + t[i] / l1[i];
    }
    free(t);
    free(rc);
    free(ec);
}

/* e += blockdiag(A_0)^{-1} v with the cell blocks (global relaxation) */
static void FN(block_apply_add)(orc_handle *h, const REAL *v, REAL *e) {
    const REAL *bi = VALS2(h->binv, h->binvf);
    if (h->bs == 3) {
        for (int64_t c = 0; c < h->ncell; ++c) {
            const REAL *B = bi + 9 * c;
            const REAL *vv = v + 3 * c;
            for (int q = 0; q < 3; ++q)
                e[3 * c + q] = e[3 * c + q] + (B[3 * q] * vv[0] + B[3 * q + 1] * vv[1] + B[3 * q + 2] * vv[2]);
        }
    } else {
        for (int64_t c = 0; c < h->ncell; ++c) e[c] = e[c] + bi[c] * v[c];
    }
}

/* F-relaxation sweeps: e_F += M_FF^{-1} (r - A e)_F with M_FF = diag(A_FF)
 * (Jacobi) or one AMG V-cycle on A_FF */
static void FN(frelax)(orc_handle *h, mgr_lev *lv, const REAL *Av, const REAL *dinv, const REAL *r, REAL *e,
                       REAL *tf, REAL *df) {
    const int64_t nF = lv->nF;
    for (int s = 0; s < h->o.f_sweeps; ++s) {
        for (int64_t f = 0; f < nF; ++f) {
            int64_t i = lv->flist[f];
            REAL acc = 0;
            for (int64_t p = lv->A.rp[i]; p < lv->A.rp[i + 1]; ++p) acc += Av[p] * e[lv->A.ci[p]];
            tf[f] = r[i] - acc;
        }
        if (lv->ff) {
            FN(amg_cycle)(lv->ff, 0, tf, df);
            for (int64_t f = 0; f < nF; ++f) e[lv->flist[f]] = e[lv->flist[f]] + df[f];
        } else {
            for (int64_t f = 0; f < nF; ++f) e[lv->flist[f]] = e[lv->flist[f]] + dinv[f] * tf[f];
        }
    }
}

static void FN(mgr_cycle)(orc_handle *h, int l, const REAL *r, REAL *e) {
    if (l == h->L) {
        FN(amg_cycle)(&h->cg, 0, r, e);
        return;
    }
    mgr_lev *lv = &h->lev[l];
    int64_t nU = lv->A.nrows, nF = lv->nF, nC = lv->nC;
    const REAL *Av = VALS(lv->A, lv->Af);
    const REAL *dinv = VALS2(lv->dinv, lv->dinvf);
    REAL *rho = (REAL *)malloc((size_t)(nU > 0 ? nU : 1) * sizeof(REAL));
    REAL *rc = (REAL *)malloc((size_t)(nC > 0 ? nC : 1) * sizeof(REAL));
    REAL *ec = (REAL *)malloc((size_t)(nC > 0 ? nC : 1) * sizeof(REAL));
    REAL *tf = (REAL *)malloc((size_t)(nF > 0 ? nF : 1) * sizeof(REAL));
    REAL *df = (REAL *)malloc((size_t)(nF > 0 ? nF : 1) * sizeof(REAL));
    for (int64_t i = 0; i < nU; ++i) e[i] = 0;
    if (h->o.cycle_post) {
        /* post-smoothing form, eq. MGR-post: the coarse-grid correction from e = 0
         * first, then the same smoother M_f as in eq. MGR-pre, with its steps in the
         * same order: the level-0 global relaxation, then the F-relaxation */
        FN(spmv)(&lv->R, VALS(lv->R, lv->Rf), r, rc);
        FN(mgr_cycle)(h, l + 1, rc, ec);
        FN(spmv_add)(&lv->P, VALS(lv->P, lv->Pf), ec, e);
        if (l == 0 && h->o.global_relax) {
            FN(residual)(&lv->A, Av, r, e, rho);
            FN(block_apply_add)(h, rho, e);
        }
        FN(frelax)(h, lv, Av, dinv, r, e, tf, df);
    } else {
        /* (1) global relaxation e = blockdiag(A)^{-1} r (level 0 only) */
        if (l == 0 && h->o.global_relax) FN(block_apply_add)(h, r, e);
        /* (2) F-relaxation */
        FN(frelax)(h, lv, Av, dinv, r, e, tf, df);
        /* (3) coarse-grid correction e += P M_c^{-1} R (r - A e) */
        FN(residual)(&lv->A, Av, r, e, rho);
        FN(spmv)(&lv->R, VALS(lv->R, lv->Rf), rho, rc);
        FN(mgr_cycle)(h, l + 1, rc, ec);
        FN(spmv_add)(&lv->P, VALS(lv->P, lv->Pf), ec, e);
    }
    free(rho);
    free(rc);
    free(ec);
    free(tf);
    free(df);
}
