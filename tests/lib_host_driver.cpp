// Every path of libmgr that runs on the host alone (no device): option
// defaults and validation, argument checks of every entry point, status
// strings and the per-thread error text.  Built with the host sanitizers by
// tests/test_lib_host_sanitized.py; exits 0 when every call returns what the
// C ABI promises.
#include <cstdio>
#include <cstring>

#include "mgr.h"

static int failures = 0;

static void expect(bool ok, const char *what) {
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s\n", what);
        ++failures;
    }
}

static void expect_invalid(int rc, const char *what) {
    expect(rc == MGR_E_INVALID, what);
    const char *e = mgr_last_error(nullptr);
    expect(e != nullptr && std::strlen(e) > 0, "error text after a rejected call");
}

int main() {
    mgr_options o;
    mgr_default_options(&o);
    expect(o.restart == 30 && o.max_iter == 400 && o.precision == 0 && o.dense_max == 4096, "defaults");
    for (int c = -8; c <= 2; ++c) expect(mgr_status_string(c) != nullptr, "status string");

    // host arrays stand in for device pointers: no call below reaches the device
    int rp[7] = {0, 0, 0, 0, 0, 0, 0}, ci[1] = {0}, lab[6] = {0, 0, 0, 0, 0, 0};
    double v[1] = {0.0};
    mgr_csr A{6, 0, rp, ci, v};
    mgr_handle *h = reinterpret_cast<mgr_handle *>(0x1);
    expect_invalid(mgr_setup(nullptr, 3, lab, &o, &h), "setup: null matrix");
    expect(h == nullptr, "setup: handle cleared on failure");
    expect_invalid(mgr_setup(&A, 3, nullptr, &o, &h), "setup: null labels");
    expect_invalid(mgr_setup(&A, 3, lab, nullptr, &h), "setup: null options");
    expect_invalid(mgr_setup(&A, 2, lab, &o, &h), "setup: block size 2");
    mgr_csr bad = A;
    bad.n = 0;
    expect_invalid(mgr_setup(&bad, 3, lab, &o, &h), "setup: n = 0");
    bad = A;
    bad.n = 7;
    expect_invalid(mgr_setup(&bad, 3, lab, &o, &h), "setup: n not a multiple of the block size");
    bad = A;
    bad.nnz = -1;
    expect_invalid(mgr_setup(&bad, 3, lab, &o, &h), "setup: negative nnz");
    bad = A;
    bad.nnz = 3;
    bad.col_idx = nullptr;
    expect_invalid(mgr_setup(&bad, 3, lab, &o, &h), "setup: entries without columns");
    bad = A;
    bad.row_ptr = nullptr;
    expect_invalid(mgr_setup(&bad, 3, lab, &o, &h), "setup: null row pointers");

    struct Opt {
        const char *what;
        void (*set)(mgr_options &);
    } opts[] = {
        {"precision 2", [](mgr_options &p) { p.precision = 2; }},
        {"restart 0", [](mgr_options &p) { p.restart = 0; }},
        {"restart 65", [](mgr_options &p) { p.restart = 65; }},
        {"max_iter -1", [](mgr_options &p) { p.max_iter = -1; }},
        {"rp_type 3", [](mgr_options &p) { p.rp_type = 3; }},
        {"f_sweeps 9", [](mgr_options &p) { p.f_sweeps = 9; }},
        {"amg_theta 1", [](mgr_options &p) { p.amg_theta = 1.0; }},
        {"amg_theta NaN", [](mgr_options &p) { p.amg_theta = 0.0 / 0.0; }},
        {"amg_pre 9", [](mgr_options &p) { p.amg_pre = 9; }},
        {"amg_post -1", [](mgr_options &p) { p.amg_post = -1; }},
        {"amg_max_levels 33", [](mgr_options &p) { p.amg_max_levels = 33; }},
        {"amg_coarse_max 0", [](mgr_options &p) { p.amg_coarse_max = 0; }},
        {"dense_max 4097", [](mgr_options &p) { p.dense_max = 4097; }},
        {"frelax_amg_mask -1", [](mgr_options &p) { p.frelax_amg_mask = -1; }},
        {"frelax_amg_pre 9", [](mgr_options &p) { p.frelax_amg_pre = 9; }},
        {"cycle_post 2", [](mgr_options &p) { p.cycle_post = 2; }},
        {"index16 2", [](mgr_options &p) { p.index16 = 2; }},
    };
    for (const Opt &c : opts) {
        mgr_options p = o;
        c.set(p);
        expect_invalid(mgr_setup(&A, 3, lab, &p, &h), c.what);
        expect(h == nullptr, c.what);
    }

    // handle entry points with no handle
    double x[6] = {0}, y[6] = {0};
    mgr_stats st{};
    expect_invalid(mgr_solve(nullptr, x, y, 1e-8, &st), "solve: null handle");
    expect_invalid(mgr_update_values(nullptr, x), "update: null handle");
    expect(mgr_pattern_outer(nullptr, x, y, x) == MGR_E_INVALID, "pattern_outer: null handle");
    expect(mgr_apply_preconditioner(nullptr, x, y) == MGR_E_INVALID, "apply: null handle");
    expect(mgr_spmv(nullptr, x, y) == MGR_E_INVALID, "spmv: null handle");
    int nm = -1, na = -1;
    expect(mgr_num_levels(nullptr, &nm, &na) == MGR_E_INVALID, "num_levels: null handle");
    int64_t nr = 0, nc = 0, nz = 0, len = 0;
    expect(mgr_get_matrix(nullptr, 0, 0, &nr, &nc, &nz, nullptr, nullptr, nullptr) == MGR_E_INVALID, "get_matrix");
    expect(mgr_get_vector(nullptr, 0, 0, nullptr, &len) == MGR_E_INVALID, "get_vector");
    expect(mgr_set_kernel_timing(nullptr, 1) == MGR_E_INVALID, "set_kernel_timing");
    double ms = 0, by = 0;
    int64_t launches = 0;
    expect(mgr_kernel_time(nullptr, 0, &ms, &launches, &by) == MGR_E_INVALID, "kernel_time");
    mgr_destroy(nullptr);
    expect(mgr_last_error(nullptr) != nullptr, "last_error(NULL)");

    // the Newton-loop entry points reject a malformed system before any launch
    int32_t labels[6] = {0};
    double R[6] = {0}, henry[2] = {0}, rn = 0;
    int64_t act = 0, chg = 0, nnz = 0;
    mgr_csr L{7, 0, rp, nullptr, nullptr};
    expect_invalid(mgr_ncp_eval(&L, henry, x, y, nullptr, 1.0, R, labels, &rn, &act, &chg, nullptr), "ncp_eval");
    expect_invalid(mgr_ncp_eval_noalloc(&L, henry, x, y, nullptr, 1.0, R, labels, &rn, &act, &chg, nullptr),
                   "ncp_eval_noalloc");
    expect_invalid(mgr_ncp_jacobian(&L, henry, labels, rp, ci, v, 1, &nnz, nullptr), "ncp_jacobian");
    mgr_csr L6{6, 0, rp, nullptr, nullptr};
    expect_invalid(mgr_ncp_eval(&L6, nullptr, x, y, nullptr, 1.0, R, labels, &rn, &act, &chg, nullptr),
                   "ncp_eval: null henry");
    expect_invalid(mgr_ncp_eval_noalloc(&L6, henry, x, y, nullptr, 1.0, nullptr, labels, &rn, &act, &chg, nullptr),
                   "ncp_eval_noalloc: null residual");
    expect_invalid(mgr_ncp_jacobian(&L6, henry, nullptr, rp, ci, v, 1, &nnz, nullptr), "ncp_jacobian: null labels");

    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    std::printf("host paths ok\n");
    return 0;
}
