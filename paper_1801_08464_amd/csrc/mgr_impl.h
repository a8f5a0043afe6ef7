// Internal declarations of libmgr (HIP, gfx950).  Not part of the C ABI.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "mgr.h"

namespace mgr {

constexpr int kWave = 64;

// Solve-phase copy of a long-row CSR matrix in row-block jagged order: the
// rows are taken in blocks of kJagRows; inside a block they are ranked by length
// (longest first, ties by row), and the block's entries are stored slot by slot
// (slot k holds the k-th entry of every row longer than k, in rank order), over
// the same entry range [rp[block start], rp[block end]) as the CSR.  Entry k of
// the row of rank s then sits at st[bst[b] + k] + s of its block, so a stream
// of consecutive entries gathers x for consecutive rows at the same stencil slot.
constexpr int kJagRows = 256;
constexpr int kJagMaxSlots = 508;  // longest row a jagged copy takes (the slot table fits 2 KB of LDS)
struct Jag {
    int64_t nblk = 0, nst = 0;
    int32_t *ci = nullptr;   // nnz, jagged order (null where co holds the columns)
    uint16_t *co = nullptr;  // nnz, jagged order: column - sb[slot] (16-bit form)
    int32_t *sb = nullptr;   // nst, parallel to st: each slot's smallest column (16-bit form)
    double *v = nullptr;     // nnz, jagged order
    float *vf = nullptr;
    int32_t *rows = nullptr; // n: row of each rank (global row index)
    int32_t *bst = nullptr;  // nblk + 1: start of each block's slot table in st
    int32_t *st = nullptr;   // per block, maxlen + 1 slot starts relative to the block's first entry
};

// Device CSR (int32 row pointers and columns).  vf is the FP32 copy of the
// values used by the mixed-precision hierarchy.  jag: the solve-phase copy of a
// long-row matrix (null when the matrix has none).
struct DCsr {
    int64_t nrows = 0, ncols = 0, nnz = 0;
    int32_t *rp = nullptr, *ci = nullptr;
    double *v = nullptr;
    float *vf = nullptr;
    Jag *jag = nullptr;
};

// Cell-sliced ELL of the level-0 operator: 64 consecutive cells form a slice;
// inside a slice, the rows of component v (u = bs*c + v) form one ELL block of
// width w[s*bs+v] stored slot-major (slot t of lane l at (off + t)*64 + l), so
// every load of a wavefront is one contiguous 256/512-byte segment and only the
// matrix's true nonzeros (plus per-slice padding) are stored.
struct CSell {
    int64_t ncell = 0, nslice = 0, nslot = 0, nnz_true = 0;
    int bs = 1;
    int32_t *off = nullptr;    // nslice*bs: first slot group of (slice, component)
    int32_t *width = nullptr;  // nslice*bs
    int32_t *col = nullptr;    // nslot*64 (-1 = padding)
    double *v = nullptr;
    float *vf = nullptr;
    // 16-bit form of the columns (null where a slot's columns span more than
    // 65534): sb[slot] = the slot's smallest column, co = column - sb (0xffff =
    // padding)
    int32_t *sb = nullptr;     // nslot
    uint16_t *co = nullptr;    // nslot*64
};

struct AmgLevel {
    int64_t n = 0, nc = 0;
    DCsr A, P, PT, S;
    int32_t *cf = nullptr;
    double *l1 = nullptr;
    float *l1f = nullptr;
    double *r = nullptr, *x = nullptr, *x2 = nullptr, *t = nullptr;
    float *rf = nullptr, *xf = nullptr, *x2f = nullptr, *tf = nullptr;
};

// Limits of the single-workgroup tail cycle (k_amg_tail, below).
constexpr int kTailThreads = 1024;
constexpr int kTailMaxLevels = 8;
constexpr int kTailMaxRows = 1024;
constexpr int kTailLdsBytes = 144 * 1024;

// one classical AMG hierarchy: the coarse-grid solver, or the F-block solver of an MGR level
struct AmgHier {
    std::vector<AmgLevel> lev;
    std::vector<std::unique_ptr<Jag>> jags;  // the jagged copies its level matrices point to
    int64_t ncoarse = 0;
    double *lu = nullptr;
    int32_t *perm = nullptr;
    int pre = 2, post = 2;
    int tail = -1;  // first level of the single-workgroup tail cycle (-1: none)
    // the tail's matrices (A, P, P^T per level, with l1), the coarsest LU
    // factors and permutation, packed in the LDS layout of the tail kernel
    unsigned char *tail_pack = nullptr;
    int64_t tail_pack_bytes = 0;
    struct TailOffsets {
        int arp, aci, av, prp, pci, pv, rrp, rci, rv, l1;
    } tail_off[kTailMaxLevels];
    int tail_lu = 0, tail_perm = 0;
};

// The bottom of an AMG V-cycle in one workgroup (k_amg_tail): levels of at most
// kTailMaxRows rows down to a dense coarsest level of at most 64 rows.  The
// matrices of those levels, their l1 norms and the coarsest LU factors are
// copied into LDS in one coalesced pass (from a device buffer in the same
// layout, built at setup), every work vector lives in LDS, and all products of
// the cycle then read LDS only.
template <typename T>
struct TailDesc {
    int nlev = 0;      // smoothing levels of the tail
    int pre = 0, post = 0;
    int x0_ready = 0;  // x0_in holds the first level's first Jacobi iterate r / l1
    int nc = 0;        // rows of the coarsest level
    int pack16 = 0;    // pack length in 16-byte words
    int lu = 0, perm = 0, vec = 0;  // byte offsets in LDS
    const uint4 *pack = nullptr;
    const T *r_in = nullptr, *x0_in = nullptr;
    T *x_out = nullptr;
    int n[kTailMaxLevels] = {};
    // byte offsets in LDS of each level's A, P (n rows), P^T (rows of the next level) and l1
    int arp[kTailMaxLevels] = {}, aci[kTailMaxLevels] = {}, av[kTailMaxLevels] = {};
    int prp[kTailMaxLevels] = {}, pci[kTailMaxLevels] = {}, pv[kTailMaxLevels] = {};
    int rrp[kTailMaxLevels] = {}, rci[kTailMaxLevels] = {}, rv[kTailMaxLevels] = {};
    int l1[kTailMaxLevels] = {};
};

struct MgrLevel {
    int64_t n = 0, nF = 0, nC = 0;
    DCsr A, P, R;
    int32_t *flist = nullptr, *clist = nullptr, *fmap = nullptr;
    int32_t *lab = nullptr, *glob = nullptr;
    double *dinv = nullptr;
    float *dinvf = nullptr;
    int32_t *cmap = nullptr;  // level row -> coarse index (-1 on F points)
    bool aff_diag = false;  // A_FF diagonal: the F-relaxation may update in place
    DCsr AF;                // compact copy of the F rows (all columns), row f = level row flist[f]
    DCsr AcF;               // the F columns of A (all rows): r - A e when e_C = 0; columns numbered by
                            // F index where fcompact, else level rows
    // one F-sweep from e = 0 in the pre-smoothing cycle without the global
    // relaxation: the correction stays compact by F index (eF, or the F-block
    // AMG's output), the residual gathers it through AcF, and the prolongation
    // writes e = correction + P e_c in one pass
    bool fcompact = false;
    double *eF = nullptr;   // nF: the Jacobi F-relaxation's compact correction
    float *eFf = nullptr;
    int flanes = 1;         // threads per F row in the F-point residual / relaxation kernels
    DCsr Aff;                     // A_FF (level 0 of ff), kept with the pattern-bound data
    std::shared_ptr<AmgHier> ff;  // AMG V-cycle on A_FF as the F-relaxation (else Jacobi)
    // V-cycle work vectors
    double *e = nullptr, *t = nullptr, *r = nullptr;
    float *ef = nullptr, *tf = nullptr, *rf = nullptr;
};

}  // namespace mgr

struct mgr_handle {
    hipStream_t stream = nullptr;
    mgr_options o{};
    int64_t n = 0, ncell = 0;
    int bs = 1, L = 0;
    std::string err;
    // device memory: `keep` holds what lives as long as the handle and depends on
    // the pattern and labels only (plus the value arrays of the MGR levels, which
    // a value update rewrites in place), `amg` the AMG hierarchies and their work
    // vectors (their coarsening depends on the values: rebuilt on a value
    // update), `scratch` the temporaries of one call (released when it returns)
    struct Arena {
        std::vector<std::pair<void *, size_t>> chunks;  // device blocks and their sizes
        char *cur = nullptr;
        size_t left = 0;
    };
    Arena keep, scratch, amg;
    Arena *live = nullptr;  // where handle-lifetime allocations go (null: keep)
    // blocks released by the arenas, reused by exact size in stream order;
    // freed (stream-ordered) when the handle object goes away
    std::multimap<size_t, void *> spare;
    int device = 0;
    mgr_handle() = default;
    mgr_handle(const mgr_handle &) = delete;
    mgr_handle &operator=(const mgr_handle &) = delete;
    ~mgr_handle();

    mgr::DCsr Ain;   // the matrix as passed (pattern of mgr_pattern_outer)
    mgr::DCsr A0;    // level-0 operator (A or A^T)
    mgr::CSell A0s;  // its sliced form
    double *binv = nullptr;  // 9 planes of ncell (bs = 3) or 1 plane (bs = 1)
    float *binvf = nullptr;
    std::vector<mgr::MgrLevel> lev;
    mgr::DCsr AL;     // the last reduction level's matrix (level 0 of cg)
    mgr::AmgHier cg;  // coarse-grid AMG on the last reduction level

    // Krylov workspace
    int m = 30;
    int64_t ld = 0;  // stride of the Krylov vectors in V, Z and w
    double *V = nullptr, *Z = nullptr, *w = nullptr, *res = nullptr;
    double *dsc = nullptr;   // device scalars and Hessenberg storage
    double *part = nullptr;  // per-block partial sums
    int nblk_red = 0;
    double *hsc = nullptr;   // pinned host mirror of a few scalars
    int *derr = nullptr;     // device error words
    int *herr = nullptr;     // pinned host copy

    // event timing (mgr_set_kernel_timing): tm[0] the level-0 sliced-ELL kernel,
    // tm[1] whole preconditioner applications (the V-cycle), tm[2] the l1-Jacobi
    // sweeps on the coarse-grid matrix (level 0 of the coarse AMG hierarchy).
    // tm[0] and tm[2] hold each launch's own start and end (events the launch
    // records); tm[1] events recorded on the stream around each application
    struct Timer {
        std::vector<hipEvent_t> ev;
        size_t used = 0;
        double bytes = 0;
        int64_t launches = 0;
    };
    bool timing = false;
    Timer tm[3];
    double vc_bytes = 0;  // algorithmic bytes of the V-cycle being recorded
    double setup_ms = 0;
};

namespace mgr {

// ---- helpers (mgr_host.cpp) ----
// device allocation from the library's stream-ordered pool on h->stream
int pool_alloc(mgr_handle *h, void **p, size_t bytes);
// bump allocation from the handle's arena (chunks from the pool), released as a
// whole when the handle ends
int alloc(mgr_handle *h, void **p, size_t bytes);
template <typename T>
inline int alloc_n(mgr_handle *h, T **p, int64_t n) {
    return alloc(h, reinterpret_cast<void **>(p), (size_t)(n > 0 ? n : 1) * sizeof(T));
}
inline unsigned nblocks(int64_t n, int bt) { return (unsigned)((n + bt - 1) / bt); }

// ---- utility kernels (k_util.hip) ----
void launch_iota(int32_t *p, int64_t n, hipStream_t s);  // p[i] = i
void launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
void launch_fill_f64(double *p, double v, int64_t n, hipStream_t s);
void launch_fill_f32(float *p, float v, int64_t n, hipStream_t s);
void launch_cast_f64_f32(const double *a, float *b, int64_t n, hipStream_t s);
void launch_cast_f32_f64(const float *a, double *b, int64_t n, hipStream_t s);
// out[0..n] = exclusive scan of in[0..n-1], out[n] = total.  tmp: >= scan_tmp_words(n) int64.
int64_t scan_tmp_words(int64_t n);
void launch_scan(const int32_t *in, int32_t *out, int64_t n, int64_t *tmp, hipStream_t s);

// ---- setup kernels (k_setup.hip) ----
void launch_validate(int64_t n, int64_t nnz, const int32_t *rp, const int32_t *ci, const int32_t *lab, int *err,
                     hipStream_t s);
void launch_csell_count(int64_t ncell, int bs, const int32_t *rp, int32_t *rowlen, hipStream_t s);
void launch_csell_width(int64_t nslice, int bs, int64_t ncell, const int32_t *rowlen, int32_t *width,
                        hipStream_t s);
void launch_csell_fill(int64_t ncell, int bs, const int32_t *rp, const int32_t *ci, const double *v,
                       const int32_t *off, const int32_t *width, int32_t *col, double *val, hipStream_t s);
// the 16-bit form of the columns: per slot the smallest column and the offsets;
// *bad = 1 where a slot's columns span more than 65534
void launch_csell_pack16(int64_t nslot, const int32_t *col, int32_t *sb, uint16_t *co, int *bad, hipStream_t s);
void launch_block_inverse(int64_t ncell, int bs, const int32_t *rp, const int32_t *ci, const double *v, double *binv,
                          int *err, hipStream_t s);
void launch_level_flags(int64_t n, const int32_t *lab, int l, int32_t *isF, int32_t *isC, hipStream_t s);
void launch_level_maps(int64_t n, const int32_t *lab, int l, const int32_t *fpos, const int32_t *cpos, int32_t *fmap,
                       int32_t *cmap, int32_t *flist, int32_t *clist, hipStream_t s);
void launch_fdiag_inverse(int64_t nF, const int32_t *flist, const int32_t *rp, const int32_t *ci, const double *v,
                          double *dinv, int *err, int *offdiag_flag, const int32_t *fmap, hipStream_t s);
// The row selections below take `lanes` lanes per row (4, 8, 16 or 32; from
// select_lanes, by the matrix's mean row length); every output row keeps the
// source row's column order.
int select_lanes(int64_t nrows, int64_t nnz);
void launch_p_count(int lanes, int64_t n, const int32_t *rp, const int32_t *ci, const int32_t *cmap, int rp_type,
                    int32_t *cnt, hipStream_t s);
void launch_p_fill(int lanes, int64_t n, const int32_t *rp, const int32_t *ci, const double *v, const int32_t *cmap,
                   const int32_t *fmap, const double *dinv, int rp_type, const int32_t *Prp, int32_t *Pci, double *Pv,
                   hipStream_t s);
void launch_r_count(int64_t nC, const int32_t *clist, const int32_t *rp, const int32_t *ci, const int32_t *fmap,
                    int rp_type, int32_t *cnt, hipStream_t s);
void launch_r_fill(int64_t nC, const int32_t *clist, const int32_t *rp, const int32_t *ci, const double *v,
                   const int32_t *fmap, const double *dinv, int rp_type, const int32_t *Rrp, int32_t *Rci,
                   double *Rv, hipStream_t s);
void launch_gather_i32(int64_t n, const int32_t *idx, const int32_t *src, int32_t *dst, hipStream_t s);
// A_FF: rows flist, columns with fmap >= 0 renumbered by fmap (fmap null: every
// column kept unrenumbered, the compact copy of the F rows)
void launch_ff_count(int lanes, int64_t nF, const int32_t *flist, const int32_t *rp, const int32_t *ci,
                     const int32_t *fmap, int32_t *cnt, hipStream_t s);
void launch_ff_fill(int lanes, int64_t nF, const int32_t *flist, const int32_t *rp, const int32_t *ci, const double *v,
                    const int32_t *fmap, const int32_t *Frp, int32_t *Fci, double *Fv, hipStream_t s);
void launch_fcol_count(int lanes, int64_t n, const int32_t *rp, const int32_t *ci, const int32_t *fmap, int32_t *cnt,
                       hipStream_t s);
// the F columns of every row; fnum: columns as F indices (fmap[j]) instead of level rows
void launch_fcol_fill(int lanes, int64_t n, const int32_t *rp, const int32_t *ci, const double *v, const int32_t *fmap,
                      const int32_t *Frp, int32_t *Fci, double *Fv, bool fnum, hipStream_t s);
// SpGEMM C = A B, canonical ascending-k summation.  pass 0 counts into cnt, pass 1 fills.
// group = lanes per output row (4, 8, 16, 32, 64); rows of A may hold up to group * 8
// entries.  nch (fill pass): chunks per lane, 1, 2, 4 or 8, with group * nch at
// least A's longest row.
int spgemm_max_row();
void launch_row_len_stats(int64_t m, const int32_t *list, const int32_t *rp, int *sum, int *mx, hipStream_t s);
void launch_spgemm(int pass, int group, int nch, int64_t m, const int32_t *Arp, const int32_t *Aci, const double *Av,
                   const int32_t *Brp, const int32_t *Bci, const double *Bv, int32_t *cnt_or_Crp, int32_t *Cci,
                   double *Cv, int *err, hipStream_t s);
// stable transpose: count (atomics), fill (atomics), then per-row sort by source row
void launch_transpose_count(int64_t nrows, const int32_t *rp, const int32_t *ci, int32_t *cnt, hipStream_t s);
void launch_transpose_fill(int64_t nrows, const int32_t *rp, const int32_t *ci, const double *v, int32_t *next,
                           int32_t *Tci, double *Tv, hipStream_t s);
void launch_transpose_sort(int64_t ncols, const int32_t *Trp, int32_t *Tci, double *Tv, hipStream_t s);
// classical AMG
void launch_strength(int pass, int64_t n, int64_t nnz, const int32_t *rp, const int32_t *ci, const double *v,
                     double theta, int32_t *cnt_or_Srp, int32_t *Sci, uint8_t *sflag, hipStream_t s);
void launch_pmis_init(int64_t n, const int32_t *STrp, int32_t *state, hipStream_t s);
void launch_pmis_select(int64_t n, const int32_t *Srp, const int32_t *Sci, const int32_t *STrp, const int32_t *STci,
                        const int32_t *state, uint64_t seed, int32_t *newc, hipStream_t s);
void launch_pmis_update(int64_t n, const int32_t *Srp, const int32_t *Sci, const int32_t *newc, int32_t *state,
                        int *counters, hipStream_t s);
void launch_cf_flags(int64_t n, const int32_t *state, int32_t *isC, hipStream_t s);
void launch_interp_count(int64_t n, const int32_t *rp, const int32_t *ci, const uint8_t *sflag, const int32_t *cf,
                         int32_t *cnt, hipStream_t s);
void launch_interp_fill(int64_t n, int64_t nnz, const int32_t *rp, const int32_t *ci, const double *v,
                        const uint8_t *sflag, const int32_t *cf, const int32_t *cmap, const int32_t *Prp, int32_t *Pci,
                        double *Pv, hipStream_t s);
void launch_l1(int64_t n, const int32_t *rp, const double *v, double *l1, int *err, hipStream_t s);
void launch_dense_lu(int64_t n, const int32_t *rp, const int32_t *ci, const double *v, double *lu, int32_t *perm,
                     int *err, hipStream_t s);
void launch_pattern_outer(int64_t n, const int32_t *rp, const int32_t *ci, const double *lam, const double *x,
                          double *d, hipStream_t s);

// ---- solve-phase kernels (k_solve.hip) ----
// Events that a timed launch records itself (hipExtLaunchKernelGGL): they then
// hold the kernel's own start and end, the interval a kernel trace reports,
// rather than the queue around it.  Null: a plain launch.
struct KEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
template <typename T>
void launch_csell(int mode, const CSell &A, const T *vals, const T *x, const T *r, T *y, hipStream_t s,
                  KEvents ev = {});
// mode 0: y = A x;  1: y = r - A x;  2: y += A x;  3: y = x + (r - A x) / d (x != y)
// Whether the solve-phase kernels would stream A as a long-row matrix (the
// matrices that get a jagged copy).
bool csr_long_rows(const DCsr &A);
// Jagged copy: per-block longest row (maxlen + 1 into cnt[b]), then, with the
// exclusive scan of cnt in bst, the ranks, slot tables and the reordered entries
// (columns into J.co and J.sb where J.co is set, else into J.ci; *bad = 1 when a
// 16-bit offset overflows).
void launch_jag_count(const DCsr &A, int32_t *cnt, hipStream_t s);
void launch_jag_fill(const DCsr &A, Jag &J, int *bad, hipStream_t s);
template <typename T>
void launch_csr(int mode, const DCsr &A, const T *vals, const T *x, const T *r, const T *d, T *y, hipStream_t s,
                KEvents ev = {});
// y[map[i]] += eF[fmap[i]] (0 where fmap[i] < 0) + (A x)[i]: a level's prolongation
// with its compact F correction, added into the finer level's vector through map
template <typename T>
void launch_csr_prolong_into(const DCsr &A, const T *vals, const T *x, const T *eF, const int32_t *fmap,
                             const int32_t *map, T *y, hipStream_t s);
// y = A x and y2 = y / d (restriction that also starts the next level's Jacobi sweeps)
template <typename T>
void launch_csr_restrict_div(const DCsr &A, const T *vals, const T *x, const T *d, T *y, T *y2, hipStream_t s);
// F-row residual t[f] = r[i] - (A e)[i], i = rows[f]; A is the compact F-row copy
// (its row f is row rows[f] of the level matrix)
template <typename T>
void launch_csr_rows_residual(const DCsr &A, int lanes, const T *vals, int64_t nrows, const int32_t *rows, const T *e,
                              const T *r, T *t, hipStream_t s);
// e = B^{-1} r with the cell-block inverses (add: e += B^{-1} r)
template <typename T>
void launch_block_apply(int64_t ncell, int bs, const T *binv, const T *r, T *e, bool add, hipStream_t s);
template <typename T>
void launch_frelax_first(int64_t n, const int32_t *fmap, const T *dinv, const T *r, T *e, hipStream_t s);
// The mixed-precision cycle's FP64 input and output folded into level 0 (3x3
// cells): rf = (float) r64 and e = B^{-1} rf; z = (double)(e + e_c on C points)
void launch_block_apply3_in64(int64_t ncell, const float *binv, const double *r64, float *rf, float *e,
                              hipStream_t s);
void launch_scatter_add_out64(int64_t n, const int32_t *cmap, const float *ec, const float *e, double *z,
                              hipStream_t s);
// eF[f] = dinv[f] r[flist[f]]: the same relaxation, the correction kept by F index
template <typename T>
void launch_frelax_first_compact(int64_t nF, const int32_t *flist, const T *dinv, const T *r, T *eF, hipStream_t s);
// e[i] = eF[fmap[i]] (F points) or 0 + ec[cmap[i]] (C points): the injection
// prolongation applied to a compact F-relaxation correction
template <typename T>
void launch_prolong_inject_compact(int64_t n, const int32_t *fmap, const int32_t *cmap, const T *eF, const T *ec,
                                   T *e, hipStream_t s);
template <typename T>
void launch_frelax_scatter(int64_t nF, const int32_t *flist, const T *dinv, const T *t, T *e, hipStream_t s);
// e[i] += dinv[f] (r[i] - (A e)[i]), i = flist[f], A the compact F-row copy; needs A_FF diagonal
template <typename T>
void launch_frelax_inplace(const DCsr &A, int lanes, const T *vals, int64_t nF, const int32_t *flist, const T *dinv,
                           const T *r, T *e, hipStream_t s);
template <typename T>
void launch_div(int64_t n, const T *r, const T *d, T *x, hipStream_t s);
// t[f] = r[idx[f]]  /  e[idx[f]] += d[f]
template <typename T>
void launch_gather(int64_t n, const int32_t *idx, const T *src, T *dst, hipStream_t s);
template <typename T>
void launch_scatter_add(int64_t n, const int32_t *idx, const T *d, T *e, hipStream_t s);
// t[f] = r[idx[f]] and x0[f] = t[f] / d[f]
template <typename T>
void launch_gather_div(int64_t n, const int32_t *idx, const T *src, const T *d, T *dst, T *x0, hipStream_t s);
// e[i] = 0 + d[map[i]] where map[i] >= 0, else 0
template <typename T>
void launch_scatter_set(int64_t n, const int32_t *map, const T *d, T *e, hipStream_t s);
template <typename T>
void launch_lu_solve(int64_t n, const double *lu, const int32_t *perm, const T *b, T *x, hipStream_t s);
template <typename T>
void launch_amg_tail(const TailDesc<T> &d, hipStream_t s);

// ---- semi-smooth Newton support (k_ncp.hip) ----
void launch_axpy_inplace(int64_t n, double alpha, const double *du, double *u, hipStream_t s);
void launch_ncp_eval(int64_t ncell, const int32_t *rp, const int32_t *ci, const double *v, const double *henry,
                     const double *f, const double *u, double *R, int32_t *labels, int *nactive, int *nchanged,
                     hipStream_t s);
void launch_ncp_jac_count(int64_t n, const int32_t *rp, const int32_t *labels, int32_t *cnt, hipStream_t s);
void launch_ncp_jac_fill(int64_t n, const int32_t *rp, const int32_t *ci, const double *v, const double *henry,
                         const int32_t *labels, const int32_t *Jrp, int32_t *Jci, double *Jv, hipStream_t s);

// ---- Krylov kernels (k_krylov.hip) ----
// The Arnoldi basis V and w are stored with a stride ld: a multiple of 64 elements
// with zero padding beyond n, so that every vector starts 512-byte aligned and the
// basis kernels read two elements per 16-byte load (an odd n reads one padding zero).
constexpr int kRedBlocks = 1024;
constexpr int kFusedMaxV = 32;  // widest basis of the fused update-and-dot kernel
int64_t krylov_ld(int64_t n);
int red_blocks(int64_t n);  // number of partial sums the reduction kernels write
// partial sums over blocks of <w, V_i> (i < nv) and <w, w>: part[b*(nv+1) + i]
void launch_mdot(int64_t n, int64_t ld, int nv, const double *V, const double *w, double *part, hipStream_t s);
// w -= sum_i h[i] V_i, then partials of <w, V_i> and <w, w> of the updated w in the
// layout of launch_mdot
void launch_maxpy_dot(int64_t n, int64_t ld, int nv, const double *V, const double *h, double *w, double *part,
                      hipStream_t s);
// w -= sum_i h[i] V_i and partial <w,w>: part[b]; skipped when guard is set and *guard == 0
void launch_maxpy_norm(int64_t n, int64_t ld, int nv, const double *V, const double *h, double *w, double *part,
                       const int *guard, hipStream_t s);
// x += sum_i y[i] Z_i
void launch_zaxpy(int64_t n, int64_t ld, int nv, const double *Z, const double *y, double *x, hipStream_t s);
void launch_norm_part(int64_t n, const double *a, double *part, hipStream_t s);
// y = a * scal[0]  (scal device), or y = a / scal[0] when divide
void launch_scale_dev(int64_t n, const double *a, const double *scal, int divide, double *y, hipStream_t s);
void launch_axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t s);
// single-block finishers operating on the device scalar block
void launch_arnoldi_fin(int stage, int j, int m, int nblk, const double *part, double *dsc, int *guard,
                        hipStream_t s);
void launch_givens(int j, int m, double *dsc, hipStream_t s);
void launch_trisolve(int k, int m, double *dsc, hipStream_t s);
// Arnoldi step j with lagged re-orthogonalisation (restart length <= kFusedMaxV):
// dots of w and of column j with columns 0..j, the coefficient algebra, the
// update writing v_j and u_{j+1}, and the Givens step with the norm of u_{j+1}
void launch_lag_dots(int64_t n, int64_t ld, int nv, const double *V, const double *w, double *part, hipStream_t s);
void launch_lag_coef(int j, int m, int nblk, const double *part, double *dsc, hipStream_t s);
void launch_lag_update(int64_t n, int64_t ld, int nv, double *V, const double *w, const double *dsc, int m,
                       double *part, hipStream_t s);
void launch_lag_givens(int j, int m, int nblk, const double *part, double *dsc, hipStream_t s);
// y_i /= s_i (the preconditioned vectors of the lagged form carry the scale s_i)
void launch_lag_yscale(int k, int m, double *dsc, hipStream_t s);
void launch_norm_fin(int nblk, const double *part, double *out, hipStream_t s);

// layout of the device scalar block dsc (doubles)
struct Dsc {
    __host__ __device__ static int H(int i, int j, int m) { return 64 + i * m + j; }  // (m+1) x m Hessenberg
    __host__ __device__ static int g(int i, int m) { return 64 + (m + 1) * m + i; }  // m+1
    __host__ __device__ static int cs(int i, int m) { return 64 + (m + 1) * m + (m + 1) + i; }
    __host__ __device__ static int sn(int i, int m) { return 64 + (m + 1) * m + (m + 1) + m + i; }
    __host__ __device__ static int y(int i, int m) { return 64 + (m + 1) * m + (m + 1) + 2 * m + i; }
    __host__ __device__ static int hcur(int i, int m) { return 64 + (m + 1) * m + (m + 1) + 3 * m + i; }
    __host__ __device__ static int h2(int i, int m) { return 64 + (m + 1) * m + (m + 1) + 4 * m + i; }
    // lagged re-orthogonalisation: the Hessenberg columns before rotation, the
    // second-pass and projection coefficients of the current step, the norms s_i
    // of the vectors the preconditioner was applied to, g before each rotation
    __host__ __device__ static int lag(int m) { return 64 + (m + 1) * m + (m + 1) + 5 * m; }
    __host__ __device__ static int Hraw(int i, int j, int m) { return lag(m) + i * m + j; }
    __host__ __device__ static int ca(int i, int m) { return lag(m) + (m + 1) * m + i; }
    __host__ __device__ static int ch(int i, int m) { return lag(m) + (m + 1) * m + m + i; }
    __host__ __device__ static int sc(int i, int m) { return lag(m) + (m + 1) * m + 2 * m + i; }
    __host__ __device__ static int gpre(int i, int m) { return lag(m) + (m + 1) * m + 3 * m + 1 + i; }
    __host__ __device__ static int size(int m) { return lag(m) + (m + 1) * m + 4 * m + 2 + 8; }
    // scalar slots (BRK: the lagged second pass found the Krylov space exhausted)
    enum { BNORM = 0, WN0 = 1, WN = 2, GABS = 3, HN = 4, BRK = 5, BETA = 6, RNORM = 7, ALPHA = 8, INVS = 9 };
};

}  // namespace mgr
