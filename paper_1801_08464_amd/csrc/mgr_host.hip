// Host orchestration of libmgr and its C ABI: hierarchy setup (every step a
// GPU kernel; the host only reads back sizes and status words), the recursive
// MGR V-cycle and the restarted GMRES driver.
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>

#include "mgr_impl.h"
#include <type_traits>

using namespace mgr;

namespace {

thread_local std::string g_err;

struct Fail {
    int code;
};

#define HIPCHK(x)                                                                                    \
    do {                                                                                             \
        hipError_t e_ = (x);                                                                         \
        if (e_ != hipSuccess) throw_err(h, MGR_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

[[noreturn]] void throw_err(mgr_handle *h, int code, const std::string &msg) {
    if (h) h->err = msg;
    g_err = msg;
    throw Fail{code};
}

// Inside a catch handler of a C-ABI entry point: the status code of the
// exception in flight (no exception may cross the C boundary).
int abi_status(mgr_handle *h) {
    try {
        throw;
    } catch (const Fail &f) {
        return f.code;
    } catch (const std::bad_alloc &) {
        g_err = "host allocation failed";
        if (h) h->err = g_err;
        return MGR_E_OOM;
    } catch (const std::exception &e) {
        g_err = e.what();
        if (h) h->err = g_err;
        return MGR_E_INVALID;
    } catch (...) {
        g_err = "unexpected error";
        if (h) h->err = g_err;
        return MGR_E_INVALID;
    }
}

void sync(mgr_handle *h) { HIPCHK(hipStreamSynchronize(h->stream)); }

template <typename T>
T *dalloc(mgr_handle *h, int64_t n) {
    T *p = nullptr;
    if (alloc_n(h, &p, n) != MGR_OK) throw_err(h, MGR_E_OOM, "device allocation failed");
    return p;
}

// Arenas: bump allocation in chunks taken from the stream-ordered pool.  Each
// pool call costs tens of microseconds, and a hierarchy needs hundreds of
// buffers, so buffers are carved out of 64 MiB chunks (a larger request gets a
// chunk of its own) and released chunk by chunk.  Released blocks are not given
// back to the pool at once: the handle reuses them by exact size (in stream
// order: a kernel queued later on the stream runs after every earlier reader),
// and a destroyed handle, once its stream has drained, leaves them to a
// per-device cache that later handles draw from.
constexpr size_t kArenaChunk = size_t(64) << 20;
constexpr size_t kArenaAlign = 256;
constexpr size_t kBlockCacheMax = size_t(16) << 30;  // per device; beyond: back to the pool

struct BlockCache {
    std::multimap<size_t, void *> blocks;
    size_t bytes = 0;
};
std::mutex g_block_mu;
std::map<int, BlockCache> g_blocks;

void *block_get(mgr_handle *h, size_t bytes) {
    auto it = h->spare.find(bytes);
    if (it != h->spare.end()) {
        void *p = it->second;
        h->spare.erase(it);
        return p;
    }
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        std::lock_guard<std::mutex> lk(g_block_mu);
        auto c = g_blocks.find(dev);
        if (c != g_blocks.end()) {
            auto b = c->second.blocks.find(bytes);
            if (b != c->second.blocks.end()) {
                void *p = b->second;
                c->second.blocks.erase(b);
                c->second.bytes -= bytes;
                return p;
            }
        }
    }
    void *p = nullptr;
    if (pool_alloc(h, &p, bytes) != MGR_OK) throw_err(h, MGR_E_OOM, "device allocation failed");
    return p;
}

// after the handle's stream has drained: its spare blocks go to the device cache
void blocks_to_cache(mgr_handle *h) {
    std::lock_guard<std::mutex> lk(g_block_mu);
    BlockCache &c = g_blocks[h->device];
    for (auto &b : h->spare) {
        if (c.bytes + b.first <= kBlockCacheMax) {
            c.blocks.emplace(b.first, b.second);
            c.bytes += b.first;
        } else {
            (void)hipFreeAsync(b.second, h->stream);
        }
    }
    h->spare.clear();
}

void *arena_alloc(mgr_handle *h, mgr_handle::Arena &a, size_t bytes) {
    bytes = (bytes + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
    if (bytes == 0) bytes = kArenaAlign;
    if (bytes > kArenaChunk / 4) {
        void *p = block_get(h, bytes);
        a.chunks.emplace_back(p, bytes);
        return p;
    }
    if (bytes > a.left) {
        void *p = block_get(h, kArenaChunk);
        a.chunks.emplace_back(p, kArenaChunk);
        a.cur = static_cast<char *>(p);
        a.left = kArenaChunk;
    }
    void *r = a.cur;
    a.cur += bytes;
    a.left -= bytes;
    return r;
}

struct ArenaMark {
    size_t nchunks;
    char *cur;
    size_t left;
};

ArenaMark arena_mark(const mgr_handle::Arena &a) { return {a.chunks.size(), a.cur, a.left}; }

// release every chunk taken after mark m and resume bump allocation where m was
void arena_reset(mgr_handle *h, mgr_handle::Arena &a, const ArenaMark &m) {
    for (size_t i = m.nchunks; i < a.chunks.size(); ++i) h->spare.emplace(a.chunks[i].second, a.chunks[i].first);
    a.chunks.resize(m.nchunks);
    a.cur = m.cur;
    a.left = m.left;
}

void arena_release(mgr_handle *h, mgr_handle::Arena &a) { arena_reset(h, a, ArenaMark{0, nullptr, 0}); }

// the scratch temporaries of one scope, released when the scope ends
struct ScratchScope {
    mgr_handle *h;
    ArenaMark m;
    explicit ScratchScope(mgr_handle *hh) : h(hh), m(arena_mark(hh->scratch)) {}
    ~ScratchScope() { arena_reset(h, h->scratch, m); }
    ScratchScope(const ScratchScope &) = delete;
    ScratchScope &operator=(const ScratchScope &) = delete;
};

// handle-lifetime allocations of a scope go to the value-dependent `amg` arena
struct AmgArenaScope {
    mgr_handle *h;
    mgr_handle::Arena *prev;
    explicit AmgArenaScope(mgr_handle *hh) : h(hh), prev(hh->live) { hh->live = &hh->amg; }
    ~AmgArenaScope() { h->live = prev; }
    AmgArenaScope(const AmgArenaScope &) = delete;
    AmgArenaScope &operator=(const AmgArenaScope &) = delete;
};

// temporary device buffer in the scratch arena
template <typename T>
struct Tmp {
    T *p = nullptr;
    Tmp(mgr_handle *h, int64_t n) {
        p = static_cast<T *>(arena_alloc(h, h->scratch, (size_t)(n > 0 ? n : 1) * sizeof(T)));
    }
    Tmp(const Tmp &) = delete;
    Tmp &operator=(const Tmp &) = delete;
};

template <typename T>
T *salloc(mgr_handle *h, int64_t n) {
    return static_cast<T *>(arena_alloc(h, h->scratch, (size_t)(n > 0 ? n : 1) * sizeof(T)));
}

// one device word to the host; through the handle's pinned block when it has
// one (a pageable destination costs a staged copy)
template <typename T>
T d2h1(mgr_handle *h, const T *p) {
    static_assert(sizeof(T) <= 8, "one word");
    T *dst = h->hsc ? reinterpret_cast<T *>(reinterpret_cast<char *>(h->hsc) + 128) : nullptr;
    T v;
    HIPCHK(hipMemcpyAsync(dst ? dst : &v, p, sizeof(T), hipMemcpyDeviceToHost, h->stream));
    sync(h);
    return dst ? *dst : v;
}

void reset_err(mgr_handle *h) {
    int init[8] = {0, 0, 0, INT_MAX, 0, 0, 0, 0};
    std::memcpy(h->herr, init, sizeof init);
    HIPCHK(hipMemcpyAsync(h->derr, h->herr, sizeof init, hipMemcpyHostToDevice, h->stream));
}

void read_err(mgr_handle *h) {
    HIPCHK(hipMemcpyAsync(h->herr, h->derr, 8 * sizeof(int), hipMemcpyDeviceToHost, h->stream));
    sync(h);
}

// exclusive scan of n counts into out[0..n]; returns the total (checked to fit
// int32).  with_err: the device error words come back with the total (one
// synchronisation for both)
int64_t scan(mgr_handle *h, const int32_t *in, int32_t *out, int64_t n, bool with_err = false) {
    Tmp<int64_t> tmp(h, scan_tmp_words(n));
    launch_scan(in, out, n, tmp.p, h->stream);
    int64_t nt = (n + 2047) / 2048;
    if (with_err) HIPCHK(hipMemcpyAsync(h->herr, h->derr, 8 * sizeof(int), hipMemcpyDeviceToHost, h->stream));
    int64_t total = 0;
    if (n > 0) total = d2h1(h, tmp.p + nt);
    else if (with_err) sync(h);
    if (total > INT_MAX) throw_err(h, MGR_E_INVALID, "a hierarchy matrix exceeds 2^31-1 entries");
    return total;
}

int choose_lanes(const DCsr &A) {
    double avg = A.nrows > 0 ? (double)A.nnz / (double)A.nrows : 0.0;
    if (avg < 2) return 1;
    if (avg < 4) return 2;
    if (avg < 8) return 4;
    if (avg < 16) return 8;
    if (avg < 40) return 16;
    return 32;
}

// lanes per output row: the smallest group (4 to 64 lanes) whose 8 chunks hold
// A's longest row (4 lanes: rows of up to 32 entries, most Galerkin operands)
int spgemm_group(int maxlen) {
    return maxlen <= 32 ? 4 : maxlen <= 64 ? 8 : maxlen <= 128 ? 16 : maxlen <= 256 ? 32 : 64;
}

// chunks per lane of the fill pass: the fewest (1, 2, 4, 8) whose group * nch
// entries hold A's longest row
int spgemm_chunks(int group, int maxlen) {
    const int need = (maxlen + group - 1) / group;
    return need <= 1 ? 1 : need <= 2 ? 2 : need <= 4 ? 4 : 8;
}

// the fill pass's group: at least the count's, and wide enough that four
// chunks per lane hold the longest row (eight chunks take twice the registers
// and halve the wavefronts a SIMD holds; the row counts do not depend on the
// group)
int spgemm_fill_group(int group, int maxlen) {
    while (group < kWave && group * 4 < maxlen) group *= 2;
    return group;
}

DCsr spgemm(mgr_handle *h, const DCsr &A, const DCsr &B, bool scratch = false) {
    DCsr C;
    C.nrows = A.nrows;
    C.ncols = B.ncols;
    Tmp<int32_t> cnt(h, A.nrows);
    C.rp = scratch ? salloc<int32_t>(h, A.nrows + 1) : dalloc<int32_t>(h, A.nrows + 1);
    // count with the group that twice the mean row length needs; a row too long
    // for it (the kernel's error word, read with the scan total) sends the count
    // to the group that the longest row needs
    int group = spgemm_group(A.nrows > 0 ? (int)(2 * A.nnz / A.nrows + 1) : 0);
    reset_err(h);
    // A's longest row (into the error word 1, read back with the scan total)
    launch_row_len_stats(A.nrows, nullptr, A.rp, nullptr, h->derr + 1, h->stream);
    launch_spgemm(0, group, 8, A.nrows, A.rp, A.ci, A.v, B.rp, B.ci, B.v, cnt.p, nullptr, nullptr, h->derr + 6,
                  h->stream);
    C.nnz = scan(h, cnt.p, C.rp, A.nrows, true);
    const int maxlen = h->herr[1];
    if (h->herr[6]) {
        if (maxlen > spgemm_max_row())
            throw_err(h, MGR_E_INVALID,
                      "SpGEMM: a left-operand row exceeds " + std::to_string(spgemm_max_row()) + " entries");
        group = spgemm_group(maxlen);
        reset_err(h);
        launch_spgemm(0, group, 8, A.nrows, A.rp, A.ci, A.v, B.rp, B.ci, B.v, cnt.p, nullptr, nullptr, h->derr + 6,
                      h->stream);
        C.nnz = scan(h, cnt.p, C.rp, A.nrows, true);
        if (h->herr[6]) throw_err(h, MGR_E_INVALID, "SpGEMM: row length check failed");
    }
    C.ci = scratch ? salloc<int32_t>(h, C.nnz) : dalloc<int32_t>(h, C.nnz);
    C.v = scratch ? salloc<double>(h, C.nnz) : dalloc<double>(h, C.nnz);
    const int fgroup = spgemm_fill_group(group, maxlen);
    launch_spgemm(1, fgroup, spgemm_chunks(fgroup, maxlen), A.nrows, A.rp, A.ci, A.v, B.rp, B.ci, B.v, C.rp, C.ci,
                  C.v, h->derr + 6, h->stream);
    return C;
}

DCsr transpose(mgr_handle *h, const DCsr &A, bool values, bool scratch = false) {
    DCsr T;
    T.nrows = A.ncols;
    T.ncols = A.nrows;
    Tmp<int32_t> cnt(h, A.ncols);
    launch_fill_i32(cnt.p, 0, A.ncols, h->stream);
    launch_transpose_count(A.nrows, A.rp, A.ci, cnt.p, h->stream);
    T.rp = scratch ? salloc<int32_t>(h, A.ncols + 1) : dalloc<int32_t>(h, A.ncols + 1);
    T.nnz = scan(h, cnt.p, T.rp, A.ncols);
    T.ci = scratch ? salloc<int32_t>(h, T.nnz) : dalloc<int32_t>(h, T.nnz);
    if (values) T.v = scratch ? salloc<double>(h, T.nnz) : dalloc<double>(h, T.nnz);
    HIPCHK(hipMemcpyAsync(cnt.p, T.rp, A.ncols * sizeof(int32_t), hipMemcpyDeviceToDevice, h->stream));
    launch_transpose_fill(A.nrows, A.rp, A.ci, values ? A.v : nullptr, cnt.p, T.ci, T.v, h->stream);
    launch_transpose_sort(A.ncols, T.rp, T.ci, T.v, h->stream);
    return T;
}

// C = A B into C's arrays, whose pattern an earlier product of the same two
// patterns produced: the value (fill) pass only
void spgemm_values(mgr_handle *h, const DCsr &A, const DCsr &B, DCsr &C) {
    reset_err(h);
    launch_row_len_stats(A.nrows, nullptr, A.rp, nullptr, h->derr + 1, h->stream);
    read_err(h);
    // (read before reset_err clears the host copy of the error words)
    const int maxlen = h->herr[1], group = spgemm_fill_group(spgemm_group(maxlen), maxlen);
    reset_err(h);
    launch_spgemm(1, group, spgemm_chunks(group, maxlen), A.nrows, A.rp, A.ci, A.v, B.rp, B.ci, B.v, C.rp, C.ci, C.v,
                  h->derr + 6, h->stream);
    read_err(h);
    if (h->herr[6]) throw_err(h, MGR_E_INVALID, "SpGEMM: row length check failed");
}

// T = A^T into T's arrays, built earlier from the same pattern (new values)
void transpose_values(mgr_handle *h, const DCsr &A, DCsr &T) {
    ScratchScope scope(h);
    Tmp<int32_t> cnt(h, A.ncols);
    launch_fill_i32(cnt.p, 0, A.ncols, h->stream);
    launch_transpose_count(A.nrows, A.rp, A.ci, cnt.p, h->stream);
    scan(h, cnt.p, T.rp, A.ncols);
    HIPCHK(hipMemcpyAsync(cnt.p, T.rp, A.ncols * sizeof(int32_t), hipMemcpyDeviceToDevice, h->stream));
    launch_transpose_fill(A.nrows, A.rp, A.ci, A.v, cnt.p, T.ci, T.v, h->stream);
    launch_transpose_sort(A.ncols, T.rp, T.ci, T.v, h->stream);
}

void build_csell(mgr_handle *h) {
    CSell &S = h->A0s;
    const DCsr &A = h->A0;
    S.bs = h->bs;
    S.ncell = h->ncell;
    S.nslice = (h->ncell + kWave - 1) / kWave;
    S.nnz_true = A.nnz;
    int64_t npair = S.nslice * S.bs;
    Tmp<int32_t> rowlen(h, A.nrows);
    launch_csell_count(h->ncell, h->bs, A.rp, rowlen.p, h->stream);
    S.width = dalloc<int32_t>(h, npair);
    launch_csell_width(S.nslice, S.bs, S.ncell, rowlen.p, S.width, h->stream);
    S.off = dalloc<int32_t>(h, npair + 1);
    S.nslot = scan(h, S.width, S.off, npair);
    S.col = dalloc<int32_t>(h, S.nslot * kWave);
    S.v = dalloc<double>(h, S.nslot * kWave);
    launch_fill_i32(S.col, -1, S.nslot * kWave, h->stream);
    launch_fill_f64(S.v, 0.0, S.nslot * kWave, h->stream);
    launch_csell_fill(S.ncell, S.bs, A.rp, A.ci, A.v, S.off, S.width, S.col, S.v, h->stream);
    if (h->o.index16) {
        // the 16-bit columns (a slot's lanes are 64 consecutive cells at one
        // stencil position: their columns lie close together); the arrays of a
        // failed attempt stay unused until the handle is destroyed
        S.sb = dalloc<int32_t>(h, S.nslot);
        S.co = dalloc<uint16_t>(h, S.nslot * kWave);
        reset_err(h);
        launch_csell_pack16(S.nslot, S.col, S.sb, S.co, h->derr + 4, h->stream);
        read_err(h);
        if (h->herr[4]) {
            S.sb = nullptr;
            S.co = nullptr;
        }
    }
}

void build_amg(mgr_handle *h, AmgHier &H, const DCsr &Atop, int pre, int post);

// D_FF^{-1} of MGR level l (its inverted F diagonal); a zero diagonal is an error
// naming the row.  Leaves the "A_FF has off-diagonal entries" flag in herr[5].
void fdiag_inverse(mgr_handle *h, int l) {
    MgrLevel &lv = h->lev[l];
    const DCsr &A = lv.A;
    reset_err(h);
    launch_fdiag_inverse(lv.nF, lv.flist, A.rp, A.ci, A.v, lv.dinv, h->derr, h->derr + 5, lv.fmap, h->stream);
    read_err(h);
    if (h->herr[3] != INT_MAX) {
        int row = h->herr[3];
        int g = d2h1(h, lv.glob + row);
        char msg[200];
        std::snprintf(msg, sizeof msg, "MGR level %d: zero diagonal at F row %d (global unknown %d)", l, row, g);
        throw_err(h, MGR_E_ZERO_FDIAG, msg);
    }
}

void build_mgr_level(mgr_handle *h, int l, DCsr &Anext, int32_t *&lab_next, int32_t *&glob_next) {
    MgrLevel &lv = h->lev[l];
    const DCsr &A = lv.A;
    const int64_t n = A.nrows;
    const int sel = select_lanes(A.nrows, A.nnz);  // lanes per row of the row selections
    lv.n = n;
    ScratchScope scope(h);
    Tmp<int32_t> isF(h, n), isC(h, n), fpos(h, n + 1), cpos(h, n + 1);
    lv.cmap = dalloc<int32_t>(h, n);
    launch_level_flags(n, lv.lab, l, isF.p, isC.p, h->stream);
    lv.nF = scan(h, isF.p, fpos.p, n);
    lv.nC = scan(h, isC.p, cpos.p, n);
    if (lv.nC == 0) throw_err(h, MGR_E_INVALID, "MGR level " + std::to_string(l) + " has no coarse points");
    lv.fmap = dalloc<int32_t>(h, n);
    lv.flist = dalloc<int32_t>(h, lv.nF);
    lv.clist = dalloc<int32_t>(h, lv.nC);
    launch_level_maps(n, lv.lab, l, fpos.p, cpos.p, lv.fmap, lv.cmap, lv.flist, lv.clist, h->stream);
    lv.dinv = dalloc<double>(h, lv.nF);
    fdiag_inverse(h, l);
    lv.aff_diag = h->herr[5] == 0;
    // compact copy of the F rows (all columns) for the F-point residual and the
    // in-place F-relaxation, at the levels whose cycle uses them
    if (lv.nF > 0 && ((l == 0 && h->o.global_relax) || h->o.f_sweeps > 1 || h->o.cycle_post)) {
        Tmp<int32_t> cnt(h, lv.nF);
        launch_ff_count(sel, lv.nF, lv.flist, A.rp, A.ci, nullptr, cnt.p, h->stream);
        lv.AF.nrows = lv.nF;
        lv.AF.ncols = n;
        lv.AF.rp = dalloc<int32_t>(h, lv.nF + 1);
        lv.AF.nnz = scan(h, cnt.p, lv.AF.rp, lv.nF);
        lv.AF.ci = dalloc<int32_t>(h, lv.AF.nnz);
        lv.AF.v = dalloc<double>(h, lv.AF.nnz);
        launch_ff_fill(sel, lv.nF, lv.flist, A.rp, A.ci, A.v, nullptr, lv.AF.rp, lv.AF.ci, lv.AF.v, h->stream);
        lv.flanes = choose_lanes(lv.AF);
    }
    // the F columns of A (all rows) for the residual that precedes the
    // restriction, at the levels where e is zero on the C points there (no global
    // relaxation, pre-smoothing cycle); with one F-sweep the correction stays
    // compact and the columns are its F indices
    if (lv.nF > 0 && !h->o.cycle_post && !(l == 0 && h->o.global_relax)) {
        lv.fcompact = h->o.f_sweeps == 1;
        Tmp<int32_t> cnt(h, n);
        launch_fcol_count(sel, n, A.rp, A.ci, lv.fmap, cnt.p, h->stream);
        lv.AcF.nrows = n;
        lv.AcF.ncols = lv.fcompact ? lv.nF : n;
        lv.AcF.rp = dalloc<int32_t>(h, n + 1);
        lv.AcF.nnz = scan(h, cnt.p, lv.AcF.rp, n);
        lv.AcF.ci = dalloc<int32_t>(h, lv.AcF.nnz);
        lv.AcF.v = dalloc<double>(h, lv.AcF.nnz);
        launch_fcol_fill(sel, n, A.rp, A.ci, A.v, lv.fmap, lv.AcF.rp, lv.AcF.ci, lv.AcF.v, lv.fcompact, h->stream);
    }
    // optional F-relaxation by one AMG V-cycle on A_FF
    if (((h->o.frelax_amg_mask >> l) & 1) && lv.nF > 0) {
        Tmp<int32_t> cnt(h, lv.nF);
        DCsr Aff;
        Aff.nrows = Aff.ncols = lv.nF;
        launch_ff_count(sel, lv.nF, lv.flist, A.rp, A.ci, lv.fmap, cnt.p, h->stream);
        Aff.rp = dalloc<int32_t>(h, lv.nF + 1);
        Aff.nnz = scan(h, cnt.p, Aff.rp, lv.nF);
        Aff.ci = dalloc<int32_t>(h, Aff.nnz);
        Aff.v = dalloc<double>(h, Aff.nnz);
        launch_ff_fill(sel, lv.nF, lv.flist, A.rp, A.ci, A.v, lv.fmap, Aff.rp, Aff.ci, Aff.v, h->stream);
        lv.Aff = Aff;
        lv.ff = std::make_shared<AmgHier>();
        AmgArenaScope amg_arena(h);
        build_amg(h, *lv.ff, Aff, h->o.frelax_amg_pre, h->o.frelax_amg_post);
    }
    const int rp_type = h->o.rp_type;
    // P = [W_p; I]
    {
        Tmp<int32_t> cnt(h, n);
        launch_p_count(sel, n, A.rp, A.ci, lv.cmap, rp_type, cnt.p, h->stream);
        lv.P.nrows = n;
        lv.P.ncols = lv.nC;
        lv.P.rp = dalloc<int32_t>(h, n + 1);
        lv.P.nnz = scan(h, cnt.p, lv.P.rp, n);
        lv.P.ci = dalloc<int32_t>(h, lv.P.nnz);
        lv.P.v = dalloc<double>(h, lv.P.nnz);
        launch_p_fill(sel, n, A.rp, A.ci, A.v, lv.cmap, lv.fmap, lv.dinv, rp_type, lv.P.rp, lv.P.ci, lv.P.v, h->stream);
    }
    // R = [W_r, I]
    {
        Tmp<int32_t> cnt(h, lv.nC);
        launch_r_count(lv.nC, lv.clist, A.rp, A.ci, lv.fmap, rp_type, cnt.p, h->stream);
        lv.R.nrows = lv.nC;
        lv.R.ncols = n;
        lv.R.rp = dalloc<int32_t>(h, lv.nC + 1);
        lv.R.nnz = scan(h, cnt.p, lv.R.rp, lv.nC);
        lv.R.ci = dalloc<int32_t>(h, lv.R.nnz);
        lv.R.v = dalloc<double>(h, lv.R.nnz);
        launch_r_fill(lv.nC, lv.clist, A.rp, A.ci, A.v, lv.fmap, lv.dinv, rp_type, lv.R.rp, lv.R.ci, lv.R.v,
                      h->stream);
    }
    // A_{l+1} = R (A P)
    {
        DCsr T = spgemm(h, A, lv.P, true);
        Anext = spgemm(h, lv.R, T);
    }
    lab_next = dalloc<int32_t>(h, lv.nC);
    glob_next = dalloc<int32_t>(h, lv.nC);
    launch_gather_i32(lv.nC, lv.clist, lv.lab, lab_next, h->stream);
    launch_gather_i32(lv.nC, lv.clist, lv.glob, glob_next, h->stream);
}

// The row-block jagged copy of a long-row level matrix for the solve-phase
// SpMV (rows longer than kJagMaxSlots keep the CSR stream kernel).  Level 0 of
// a mixed-precision hierarchy (c16) stores 16-bit column offsets where the
// option asks for them and every slot's columns lie within 65535 of its
// smallest: its rows keep the grid's stencil order, so a slot's columns are
// close together, and the FP32 kernel gains from the smaller stream (8 -> 6
// bytes per entry).  On the coarsened levels the decode outweighed the bytes,
// and in FP64 (12 -> 10 bytes) the gain was under 1 % of a V-cycle.  Else 32-bit
// columns; the 16-bit arrays of a failed attempt stay unused in the arena until
// the hierarchy is rebuilt.
void build_jag(mgr_handle *h, AmgHier &H, DCsr &A, bool c16) {
    if (!csr_long_rows(A)) return;
    reset_err(h);
    launch_row_len_stats(A.nrows, nullptr, A.rp, nullptr, h->derr + 1, h->stream);
    read_err(h);
    if (h->herr[1] > kJagMaxSlots) return;
    auto J = std::make_unique<Jag>();
    J->nblk = (A.nrows + kJagRows - 1) / kJagRows;
    {
        ScratchScope scope(h);
        Tmp<int32_t> cnt(h, J->nblk);
        launch_jag_count(A, cnt.p, h->stream);
        J->bst = dalloc<int32_t>(h, J->nblk + 1);
        J->nst = scan(h, cnt.p, J->bst, J->nblk);
    }
    J->st = dalloc<int32_t>(h, J->nst);
    J->rows = dalloc<int32_t>(h, A.nrows);
    J->v = dalloc<double>(h, A.nnz);
    bool wide = !(c16 && h->o.index16);
    if (!wide) {
        J->co = dalloc<uint16_t>(h, A.nnz);
        J->sb = dalloc<int32_t>(h, J->nst);
        reset_err(h);
        launch_jag_fill(A, *J, h->derr + 4, h->stream);
        read_err(h);
        wide = h->herr[4] != 0;
        if (wide) {
            J->co = nullptr;
            J->sb = nullptr;
        }
    }
    if (wide) {
        J->ci = dalloc<int32_t>(h, A.nnz);
        launch_jag_fill(A, *J, nullptr, h->stream);
    }
    A.jag = J.get();
    H.jags.push_back(std::move(J));
}

// The levels the single-workgroup tail kernel takes (the longest run of levels
// above the coarsest with at most kTailMaxRows rows whose matrices, l1 norms,
// LU factors and work vectors fit its LDS; the coarsest level a dense solve of
// at most 64 rows), and their packed copy in the kernel's LDS layout: first the
// index arrays (A, P, P^T row pointers and columns of each level, the LU
// permutation), then the values (A, P, P^T, l1 of each level, in the
// hierarchy's precision), then the LU factors.  Built after the FP32 copies.
void build_tail(mgr_handle *h, AmgHier &H) {
    H.tail = -1;
    H.tail_pack = nullptr;
    H.tail_pack_bytes = 0;
    const int K = (int)H.lev.size() - 1;
    if (K < 1 || H.ncoarse < 1 || H.ncoarse > kWave) return;
    const int64_t S = h->o.precision == 1 ? 4 : 8;
    const int64_t nc = H.ncoarse;
    auto a16 = [](int64_t b) { return (b + 15) / 16 * 16; };
    // LDS bytes of the tail starting at level k0
    auto bytes = [&](int k0) {
        int64_t ib = 4 * nc, vb = 0, vec = 2 * nc;
        for (int j = k0; j < K; ++j) {
            const AmgLevel &lv = H.lev[j];
            ib += 4 * (lv.n + 1 + lv.A.nnz) + 4 * (lv.n + 1 + lv.P.nnz) + 4 * (lv.PT.nrows + 1 + lv.PT.nnz);
            vb += S * (lv.A.nnz + lv.P.nnz + lv.PT.nnz + lv.n);
            vec += 4 * lv.n;
        }
        return a16(ib) + a16(vb) + a16(8 * nc * nc) + vec * S;
    };
    int k0 = K;
    while (k0 > 0 && K - (k0 - 1) <= kTailMaxLevels && H.lev[k0 - 1].n <= kTailMaxRows &&
           bytes(k0 - 1) <= kTailLdsBytes)
        --k0;
    if (k0 == K) return;
    // offsets
    int64_t o = 0;
    for (int j = k0; j < K; ++j) {
        const AmgLevel &lv = H.lev[j];
        AmgHier::TailOffsets &t = H.tail_off[j - k0];
        t.arp = (int)o; o += 4 * (lv.n + 1);
        t.aci = (int)o; o += 4 * lv.A.nnz;
        t.prp = (int)o; o += 4 * (lv.n + 1);
        t.pci = (int)o; o += 4 * lv.P.nnz;
        t.rrp = (int)o; o += 4 * (lv.PT.nrows + 1);
        t.rci = (int)o; o += 4 * lv.PT.nnz;
    }
    H.tail_perm = (int)o;
    o = a16(o + 4 * nc);
    for (int j = k0; j < K; ++j) {
        const AmgLevel &lv = H.lev[j];
        AmgHier::TailOffsets &t = H.tail_off[j - k0];
        t.av = (int)o; o += S * lv.A.nnz;
        t.pv = (int)o; o += S * lv.P.nnz;
        t.rv = (int)o; o += S * lv.PT.nnz;
        t.l1 = (int)o; o += S * lv.n;
    }
    o = a16(o);
    H.tail_lu = (int)o;
    o = a16(o + 8 * nc * nc);
    H.tail_pack_bytes = o;
    H.tail_pack = dalloc<unsigned char>(h, o);
    unsigned char *P = H.tail_pack;
    hipStream_t s = h->stream;
    auto put = [&](int off, const void *src, int64_t b) {
        if (b > 0) HIPCHK(hipMemcpyAsync(P + off, src, b, hipMemcpyDeviceToDevice, s));
    };
    const bool f32 = S == 4;
    for (int j = k0; j < K; ++j) {
        const AmgLevel &lv = H.lev[j];
        const AmgHier::TailOffsets &t = H.tail_off[j - k0];
        put(t.arp, lv.A.rp, 4 * (lv.n + 1));
        put(t.aci, lv.A.ci, 4 * lv.A.nnz);
        put(t.prp, lv.P.rp, 4 * (lv.n + 1));
        put(t.pci, lv.P.ci, 4 * lv.P.nnz);
        put(t.rrp, lv.PT.rp, 4 * (lv.PT.nrows + 1));
        put(t.rci, lv.PT.ci, 4 * lv.PT.nnz);
        put(t.av, f32 ? (const void *)lv.A.vf : (const void *)lv.A.v, S * lv.A.nnz);
        put(t.pv, f32 ? (const void *)lv.P.vf : (const void *)lv.P.v, S * lv.P.nnz);
        put(t.rv, f32 ? (const void *)lv.PT.vf : (const void *)lv.PT.v, S * lv.PT.nnz);
        put(t.l1, f32 ? (const void *)lv.l1f : (const void *)lv.l1, S * lv.n);
    }
    put(H.tail_perm, H.perm, 4 * nc);
    put(H.tail_lu, H.lu, 8 * nc * nc);
    H.tail = k0;
}

// the tails of the coarse-grid hierarchy and of every F-block hierarchy
void build_tails(mgr_handle *h) {
    AmgArenaScope amg_arena(h);
    build_tail(h, h->cg);
    for (auto &lv : h->lev)
        if (lv.ff) build_tail(h, *lv.ff);
}

// Classical AMG hierarchy on Atop (kept as its level 0): strength -> PMIS ->
// classical interpolation -> Galerkin P^T (A P), down to a dense LU.
void build_amg(mgr_handle *h, AmgHier &H, const DCsr &Atop, int pre, int post) {
    const mgr_options &o = h->o;
    H.pre = pre;
    H.post = post;
    DCsr A = Atop;
    for (int k = 0;; ++k) {
        build_jag(h, H, A, k == 0 && o.precision == 1);
        H.lev.emplace_back();
        AmgLevel &lv = H.lev.back();
        lv.A = A;
        lv.n = A.nrows;
        const int64_t n = A.nrows;
        ScratchScope scope(h);
        bool coarsest = n <= o.amg_coarse_max || k == o.amg_max_levels - 1;
        if (!coarsest) {
            // strength of connection
            Tmp<int32_t> cnt(h, n);
            Tmp<uint8_t> sflag(h, A.nnz);
            launch_strength(0, n, A.nnz, A.rp, A.ci, A.v, o.amg_theta, cnt.p, nullptr, nullptr, h->stream);
            lv.S.nrows = n;
            lv.S.ncols = n;
            lv.S.rp = dalloc<int32_t>(h, n + 1);
            lv.S.nnz = scan(h, cnt.p, lv.S.rp, n);
            lv.S.ci = dalloc<int32_t>(h, lv.S.nnz);
            launch_strength(1, n, A.nnz, A.rp, A.ci, A.v, o.amg_theta, lv.S.rp, lv.S.ci, sflag.p, h->stream);
            DCsr ST = transpose(h, lv.S, false, true);
            // PMIS
            lv.cf = dalloc<int32_t>(h, n);
            Tmp<int32_t> newc(h, n);
            launch_pmis_init(n, ST.rp, lv.cf, h->stream);
            // two rounds per read-back of the counters (those of the second round):
            // once no point is undecided a round changes nothing, and a round
            // without progress repeats itself, so the outcome is that of checking
            // after every round
            for (int round = 0;; round += 2) {
                for (int r = 0; r < 2; ++r) {
                    reset_err(h);
                    launch_pmis_select(n, lv.S.rp, lv.S.ci, ST.rp, ST.ci, lv.cf, o.pmis_seed, newc.p, h->stream);
                    launch_pmis_update(n, lv.S.rp, lv.S.ci, newc.p, lv.cf, h->derr + 6, h->stream);
                }
                read_err(h);
                if (h->herr[6] == 0) break;
                if (h->herr[7] == 0 || round > 100000) throw_err(h, MGR_E_INVALID, "PMIS made no progress");
            }
            Tmp<int32_t> isC(h, n), cmap(h, n + 1);
            launch_cf_flags(n, lv.cf, isC.p, h->stream);
            const int64_t nc = scan(h, isC.p, cmap.p, n);
            if (nc == 0 || nc == n || (double)nc > 0.9 * (double)n) {
                coarsest = true;
            } else {
                lv.nc = nc;
                launch_interp_count(n, A.rp, A.ci, sflag.p, lv.cf, cnt.p, h->stream);
                lv.P.nrows = n;
                lv.P.ncols = nc;
                lv.P.rp = dalloc<int32_t>(h, n + 1);
                lv.P.nnz = scan(h, cnt.p, lv.P.rp, n);
                lv.P.ci = dalloc<int32_t>(h, lv.P.nnz);
                lv.P.v = dalloc<double>(h, lv.P.nnz);
                launch_interp_fill(n, A.nnz, A.rp, A.ci, A.v, sflag.p, lv.cf, cmap.p, lv.P.rp, lv.P.ci, lv.P.v,
                                   h->stream);
                lv.PT = transpose(h, lv.P, true);
                DCsr T = spgemm(h, A, lv.P, true);
                DCsr Ac = spgemm(h, lv.PT, T);
                lv.l1 = dalloc<double>(h, n);
                reset_err(h);
                launch_l1(n, A.rp, A.v, lv.l1, h->derr, h->stream);
                read_err(h);
                if (h->herr[3] != INT_MAX)
                    throw_err(h, MGR_E_SINGULAR_BLOCK,
                              "AMG level " + std::to_string(k) + ": empty row " + std::to_string(h->herr[3]));
                A = Ac;
                continue;
            }
        }
        // coarsest level: dense LU
        if (n > o.dense_max)
            throw_err(h, MGR_E_INVALID, "AMG coarsening stalled at " + std::to_string(n) +
                                            " unknowns, above the dense coarse-solve limit");
        H.ncoarse = n;
        H.lu = dalloc<double>(h, n * n);
        H.perm = dalloc<int32_t>(h, n);
        reset_err(h);
        launch_dense_lu(n, A.rp, A.ci, A.v, H.lu, H.perm, h->derr, h->stream);
        read_err(h);
        if (h->herr[4]) throw_err(h, MGR_E_SINGULAR_BLOCK, "AMG: coarsest matrix is singular");
        return;
    }
}

float *to_f32(mgr_handle *h, const double *v, int64_t n) {
    float *f = dalloc<float>(h, n);
    launch_cast_f64_f32(v, f, n, h->stream);
    return f;
}

// V-cycle work vectors; `update`: the MGR-level ones exist, the AMG ones are new
void alloc_work(mgr_handle *h, bool update = false) {
    const bool mixed = h->o.precision == 1;
    for (size_t l = 0; l < h->lev.size() && !update; ++l) {
        MgrLevel &lv = h->lev[l];
        const bool eF = lv.fcompact && !lv.ff;  // the Jacobi relaxation's compact correction
        if (mixed) {
            lv.rf = dalloc<float>(h, lv.n);
            lv.ef = dalloc<float>(h, lv.n);
            lv.tf = dalloc<float>(h, lv.n);
            if (eF) lv.eFf = dalloc<float>(h, lv.nF);
        } else {
            lv.r = dalloc<double>(h, lv.n);
            lv.e = dalloc<double>(h, lv.n);
            lv.t = dalloc<double>(h, lv.n);
            if (eF) lv.eF = dalloc<double>(h, lv.nF);
        }
    }
    auto amg_work = [&](AmgHier &H) {
        AmgArenaScope amg_arena(h);
        for (auto &lv : H.lev) {
            if (mixed) {
                lv.rf = dalloc<float>(h, lv.n);
                lv.xf = dalloc<float>(h, lv.n);
                lv.x2f = dalloc<float>(h, lv.n);
                lv.tf = dalloc<float>(h, lv.n);
            } else {
                lv.r = dalloc<double>(h, lv.n);
                lv.x = dalloc<double>(h, lv.n);
                lv.x2 = dalloc<double>(h, lv.n);
                lv.t = dalloc<double>(h, lv.n);
            }
        }
    };
    amg_work(h->cg);
    for (auto &lv : h->lev)
        if (lv.ff) amg_work(*lv.ff);
}

void amg_to_mixed(mgr_handle *h, AmgHier &H) {
    AmgArenaScope amg_arena(h);
    for (size_t k = 0; k + 1 < H.lev.size(); ++k) {
        AmgLevel &lv = H.lev[k];
        lv.A.vf = to_f32(h, lv.A.v, lv.A.nnz);
        if (lv.A.jag) lv.A.jag->vf = to_f32(h, lv.A.jag->v, lv.A.nnz);
        lv.P.vf = to_f32(h, lv.P.v, lv.P.nnz);
        lv.PT.vf = to_f32(h, lv.PT.v, lv.PT.nnz);
        lv.l1f = to_f32(h, lv.l1, lv.n);
    }
}

// FP32 copies of the hierarchy's values; `update`: the MGR-level copies exist
// (rewritten in place), the AMG ones belong to freshly built hierarchies
void to_mixed(mgr_handle *h, bool update = false) {
    auto cast = [&](float *&f, const double *v, int64_t n) {
        if (update) launch_cast_f64_f32(v, f, n, h->stream);
        else f = to_f32(h, v, n);
    };
    if (h->binv) cast(h->binvf, h->binv, h->ncell * h->bs * h->bs);
    cast(h->A0s.vf, h->A0s.v, h->A0s.nslot * kWave);
    for (auto &lv : h->lev) {
        cast(lv.A.vf, lv.A.v, lv.A.nnz);
        cast(lv.P.vf, lv.P.v, lv.P.nnz);
        cast(lv.R.vf, lv.R.v, lv.R.nnz);
        if (lv.AF.v) cast(lv.AF.vf, lv.AF.v, lv.AF.nnz);
        if (lv.AcF.v) cast(lv.AcF.vf, lv.AcF.v, lv.AcF.nnz);
        cast(lv.dinvf, lv.dinv, lv.nF);
        if (lv.ff) amg_to_mixed(h, *lv.ff);
    }
    amg_to_mixed(h, h->cg);
}

// ---------------- V-cycle ----------------
template <typename T>
struct P_;
template <>
struct P_<double> {
    static const double *v(const DCsr &A) { return A.v; }
    static const double *v(const CSell &A) { return A.v; }
    static const double *binv(const mgr_handle *h) { return h->binv; }
    static const double *dinv(const MgrLevel &l) { return l.dinv; }
    static const double *l1(const AmgLevel &l) { return l.l1; }
    static double *r(MgrLevel &l) { return l.r; }
    static double *e(MgrLevel &l) { return l.e; }
    static double *t(MgrLevel &l) { return l.t; }
    static double *eF(MgrLevel &l) { return l.eF; }
    static double *r(AmgLevel &l) { return l.r; }
    static double *x(AmgLevel &l) { return l.x; }
    static double *x2(AmgLevel &l) { return l.x2; }
    static double *t(AmgLevel &l) { return l.t; }
    static void fill(double *p, int64_t n, hipStream_t s) { launch_fill_f64(p, 0.0, n, s); }
};
template <>
struct P_<float> {
    static const float *v(const DCsr &A) { return A.vf; }
    static const float *v(const CSell &A) { return A.vf; }
    static const float *binv(const mgr_handle *h) { return h->binvf; }
    static const float *dinv(const MgrLevel &l) { return l.dinvf; }
    static const float *l1(const AmgLevel &l) { return l.l1f; }
    static float *r(MgrLevel &l) { return l.rf; }
    static float *e(MgrLevel &l) { return l.ef; }
    static float *t(MgrLevel &l) { return l.tf; }
    static float *eF(MgrLevel &l) { return l.eFf; }
    static float *r(AmgLevel &l) { return l.rf; }
    static float *x(AmgLevel &l) { return l.xf; }
    static float *x2(AmgLevel &l) { return l.x2f; }
    static float *t(AmgLevel &l) { return l.tf; }
    static void fill(float *p, int64_t n, hipStream_t s) { launch_fill_f32(p, 0.0f, n, s); }
};

// ---- event timing and algorithmic-byte accounting ----
// Algorithmic bytes count every array a launch reads or writes once: stored
// values and column indices, row pointers, the gathered vector at its length,
// and each dense vector the launch touches.
hipEvent_t timer_event(mgr_handle *h, mgr_handle::Timer &t) {
    if (t.ev.size() <= t.used) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        t.ev.push_back(e);
    }
    return t.ev[t.used++];
}

hipEvent_t timer_mark(mgr_handle *h, mgr_handle::Timer &t) {
    hipEvent_t e = timer_event(h, t);
    HIPCHK(hipEventRecord(e, h->stream));
    return e;
}

// the next event pair of t, for a launch that records them itself (a single
// kernel: the pair then holds its own start and end)
KEvents timer_kernel(mgr_handle *h, mgr_handle::Timer &t) {
    KEvents ev;
    ev.start = timer_event(h, t);
    ev.stop = timer_event(h, t);
    return ev;
}

inline void acct(mgr_handle *h, double bytes) {
    if (h->timing) h->vc_bytes += bytes;
}

double csr_bytes(const DCsr &A, int mode, double S) {
    // row pointers, or for a jagged copy the rank-to-row map, the slot tables
    // (with the 16-bit columns also the slot bases) and two row pointers and two
    // table offsets per block
    const bool jag = A.jag && csr_long_rows(A);
    const bool c16 = jag && A.jag->co;
    const double index = jag ? 4.0 * (double)A.nrows + (c16 ? 8.0 : 4.0) * (double)A.jag->nst +
                                   16.0 * (double)A.jag->nblk
                             : 4.0 * (double)(A.nrows + 1);
    double b = (double)A.nnz * (S + (c16 ? 2.0 : 4.0)) + index + S * (double)A.ncols + S * (double)A.nrows;
    if (mode == 1 || mode == 2) b += S * (double)A.nrows;
    if (mode == 3) b += 2.0 * S * (double)A.nrows;
    return b;
}

// the fine-level sliced-ELL kernel, timed by its own start and end events when
// timing is on
template <typename T>
void fine_op(mgr_handle *h, int mode, const T *x, const T *r, T *y) {
    // (events only for a launch that happens: an empty operator launches nothing)
    const bool timed = h->timing && h->A0s.nslice > 0;
    launch_csell<T>(mode, h->A0s, P_<T>::v(h->A0s), x, r, y, h->stream, timed ? timer_kernel(h, h->tm[0]) : KEvents{});
    if (timed) {
        // values + columns of the true nonzeros, row pointers, x and y, plus r
        // for the residual form
        const double n = (double)h->n;
        // (16-bit columns: 2 bytes per entry and the slot bases)
        const double cb = h->A0s.co ? 2.0 * (double)h->A0s.nnz_true + 4.0 * (double)h->A0s.nslot
                                    : 4.0 * (double)h->A0s.nnz_true;
        const double b = (double)h->A0s.nnz_true * sizeof(T) + cb + 4.0 * (n + 1) + 2.0 * n * sizeof(T) +
                         (mode == 1 ? n * sizeof(T) : 0.0);
        h->tm[0].bytes += b;
        h->tm[0].launches++;
        h->vc_bytes += b;
    }
}

template <typename T>
void csr(mgr_handle *h, int mode, const DCsr &A, const T *vals, const T *x, const T *r, const T *d, T *y,
         KEvents ev = {}) {
    launch_csr<T>(mode, A, vals, x, r, d, y, h->stream, ev);
    acct(h, csr_bytes(A, mode, sizeof(T)));
}

// a Jacobi sweep on level k of hierarchy H; the sweeps on the coarse-grid matrix
// itself (level 0 of the coarse hierarchy) are timed by their own start and end
// events when timing is on
template <typename T>
void sweep(mgr_handle *h, const AmgHier &H, int k, const DCsr &A, const T *vals, const T *x, const T *r,
           const T *d, T *y) {
    const bool timed = h->timing && &H == &h->cg && k == 0 && A.nrows > 0;
    csr<T>(h, 3, A, vals, x, r, d, y, timed ? timer_kernel(h, h->tm[2]) : KEvents{});
    if (timed) {
        h->tm[2].bytes += csr_bytes(A, 3, sizeof(T));
        h->tm[2].launches++;
    }
}

// Where level k of H (not its coarsest) reads its first Jacobi iterate when the
// cycle's output goes to x: the sweeps ping-pong between x and x2, arranged so
// that the last one writes x.
template <typename T>
T *amg_x0_buffer(AmgHier &H, int k, T *x) {
    const int swaps = (H.pre > 0 ? H.pre - 1 : 0) + H.post;
    return (swaps % 2 == 0) ? x : P_<T>::x2(H.lev[k]);
}

// the first sweep of level 0 of H can start from an x0 = r / l1 written by the
// caller's restriction or gather
template <typename T>
bool amg_takes_x0(const AmgHier &H) {
    return H.pre > 0 && H.lev.size() > 1;
}

// x0_ready: the caller's restriction already wrote x0 = r / l1 (the first Jacobi
// iterate from zero) where this level's first sweep reads it
// Levels k.. of H in one launch of the tail kernel (same steps and roundings as
// the recursion below).  Bytes: what the kernel reads and writes in memory (its
// packed matrices, l1 and LU factors once, r, x0 and x of level k).
template <typename T>
void tail_cycle(mgr_handle *h, AmgHier &H, int k, const T *r, T *x, bool x0_ready) {
    const int K = (int)H.lev.size() - 1;
    TailDesc<T> d;
    d.nlev = K - k;
    d.pre = H.pre;
    d.post = H.post;
    d.x0_ready = x0_ready ? 1 : 0;
    d.nc = (int)H.ncoarse;
    d.pack16 = (int)(H.tail_pack_bytes / 16);
    d.lu = H.tail_lu;
    d.perm = H.tail_perm;
    d.vec = (int)H.tail_pack_bytes;
    d.pack = reinterpret_cast<const uint4 *>(H.tail_pack);
    d.r_in = r;
    d.x0_in = x0_ready ? amg_x0_buffer<T>(H, k, x) : nullptr;
    d.x_out = x;
    for (int j = 0; j < d.nlev; ++j) {
        const AmgHier::TailOffsets &t = H.tail_off[j];
        d.n[j] = (int)H.lev[k + j].n;
        d.arp[j] = t.arp;
        d.aci[j] = t.aci;
        d.av[j] = t.av;
        d.prp[j] = t.prp;
        d.pci[j] = t.pci;
        d.pv[j] = t.pv;
        d.rrp[j] = t.rrp;
        d.rci[j] = t.rci;
        d.rv[j] = t.rv;
        d.l1[j] = t.l1;
    }
    launch_amg_tail<T>(d, h->stream);
    acct(h, (double)H.tail_pack_bytes + (double)sizeof(T) * (double)d.n[0] * (x0_ready ? 3.0 : 2.0));
}

template <typename T>
void amg_cycle(mgr_handle *h, AmgHier &H, int k, const T *r, T *x, bool x0_ready = false) {
    AmgLevel &lv = H.lev[k];
    hipStream_t s = h->stream;
    const int64_t n = lv.n;
    const double S = sizeof(T);
    if (k == (int)H.lev.size() - 1) {
        launch_lu_solve<T>(n, H.lu, H.perm, r, x, s);
        acct(h, 8.0 * n * n + 4.0 * n + 2.0 * S * n);
        return;
    }
    if (k == H.tail) {
        tail_cycle<T>(h, H, k, r, x, x0_ready);
        return;
    }
    const T *Av = P_<T>::v(lv.A);
    const T *l1 = P_<T>::l1(lv);
    const int pre = H.pre, post = H.post;
    // ping-pong buffers arranged so that the last sweep writes x
    T *cur = amg_x0_buffer<T>(H, k, x);
    T *oth = (cur == x) ? P_<T>::x2(lv) : x;
    for (int it = 0; it < pre; ++it) {
        if (it == 0) {
            if (!x0_ready) {
                launch_div<T>(n, r, l1, cur, s);
                acct(h, 3.0 * S * n);
            }
        } else {
            sweep<T>(h, H, k, lv.A, Av, cur, r, l1, oth);
            std::swap(cur, oth);
        }
    }
    if (pre == 0) {
        P_<T>::fill(cur, n, s);
        acct(h, S * n);
    }
    T *t = P_<T>::t(lv);
    csr<T>(h, 1, lv.A, Av, cur, r, nullptr, t);
    AmgLevel &nx = H.lev[k + 1];
    if (pre > 0 && k + 1 < (int)H.lev.size() - 1) {
        // restriction + the next level's x0 = r / l1, written where its first sweep reads it
        T *nx_cur = amg_x0_buffer<T>(H, k + 1, P_<T>::x(nx));
        launch_csr_restrict_div<T>(lv.PT, P_<T>::v(lv.PT), t, P_<T>::l1(nx), P_<T>::r(nx), nx_cur, s);
        acct(h, csr_bytes(lv.PT, 0, S) + 2.0 * S * (double)nx.n);
        amg_cycle<T>(h, H, k + 1, P_<T>::r(nx), P_<T>::x(nx), true);
    } else {
        csr<T>(h, 0, lv.PT, P_<T>::v(lv.PT), t, nullptr, nullptr, P_<T>::r(nx));
        amg_cycle<T>(h, H, k + 1, P_<T>::r(nx), P_<T>::x(nx));
    }
    csr<T>(h, 2, lv.P, P_<T>::v(lv.P), P_<T>::x(nx), nullptr, nullptr, cur);
    for (int it = 0; it < post; ++it) {
        sweep<T>(h, H, k, lv.A, Av, cur, r, l1, oth);
        std::swap(cur, oth);
    }
}

// x0_ready (l == L only): the restriction into the coarse grid already wrote the
// first Jacobi iterate of the coarse-grid AMG cycle
// The mixed-precision cycle's FP64 ends, taken by level 0 where its first and
// last steps can absorb the casts: in is cast into rf (the level's r)
struct Io64 {
    const double *in = nullptr;
    float *rf = nullptr;
    double *out = nullptr;
};

// Where the finer level's prolongation is e_C += e_c (W_p = 0), that level may
// hand its vector and C list down: the coarser level then adds its result into
// dst[map[i]] instead of writing e (its last launch does both).
template <typename T>
struct OutMap {
    const int32_t *map = nullptr;
    T *dst = nullptr;
};

template <typename T>
void mgr_cycle(mgr_handle *h, int l, const T *r, T *e, bool x0_ready = false, const Io64 *io = nullptr,
               const OutMap<T> *om = nullptr) {
    if (l == h->L) {
        amg_cycle<T>(h, h->cg, 0, r, e, x0_ready);
        return;
    }
    MgrLevel &lv = h->lev[l];
    hipStream_t s = h->stream;
    const T *Av = P_<T>::v(lv.A);
    const T *dinv = P_<T>::dinv(lv);
    T *t = P_<T>::t(lv);
    const double S = sizeof(T), n = (double)lv.n, nF = (double)lv.nF;
    // bytes of a compact F-row product (values, columns, row pointers, F list, e gathered)
    const double afb = (double)lv.AF.nnz * (S + 4.0) + 4.0 * (nF + 1.0) + 4.0 * nF + S * n;
    T *rc, *ec;
    if (l + 1 < h->L) {
        rc = P_<T>::r(h->lev[l + 1]);
        ec = P_<T>::e(h->lev[l + 1]);
    } else {
        rc = P_<T>::r(h->cg.lev[0]);
        ec = P_<T>::x(h->cg.lev[0]);
    }
    // restriction rc = R src, then the next level's cycle; into the coarse grid the
    // restriction also writes the AMG cycle's first Jacobi iterate rc / l1
    auto coarse_correction = [&](const T *src, const OutMap<T> *into = nullptr) {
        if (l + 1 == h->L && amg_takes_x0<T>(h->cg)) {
            AmgLevel &c0 = h->cg.lev[0];
            launch_csr_restrict_div<T>(lv.R, P_<T>::v(lv.R), src, P_<T>::l1(c0), rc, amg_x0_buffer<T>(h->cg, 0, ec),
                                       s);
            acct(h, csr_bytes(lv.R, 0, S) + 2.0 * S * (double)c0.n);
            mgr_cycle<T>(h, l + 1, rc, ec, true);
        } else {
            csr<T>(h, 0, lv.R, P_<T>::v(lv.R), src, nullptr, nullptr, rc);
            mgr_cycle<T>(h, l + 1, rc, ec, false, nullptr, into);
        }
    };
    // F-relaxation sweeps: Jacobi with diag(A_FF), or one AMG V-cycle on A_FF;
    // `have` tells whether e already holds a value (else e = 0 is implied)
    auto frelax = [&](bool have) {
        for (int sw = 0; sw < h->o.f_sweeps; ++sw) {
            if (lv.ff) {
                AmgLevel &f0 = lv.ff->lev[0];
                T *rF = P_<T>::r(f0), *dF = P_<T>::x(f0);
                if (!have) {
                    // from e = 0: gather r_F (with the AMG cycle's first iterate
                    // r_F / l1 where the cycle takes it), cycle, then e = 0 + d on F
                    // and 0 on C in one pass
                    if (amg_takes_x0<T>(*lv.ff)) {
                        launch_gather_div<T>(lv.nF, lv.flist, r, P_<T>::l1(f0), rF, amg_x0_buffer<T>(*lv.ff, 0, dF), s);
                        acct(h, 4.0 * nF + 4.0 * S * nF);
                        amg_cycle<T>(h, *lv.ff, 0, rF, dF, true);
                    } else {
                        launch_gather<T>(lv.nF, lv.flist, r, rF, s);
                        acct(h, 4.0 * nF + 2.0 * S * nF);
                        amg_cycle<T>(h, *lv.ff, 0, rF, dF);
                    }
                    launch_scatter_set<T>(lv.n, lv.fmap, dF, e, s);
                    acct(h, 4.0 * n + S * nF + S * n);
                    have = true;
                } else {
                    launch_csr_rows_residual<T>(lv.AF, lv.flanes, P_<T>::v(lv.AF), lv.nF, lv.flist, e, r, rF, s);
                    acct(h, afb + 2.0 * S * nF);
                    amg_cycle<T>(h, *lv.ff, 0, rF, dF);
                    launch_scatter_add<T>(lv.nF, lv.flist, dF, e, s);
                    acct(h, 4.0 * nF + 3.0 * S * nF);
                }
            } else if (!have) {
                launch_frelax_first<T>(lv.n, lv.fmap, dinv, r, e, s);
                acct(h, 4.0 * n + S * nF + 2.0 * S * n);
                have = true;
            } else if (lv.aff_diag) {
                launch_frelax_inplace<T>(lv.AF, lv.flanes, P_<T>::v(lv.AF), lv.nF, lv.flist, dinv, r, e, s);
                acct(h, afb + 3.0 * S * nF);
            } else {
                launch_csr_rows_residual<T>(lv.AF, lv.flanes, P_<T>::v(lv.AF), lv.nF, lv.flist, e, r, t, s);
                launch_frelax_scatter<T>(lv.nF, lv.flist, dinv, t, e, s);
                acct(h, afb + 2.0 * S * nF + 4.0 * nF + 4.0 * S * nF);
            }
        }
        return have;
    };
    const bool global = l == 0 && h->o.global_relax;
    const double gbytes = (double)h->bs * h->bs * S * h->ncell + 2.0 * S * n;
    if (lv.fcompact) {
        // one F-sweep from e = 0 with the correction kept by F index (the same
        // products and sums as with it scattered into e, whose C entries are 0):
        // F-relaxation, residual r - A_{:,F} e_F, coarse-grid correction, then
        // e = e_F + P e_c in one pass
        const T *eF;
        if (lv.ff) {
            AmgLevel &f0 = lv.ff->lev[0];
            T *rF = P_<T>::r(f0), *dF = P_<T>::x(f0);
            if (amg_takes_x0<T>(*lv.ff)) {
                launch_gather_div<T>(lv.nF, lv.flist, r, P_<T>::l1(f0), rF, amg_x0_buffer<T>(*lv.ff, 0, dF), s);
                acct(h, 4.0 * nF + 4.0 * S * nF);
                amg_cycle<T>(h, *lv.ff, 0, rF, dF, true);
            } else {
                launch_gather<T>(lv.nF, lv.flist, r, rF, s);
                acct(h, 4.0 * nF + 2.0 * S * nF);
                amg_cycle<T>(h, *lv.ff, 0, rF, dF);
            }
            eF = dF;
        } else {
            T *e1 = P_<T>::eF(lv);
            launch_frelax_first_compact<T>(lv.nF, lv.flist, dinv, r, e1, s);
            acct(h, 4.0 * nF + 4.0 * S * nF);
            eF = e1;
        }
        // AcF's columns are F indices: the gathered vector is e_F (nF long)
        launch_csr<T>(1, lv.AcF, P_<T>::v(lv.AcF), eF, r, nullptr, t, s);
        acct(h, csr_bytes(lv.AcF, 1, S));
        coarse_correction(t);
        if (om && lv.P.nnz != lv.nC) {
            // e is not kept: the result goes straight into the finer level's vector
            launch_csr_prolong_into<T>(lv.P, P_<T>::v(lv.P), ec, eF, lv.fmap, om->map, om->dst, s);
            // mode 5's count, the map, and the finer vector read where it is updated
            acct(h, csr_bytes(lv.P, 0, S) + 4.0 * n + S * nF + 4.0 * n + S * n);
            return;
        }
        if (lv.P.nnz == lv.nC) {
            launch_prolong_inject_compact<T>(lv.n, lv.fmap, lv.cmap, eF, ec, e, s);
            acct(h, 8.0 * n + S * nF + S * (double)lv.nC + S * n);
        } else {
            launch_csr<T>(5, lv.P, P_<T>::v(lv.P), ec, eF, reinterpret_cast<const T *>(lv.fmap), e, s);
            // the gathered e_c and the written e (mode 0's count), the F map and e_F
            acct(h, csr_bytes(lv.P, 0, S) + 4.0 * n + S * nF);
        }
        if (om) {
            launch_scatter_add<T>(lv.n, om->map, e, om->dst, s);
            acct(h, 4.0 * n + 3.0 * S * n);
        }
        return;
    }
    if (h->o.cycle_post) {
        // eq. MGR-post: coarse-grid correction from e = 0, then the smoother M_f of
        // the pre-smoothing form with its steps in the same order (global
        // relaxation at level 0, then F-relaxation)
        coarse_correction(r);
        csr<T>(h, 0, lv.P, P_<T>::v(lv.P), ec, nullptr, nullptr, e);
        if (global) {
            fine_op<T>(h, 1, e, r, t);
            launch_block_apply<T>(h->ncell, h->bs, P_<T>::binv(h), t, e, true, s);
            acct(h, gbytes + S * n);
        }
        frelax(true);
        return;
    }
    // (1) global relaxation with the cell blocks (level 0)
    bool have = false;
    if (global) {
        if constexpr (std::is_same<T, float>::value) {
            if (io) {
                // the FP64 input cast in the same pass
                launch_block_apply3_in64(h->ncell, P_<T>::binv(h), io->in, io->rf, e, s);
                acct(h, gbytes + 8.0 * n);
                have = true;
            }
        }
        if (!have) {
            launch_block_apply<T>(h->ncell, h->bs, P_<T>::binv(h), r, e, false, s);
            acct(h, gbytes);
            have = true;
        }
    }
    // (2) F-relaxation
    have = frelax(have);
    if (!have) {
        P_<T>::fill(e, lv.n, s);
        acct(h, S * n);
    }
    // (3) coarse-grid correction e += P M_c^{-1} R (r - A e); without a global
    // relaxation e is zero on the C points here, so r - A e needs only A's F columns
    if (lv.AcF.v && !global) csr<T>(h, 1, lv.AcF, P_<T>::v(lv.AcF), e, r, nullptr, t);
    else if (l == 0) fine_op<T>(h, 1, e, r, t);
    else csr<T>(h, 1, lv.A, Av, e, r, nullptr, t);
    if (lv.P.nnz == lv.nC && l + 1 < h->L && h->lev[l + 1].fcompact && !io && !om) {
        // e_C += e_c done by the next level's last launch, into e through the C list
        OutMap<T> into;
        into.map = lv.clist;
        into.dst = e;
        coarse_correction(t, &into);
        return;
    }
    coarse_correction(t);
    if constexpr (std::is_same<T, float>::value) {
        if (io && lv.P.nnz == lv.nC) {
            // e_C += e_c and the FP64 output cast in one pass
            launch_scatter_add_out64(lv.n, lv.cmap, ec, e, io->out, s);
            acct(h, 8.0 * n + 4.0 * (double)lv.nC + 8.0 * n);
            return;
        }
    }
    if (lv.P.nnz == lv.nC) {
        // W_p = 0 (every F row of P empty, the C rows the identity): the
        // prolongation is e_C += e_c
        launch_scatter_add<T>(lv.nC, lv.clist, ec, e, s);
        acct(h, 4.0 * (double)lv.nC + 3.0 * S * (double)lv.nC);
    } else {
        csr<T>(h, 2, lv.P, P_<T>::v(lv.P), ec, nullptr, nullptr, e);
    }
    if constexpr (std::is_same<T, float>::value) {
        if (io) {
            launch_cast_f32_f64(e, io->out, lv.n, s);
            acct(h, 12.0 * n);
        }
    }
    if (om) {
        // (not reached by the cycles built here: only compact levels get a map)
        launch_scatter_add<T>(lv.n, om->map, e, om->dst, s);
        acct(h, 4.0 * n + 3.0 * S * n);
    }
}

void apply_prec(mgr_handle *h, const double *v, double *z) {
    if (h->timing) {
        timer_mark(h, h->tm[1]);
        h->vc_bytes = 0;
    }
    if (h->o.precision == 1) {
        float *rf = h->L > 0 ? h->lev[0].rf : h->cg.lev[0].rf;
        float *ef = h->L > 0 ? h->lev[0].ef : h->cg.lev[0].xf;
        if (h->L > 0 && h->bs == 3 && h->o.global_relax && !h->o.cycle_post) {
            // level 0 opens with the cell-block relaxation of r and ends with a
            // prolongation: both casts ride on those passes
            Io64 io;
            io.in = v;
            io.rf = rf;
            io.out = z;
            mgr_cycle<float>(h, 0, rf, ef, false, &io);
        } else {
            launch_cast_f64_f32(v, rf, h->n, h->stream);
            mgr_cycle<float>(h, 0, rf, ef);
            launch_cast_f32_f64(ef, z, h->n, h->stream);
            acct(h, 24.0 * h->n);
        }
    } else {
        mgr_cycle<double>(h, 0, v, z);
    }
    if (h->timing) {
        timer_mark(h, h->tm[1]);
        h->tm[1].bytes += h->vc_bytes;
        h->tm[1].launches++;
    }
}

double dev_norm(mgr_handle *h, const double *a, double *out) {
    launch_norm_part(h->n, a, h->part, h->stream);
    launch_norm_fin(red_blocks(h->n), h->part, out, h->stream);
    return d2h1(h, out);
}

int gmres(mgr_handle *h, const double *b, double *x, double tol, mgr_stats *st) {
    const int64_t n = h->n;
    const int m = h->m;
    const int64_t ld = h->ld;
    hipStream_t s = h->stream;
    double *dsc = h->dsc;
    const int nblk = red_blocks(n);
    int *guard = h->derr + 7;
    const bool lagged = m <= kFusedMaxV;
    if (ld > n) launch_fill_f64(h->w + n, 0.0, ld - n, s);  // a breakdown may have left NaN there
    int its = 0;
    double rel = 0.0;
    if (st) st->res_history_len = 0;
    const double bnorm = dev_norm(h, b, dsc + Dsc::BNORM);
    if (!std::isfinite(bnorm)) return MGR_E_BREAKDOWN;
    if (!h->o.use_x0) launch_fill_f64(x, 0.0, n, s);
    if (bnorm == 0.0) {
        launch_fill_f64(x, 0.0, n, s);
        sync(h);
        if (st) {
            st->iterations = 0;
            st->rel_residual = 0.0;
        }
        return MGR_OK;
    }
    int status = MGR_NOT_CONVERGED;
    for (;;) {
        fine_op<double>(h, 1, x, b, h->res);
        const double beta = dev_norm(h, h->res, dsc + Dsc::BETA);
        rel = beta / bnorm;
        if (!std::isfinite(beta)) {
            status = MGR_E_BREAKDOWN;
            break;
        }
        if (beta <= tol * bnorm) {
            status = MGR_OK;
            break;
        }
        if (its >= h->o.max_iter) {
            status = MGR_NOT_CONVERGED;
            break;
        }
        launch_scale_dev(n, h->res, dsc + Dsc::BETA, 1, h->V, s);
        launch_fill_f64(dsc + Dsc::g(0, m), 0.0, m + 1, s);
        HIPCHK(hipMemcpyAsync(dsc + Dsc::g(0, m), dsc + Dsc::BETA, sizeof(double), hipMemcpyDeviceToDevice, s));
        int k = 0;
        bool broke = false;
        for (int j = 0; j < m; ++j) {
            double *vj = h->V + (int64_t)j * ld;
            double *zj = h->Z + (int64_t)j * ld;
            apply_prec(h, vj, zj);
            fine_op<double>(h, 0, zj, nullptr, h->w);
            if (lagged) {
                // classical Gram-Schmidt twice, the second pass of column j
                // merged with the first pass of w (two reads of the basis)
                launch_lag_dots(n, ld, j + 1, h->V, h->w, h->part, s);
                launch_lag_coef(j, m, nblk, h->part, dsc, s);
                launch_lag_update(n, ld, j + 1, h->V, h->w, dsc, m, h->part, s);
                launch_lag_givens(j, m, nblk, h->part, dsc, s);
            } else {
                // classical Gram-Schmidt; the DGKS second projection runs only when
                // the first one cancelled more than half of ||w||^2 (guard on device)
                launch_mdot(n, ld, j + 1, h->V, h->w, h->part, s);
                launch_arnoldi_fin(0, j, m, nblk, h->part, dsc, guard, s);
                launch_maxpy_dot(n, ld, j + 1, h->V, dsc + Dsc::hcur(0, m), h->w, h->part, s);
                launch_arnoldi_fin(1, j, m, nblk, h->part, dsc, guard, s);
                launch_maxpy_norm(n, ld, j + 1, h->V, dsc + Dsc::h2(0, m), h->w, h->part, guard, s);
                launch_arnoldi_fin(3, j, m, nblk, h->part, dsc, guard, s);
                launch_givens(j, m, dsc, s);
            }
            HIPCHK(hipMemcpyAsync(h->hsc, dsc + Dsc::GABS, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
            sync(h);
            const double gabs = h->hsc[0], hn = h->hsc[1];
            its++;
            if (lagged && h->hsc[2] != 0.0) {
                // the second pass found u_j inside the span of v_0..v_{j-1}: the
                // Krylov space was exhausted at step j-1, which ends the cycle
                k = j;
                break;
            }
            k = j + 1;
            if (st && st->res_history && st->res_history_len < st->res_history_cap)
                st->res_history[st->res_history_len++] = gabs / bnorm;
            if (!std::isfinite(gabs) || !std::isfinite(hn)) {
                broke = true;
                break;
            }
            if (gabs <= tol * bnorm || hn == 0.0 || its >= h->o.max_iter) break;
            if (!lagged) launch_scale_dev(n, h->w, dsc + Dsc::HN, 1, h->V + (int64_t)(j + 1) * ld, s);
        }
        if (broke) {
            status = MGR_E_BREAKDOWN;
            break;
        }
        launch_trisolve(k, m, dsc, s);
        if (lagged) launch_lag_yscale(k, m, dsc, s);
        launch_zaxpy(n, ld, k, h->Z, dsc + Dsc::y(0, m), x, s);
    }
    sync(h);
    if (st) {
        st->iterations = its;
        st->rel_residual = rel;
    }
    return status;
}

void fill_stats(mgr_handle *h, mgr_stats *st) {
    if (!st) return;
    st->setup_ms = h->setup_ms;
    int k = 0;
    for (auto &lv : h->lev)
        if (k < 64) {
            st->level_n[k] = lv.A.nrows;
            st->level_nnz[k] = lv.A.nnz;
            k++;
        }
    for (auto &lv : h->cg.lev)
        if (k < 64) {
            st->level_n[k] = lv.A.nrows;
            st->level_nnz[k] = lv.A.nnz;
            k++;
        }
    st->n_levels = k;
}

// Small pinned host blocks for the per-handle read-back words, kept for the life
// of the process: pinning and unpinning cost milliseconds each, far more than a
// handle's setup would otherwise spend on them.
constexpr size_t kPinnedBlock = 256;
std::mutex g_pinned_mu;
std::vector<void *> g_pinned_free;

void *pinned_get(mgr_handle *h) {
    {
        std::lock_guard<std::mutex> lk(g_pinned_mu);
        if (!g_pinned_free.empty()) {
            void *p = g_pinned_free.back();
            g_pinned_free.pop_back();
            return p;
        }
    }
    void *p = nullptr;
    HIPCHK(hipHostMalloc(&p, kPinnedBlock, hipHostMallocDefault));
    return p;
}

void pinned_put(void *p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_pinned_mu);
    g_pinned_free.push_back(p);
}

}  // namespace

// blocks still held (a handle that never reached the device cache, or the
// temporary handle of a handle-free entry point): back to the pool, in order
mgr_handle::~mgr_handle() {
    for (auto &b : spare) (void)hipFreeAsync(b.second, stream);
}

namespace {

void destroy_impl(mgr_handle *h) {
    if (!h) return;
    arena_release(h, h->scratch);
    arena_release(h, h->amg);
    arena_release(h, h->keep);
    if (hipStreamSynchronize(h->stream) == hipSuccess) blocks_to_cache(h);
    for (auto &t : h->tm)
        for (auto e : t.ev) (void)hipEventDestroy(e);
    pinned_put(h->hsc);
    pinned_put(h->herr);
    delete h;
}

int check_options(const mgr_options *o, std::string &why) {
    if (o->precision != 0 && o->precision != 1) why = "precision must be 0 or 1";
    else if (o->restart < 1 || o->restart > 64) why = "restart must be in [1, 64]";
    else if (o->max_iter < 0) why = "max_iter must be >= 0";
    else if (o->rp_type < 0 || o->rp_type > 2) why = "rp_type must be 0, 1 or 2";
    else if (o->f_sweeps < 0 || o->f_sweeps > 8) why = "f_sweeps must be in [0, 8]";
    else if (!(o->amg_theta >= 0.0 && o->amg_theta < 1.0)) why = "amg_theta must be in [0, 1)";
    else if (o->amg_pre < 0 || o->amg_pre > 8 || o->amg_post < 0 || o->amg_post > 8) why = "amg_pre/post in [0, 8]";
    else if (o->amg_max_levels < 1 || o->amg_max_levels > 32) why = "amg_max_levels must be in [1, 32]";
    else if (o->amg_coarse_max < 1) why = "amg_coarse_max must be >= 1";
    else if (o->dense_max < 1 || o->dense_max > 4096) why = "dense_max must be in [1, 4096]";
    else if (o->frelax_amg_mask < 0) why = "frelax_amg_mask must be >= 0";
    else if (o->frelax_amg_pre < 0 || o->frelax_amg_pre > 8 || o->frelax_amg_post < 0 || o->frelax_amg_post > 8)
        why = "frelax_amg_pre/post in [0, 8]";
    else if (o->cycle_post != 0 && o->cycle_post != 1) why = "cycle_post must be 0 or 1";
    else if (o->index16 != 0 && o->index16 != 1) why = "index16 must be 0 or 1";
    else return MGR_OK;
    return MGR_E_INVALID;
}

// Value update of MGR level l (same pattern and labels as at setup): D_FF^{-1},
// the F-row copies, W_p and W_r in P and R, and A_{l+1} = R (A P), each written
// over its arrays (the patterns, level maps and row pointers are kept); the AMG
// F-relaxation hierarchy on A_FF is built anew, since its coarsening depends on
// the values.  The same kernels as the setup, in the same order: the result is
// bitwise the setup's.
void update_mgr_level(mgr_handle *h, int l, DCsr &Anext) {
    MgrLevel &lv = h->lev[l];
    const DCsr &A = lv.A;
    const int sel = select_lanes(A.nrows, A.nnz);
    ScratchScope scope(h);
    fdiag_inverse(h, l);
    if (lv.AF.v) launch_ff_fill(sel, lv.nF, lv.flist, A.rp, A.ci, A.v, nullptr, lv.AF.rp, lv.AF.ci, lv.AF.v, h->stream);
    if (lv.AcF.v)
        launch_fcol_fill(sel, lv.n, A.rp, A.ci, A.v, lv.fmap, lv.AcF.rp, lv.AcF.ci, lv.AcF.v, lv.fcompact, h->stream);
    if (lv.Aff.v) {  // the level relaxes its F points with an AMG cycle on A_FF
        launch_ff_fill(sel, lv.nF, lv.flist, A.rp, A.ci, A.v, lv.fmap, lv.Aff.rp, lv.Aff.ci, lv.Aff.v, h->stream);
        lv.ff = std::make_shared<AmgHier>();
        AmgArenaScope amg_arena(h);
        build_amg(h, *lv.ff, lv.Aff, h->o.frelax_amg_pre, h->o.frelax_amg_post);
    }
    const int rp_type = h->o.rp_type;
    launch_p_fill(sel, lv.n, A.rp, A.ci, A.v, lv.cmap, lv.fmap, lv.dinv, rp_type, lv.P.rp, lv.P.ci, lv.P.v, h->stream);
    launch_r_fill(lv.nC, lv.clist, A.rp, A.ci, A.v, lv.fmap, lv.dinv, rp_type, lv.R.rp, lv.R.ci, lv.R.v,
                  h->stream);
    DCsr T = spgemm(h, A, lv.P, true);
    spgemm_values(h, lv.R, T, Anext);
}

// New values on the setup's pattern and labels: everything that depends only on
// them (the validated pattern, level maps, sliced-ELL layout, the patterns of
// P, R, the F-row copies and the reduced operators, the Krylov workspace) is
// kept; the values are recomputed in place, and the AMG hierarchies are built
// anew in their own arena.
void update_impl(mgr_handle *h, const double *values) {
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = h->stream;
    if (h->Ain.nnz > 0)
        HIPCHK(hipMemcpyAsync(h->Ain.v, values, h->Ain.nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (h->o.transpose) transpose_values(h, h->Ain, h->A0);
    const CSell &S = h->A0s;
    launch_csell_fill(S.ncell, S.bs, h->A0.rp, h->A0.ci, h->A0.v, S.off, S.width, S.col, S.v, s);
    if (h->binv) {
        reset_err(h);
        launch_block_inverse(h->ncell, h->bs, h->A0.rp, h->A0.ci, h->A0.v, h->binv, h->derr, s);
        read_err(h);
        if (h->herr[3] != INT_MAX)
            throw_err(h, MGR_E_SINGULAR_BLOCK, "singular diagonal cell block at cell " + std::to_string(h->herr[3]));
    }
    // the previous AMG hierarchies (stream-ordered release: every kernel that
    // reads them is queued before the kernels that reuse the memory)
    for (auto &lv : h->lev) lv.ff.reset();
    h->cg = AmgHier();
    arena_release(h, h->amg);
    for (int l = 0; l < h->L; ++l) update_mgr_level(h, l, l + 1 < h->L ? h->lev[l + 1].A : h->AL);
    {
        AmgArenaScope amg_arena(h);
        build_amg(h, h->cg, h->AL, h->o.amg_pre, h->o.amg_post);
    }
    if (h->o.precision == 1) to_mixed(h, true);
    alloc_work(h, true);
    build_tails(h);
    arena_release(h, h->scratch);
    sync(h);
    h->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

int setup_impl(const mgr_csr *Ain, int bs, const int32_t *labels, const mgr_options *opts, mgr_handle **out) {
    *out = nullptr;
    std::string why;
    if (!Ain || !labels || !opts) {
        g_err = "null argument";
        return MGR_E_INVALID;
    }
    if (Ain->n <= 0 || Ain->nnz < 0 || Ain->nnz > INT_MAX || Ain->n > INT_MAX / 4 || (bs != 1 && bs != 3) ||
        Ain->n % bs != 0 || !Ain->row_ptr || (Ain->nnz > 0 && (!Ain->col_idx || !Ain->values))) {
        g_err = "invalid matrix size, block size or pointer";
        return MGR_E_INVALID;
    }
    if (check_options(opts, why) != MGR_OK) {
        g_err = why;
        return MGR_E_INVALID;
    }
    mgr_handle *h = new (std::nothrow) mgr_handle();
    if (!h) {
        g_err = "host allocation failed";
        return MGR_E_OOM;
    }
    try {
        auto t0 = std::chrono::steady_clock::now();
        h->stream = (hipStream_t)opts->stream;
        HIPCHK(hipGetDevice(&h->device));
        h->o = *opts;
        h->n = Ain->n;
        h->bs = bs;
        h->ncell = Ain->n / bs;
        h->m = opts->restart;
        h->herr = static_cast<int *>(pinned_get(h));
        h->hsc = static_cast<double *>(pinned_get(h));
        h->derr = dalloc<int>(h, 8);
        const int64_t n = Ain->n, nnz = Ain->nnz;
        // pattern and labels
        int32_t ends[2];
        HIPCHK(hipMemcpyAsync(&ends[0], Ain->row_ptr, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipMemcpyAsync(&ends[1], Ain->row_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
        sync(h);
        if (ends[0] != 0 || ends[1] != nnz) throw_err(h, MGR_E_INVALID, "row_ptr[0] != 0 or row_ptr[n] != nnz");
        reset_err(h);
        launch_validate(n, nnz, Ain->row_ptr, Ain->col_idx, labels, h->derr, h->stream);
        read_err(h);
        if (h->herr[0]) throw_err(h, MGR_E_INVALID, "row pointers or column indices invalid (need sorted, unique, in range)");
        if (h->herr[2]) throw_err(h, MGR_E_INVALID, "cf_labels outside [0, 31]");
        h->L = h->herr[1];
        // private copy of A
        DCsr &A = h->Ain;
        A.nrows = A.ncols = n;
        A.nnz = nnz;
        A.rp = dalloc<int32_t>(h, n + 1);
        A.ci = dalloc<int32_t>(h, nnz);
        A.v = dalloc<double>(h, nnz);
        HIPCHK(hipMemcpyAsync(A.rp, Ain->row_ptr, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, h->stream));
        if (nnz > 0) {
            HIPCHK(hipMemcpyAsync(A.ci, Ain->col_idx, nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, h->stream));
            HIPCHK(hipMemcpyAsync(A.v, Ain->values, nnz * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
        }
        h->A0 = opts->transpose ? transpose(h, A, true) : A;
        build_csell(h);
        if (opts->global_relax && h->L > 0) {
            h->binv = dalloc<double>(h, h->ncell * bs * bs);
            reset_err(h);
            launch_block_inverse(h->ncell, bs, h->A0.rp, h->A0.ci, h->A0.v, h->binv, h->derr, h->stream);
            read_err(h);
            if (h->herr[3] != INT_MAX)
                throw_err(h, MGR_E_SINGULAR_BLOCK, "singular diagonal cell block at cell " + std::to_string(h->herr[3]));
        }
        DCsr Acur = h->A0;
        int32_t *lab = dalloc<int32_t>(h, n);
        int32_t *glob = dalloc<int32_t>(h, n);
        HIPCHK(hipMemcpyAsync(lab, labels, n * sizeof(int32_t), hipMemcpyDeviceToDevice, h->stream));
        launch_iota(glob, n, h->stream);
        h->lev.resize(h->L);
        for (int l = 0; l < h->L; ++l) {
            h->lev[l].A = Acur;
            h->lev[l].lab = lab;
            h->lev[l].glob = glob;
            DCsr An;
            build_mgr_level(h, l, An, lab, glob);
            Acur = An;
        }
        h->AL = Acur;
        {
            AmgArenaScope amg_arena(h);
            build_amg(h, h->cg, Acur, opts->amg_pre, opts->amg_post);
        }
        if (h->o.precision == 1) to_mixed(h);
        alloc_work(h);
        build_tails(h);
        const int m = h->m;
        h->ld = krylov_ld(n);
        h->V = dalloc<double>(h, (int64_t)(m + 1) * h->ld);
        h->Z = dalloc<double>(h, (int64_t)m * h->ld);
        h->w = dalloc<double>(h, h->ld);
        // the padding of V and w beyond n stays zero (the basis kernels read it)
        launch_fill_f64(h->V, 0.0, (int64_t)(m + 1) * h->ld, h->stream);
        launch_fill_f64(h->w, 0.0, h->ld, h->stream);
        h->res = dalloc<double>(h, n);
        h->dsc = dalloc<double>(h, Dsc::size(m));
        launch_fill_f64(h->dsc, 0.0, Dsc::size(m), h->stream);
        h->part = dalloc<double>(h, (int64_t)kRedBlocks * 130);
        arena_release(h, h->scratch);
        sync(h);
        h->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        *out = h;
        return MGR_OK;
    } catch (...) {
        const int rc = abi_status(nullptr);
        destroy_impl(h);
        return rc;
    }
}

}  // namespace

namespace mgr {
// Device memory comes from one stream-ordered pool per device, owned by the
// library: allocations and releases are queued on the handle's stream (no
// device-wide synchronisation, no driver call once the pool is warm), and memory
// a handle releases stays in the pool for later handles in the process.
int pool_alloc(mgr_handle *h, void **p, size_t bytes) {
    static std::mutex mu;
    static std::map<int, hipMemPool_t> pools;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MGR_E_HIP;
    hipMemPool_t pool = nullptr;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = pools.find(dev);
        if (it == pools.end()) {
            hipMemPoolProps props{};
            props.allocType = hipMemAllocationTypePinned;
            props.location.type = hipMemLocationTypeDevice;
            props.location.id = dev;
            if (hipMemPoolCreate(&pool, &props) != hipSuccess) return MGR_E_HIP;
            uint64_t keep = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
            pools[dev] = pool;
        } else {
            pool = it->second;
        }
    }
    if (hipMallocFromPoolAsync(p, bytes, pool, h->stream) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return MGR_E_OOM;
    }
    return MGR_OK;
}

int alloc(mgr_handle *h, void **p, size_t bytes) {
    try {
        *p = arena_alloc(h, h->live ? *h->live : h->keep, bytes);
        return MGR_OK;
    } catch (...) {
        *p = nullptr;
        return abi_status(h);
    }
}
}  // namespace mgr

extern "C" {

void mgr_default_options(mgr_options *o) {
    std::memset(o, 0, sizeof *o);
    o->stream = nullptr;
    o->precision = 0;
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
    o->transpose = 0;
    o->use_x0 = 0;
    o->frelax_amg_mask = 0;
    o->frelax_amg_pre = 1;
    o->frelax_amg_post = 1;
    o->cycle_post = 0;
    o->index16 = 1;
}

int mgr_setup(const mgr_csr *A, int block_size, const int32_t *cf_labels, const mgr_options *opts,
              mgr_handle **out) {
    if (!out) {
        g_err = "null output handle pointer";
        return MGR_E_INVALID;
    }
    return setup_impl(A, block_size, cf_labels, opts, out);
}

int mgr_update_values(mgr_handle *h, const double *values) {
    if (!h || (h->Ain.nnz > 0 && !values)) {
        g_err = "invalid update arguments";
        if (h) h->err = g_err;
        return MGR_E_INVALID;
    }
    try {
        update_impl(h, values);
        return MGR_OK;
    } catch (...) {
        return abi_status(h);
    }
}

int mgr_solve(mgr_handle *h, const double *b, double *x, double tol, mgr_stats *st) {
    if (!h || !b || !x || !(tol >= 0.0)) {
        g_err = "invalid solve arguments";
        if (h) h->err = g_err;
        return MGR_E_INVALID;
    }
    try {
        auto t0 = std::chrono::steady_clock::now();
        int rc = gmres(h, b, x, tol, st);
        if (st) {
            st->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            fill_stats(h, st);
        }
        if (rc == MGR_E_BREAKDOWN) h->err = "NaN or Inf in the right-hand side or the Krylov recurrence";
        return rc;
    } catch (...) {
        return abi_status(h);
    }
}

int mgr_pattern_outer(mgr_handle *h, const double *lambda, const double *x, double *dvals) {
    if (!h || !lambda || !x || !dvals) return MGR_E_INVALID;
    try {
        launch_pattern_outer(h->Ain.nrows, h->Ain.rp, h->Ain.ci, lambda, x, dvals, h->stream);
        HIPCHK(hipGetLastError());
        return MGR_OK;
    } catch (...) {
        return abi_status(h);
    }
}

int mgr_apply_preconditioner(mgr_handle *h, const double *r, double *z) {
    if (!h || !r || !z) return MGR_E_INVALID;
    try {
        apply_prec(h, r, z);
        sync(h);
        return MGR_OK;
    } catch (...) {
        return abi_status(h);
    }
}

int mgr_spmv(mgr_handle *h, const double *x, double *y) {
    if (!h || !x || !y) return MGR_E_INVALID;
    try {
        fine_op<double>(h, 0, x, nullptr, y);
        sync(h);
        return MGR_OK;
    } catch (...) {
        return abi_status(h);
    }
}

void mgr_destroy(mgr_handle *h) { destroy_impl(h); }

const char *mgr_status_string(int code) {
    switch (code) {
    case MGR_OK: return "MGR_OK";
    case MGR_NOT_CONVERGED: return "MGR_NOT_CONVERGED";
    case MGR_E_INVALID: return "MGR_E_INVALID";
    case MGR_E_ZERO_FDIAG: return "MGR_E_ZERO_FDIAG";
    case MGR_E_SINGULAR_BLOCK: return "MGR_E_SINGULAR_BLOCK";
    case MGR_E_BREAKDOWN: return "MGR_E_BREAKDOWN";
    case MGR_E_HIP: return "MGR_E_HIP";
    case MGR_E_OOM: return "MGR_E_OOM";
    }
    return "unknown status";
}

const char *mgr_last_error(const mgr_handle *h) { return h ? h->err.c_str() : g_err.c_str(); }

int mgr_num_levels(mgr_handle *h, int *nm, int *na) {
    if (!h) return MGR_E_INVALID;
    if (nm) *nm = h->L;
    if (na) *na = (int)h->cg.lev.size();
    return MGR_OK;
}

// the AMG hierarchy a query refers to: the F-relaxation AMG of MGR level
// (level >> 8) for the F-block kinds (level becomes its low byte), else the coarse grid
static AmgHier *query_hier(mgr_handle *h, bool ff_kind, int &level) {
    if (!ff_kind) return &h->cg;
    const int l = level >> 8;
    level &= 0xff;
    if (l < 0 || l >= h->L || !h->lev[l].ff) return nullptr;
    return h->lev[l].ff.get();
}

int mgr_get_matrix(mgr_handle *h, int kind, int level, int64_t *nrows, int64_t *ncols, int64_t *nnz,
                   int32_t *row_ptr, int32_t *col_idx, double *values) {
    if (!h) return MGR_E_INVALID;
    const DCsr *M = nullptr;
    if (kind >= 0 && kind <= 2) {
        if (level < 0 || level >= h->L) return MGR_E_INVALID;
        M = kind == 0 ? &h->lev[level].A : kind == 1 ? &h->lev[level].P : &h->lev[level].R;
    } else if (kind >= 3 && kind <= 7) {
        AmgHier *H = query_hier(h, kind >= 6, level);
        if (!H) return MGR_E_INVALID;
        const int na = (int)H->lev.size();
        if (kind == 3 || kind == 6) {
            if (level < 0 || level >= na) return MGR_E_INVALID;
            M = &H->lev[level].A;
        } else {
            if (level < 0 || level >= na - 1) return MGR_E_INVALID;
            M = (kind == 4 || kind == 7) ? &H->lev[level].P : &H->lev[level].S;
        }
    } else {
        return MGR_E_INVALID;
    }
    if (nrows) *nrows = M->nrows;
    if (ncols) *ncols = M->ncols;
    if (nnz) *nnz = M->nnz;
    if (!row_ptr) return MGR_OK;
    try {
        sync(h);
        HIPCHK(hipMemcpy(row_ptr, M->rp, (M->nrows + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
        if (col_idx && M->nnz) HIPCHK(hipMemcpy(col_idx, M->ci, M->nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
        if (values && M->v && M->nnz) HIPCHK(hipMemcpy(values, M->v, M->nnz * sizeof(double), hipMemcpyDeviceToHost));
        return MGR_OK;
    } catch (...) {
        return abi_status(h);
    }
}

int mgr_get_vector(mgr_handle *h, int kind, int level, void *out, int64_t *len) {
    if (!h || !len) return MGR_E_INVALID;
    const void *src = nullptr;
    size_t esz = 8;
    int64_t n = -1;
    if (kind >= 0 && kind <= 3) {
        switch (kind) {
        case 0: n = h->binv ? h->ncell * h->bs * h->bs : 0; src = h->binv; break;
        case 1: if (level >= 0 && level < h->L) { n = h->lev[level].nF; src = h->lev[level].dinv; } break;
        case 2: if (level >= 0 && level < h->L) { n = h->lev[level].nF; src = h->lev[level].flist; esz = 4; } break;
        case 3: if (level >= 0 && level < h->L) { n = h->lev[level].nC; src = h->lev[level].clist; esz = 4; } break;
        }
    } else if (kind >= 4 && kind <= 11) {
        AmgHier *H = query_hier(h, kind >= 8, level);
        const int base = kind >= 8 ? kind - 4 : kind;
        if (H) {
            const int na = (int)H->lev.size();
            switch (base) {
            case 4: if (level >= 0 && level < na - 1) { n = H->lev[level].n; src = H->lev[level].cf; esz = 4; } break;
            case 5: if (level >= 0 && level < na - 1) { n = H->lev[level].n; src = H->lev[level].l1; } break;
            case 6: n = H->ncoarse * H->ncoarse; src = H->lu; break;
            case 7: n = H->ncoarse; src = H->perm; esz = 4; break;
            }
        }
    }
    if (n < 0) return MGR_E_INVALID;
    *len = n;
    if (!out || n == 0) return MGR_OK;
    try {
        sync(h);
        if (kind == 0) {
            // device planes -> row-major 3x3 (or 1x1) per cell
            const int bb = h->bs * h->bs;
            std::vector<double> planes(n);
            HIPCHK(hipMemcpy(planes.data(), src, n * sizeof(double), hipMemcpyDeviceToHost));
            double *o = static_cast<double *>(out);
            for (int64_t c = 0; c < h->ncell; ++c)
                for (int k = 0; k < bb; ++k) o[c * bb + k] = planes[(int64_t)k * h->ncell + c];
        } else {
            HIPCHK(hipMemcpy(out, src, n * esz, hipMemcpyDeviceToHost));
        }
        return MGR_OK;
    } catch (...) {
        return abi_status(h);
    }
}

static int check_ncp_csr(const mgr_csr *L) {
    if (!L || L->n <= 0 || L->n % 3 != 0 || L->nnz < 0 || !L->row_ptr || (L->nnz > 0 && (!L->col_idx || !L->values))) {
        g_err = "L must be a CSR with 3 rows per cell";
        return MGR_E_INVALID;
    }
    return MGR_OK;
}

int mgr_ncp_eval(const mgr_csr *L, const double *henry, const double *f, double *u, const double *du, double alpha,
                 double *R, int32_t *labels, double *rnorm, int64_t *nactive, int64_t *nchanged, void *stream) {
    if (check_ncp_csr(L) != MGR_OK) return MGR_E_INVALID;
    if (!henry || !f || !u || !R || !labels) {
        g_err = "null argument";
        return MGR_E_INVALID;
    }
    mgr_handle t;
    t.stream = (hipStream_t)stream;
    mgr_handle *h = &t;
    ScratchScope scope(h);
    try {
        const int64_t n = L->n, ncell = n / 3;
        if (du) launch_axpy_inplace(n, alpha, du, u, h->stream);
        Tmp<int> cnt(h, 2);  // active cells, cells whose labels changed
        launch_fill_i32(cnt.p, 0, 2, h->stream);
        launch_ncp_eval(ncell, L->row_ptr, L->col_idx, L->values, henry, f, u, R, labels, cnt.p, cnt.p + 1,
                        h->stream);
        Tmp<double> part(h, kRedBlocks + 1);
        launch_norm_part(n, R, part.p, h->stream);
        launch_norm_fin(red_blocks(n), part.p, part.p + kRedBlocks, h->stream);
        double rn = 0.0;
        int na[2] = {0, 0};
        HIPCHK(hipMemcpyAsync(&rn, part.p + kRedBlocks, sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipMemcpyAsync(na, cnt.p, 2 * sizeof(int), hipMemcpyDeviceToHost, h->stream));
        sync(h);
        if (rnorm) *rnorm = rn;
        if (nactive) *nactive = na[0];
        if (nchanged) *nchanged = na[1];
        return std::isfinite(rn) ? MGR_OK : MGR_E_BREAKDOWN;
    } catch (...) {
        return abi_status(nullptr);
    }
}

}  // extern "C"

// Allocation-free form of mgr_ncp_eval.  Its device scratch (the partial sums
// of the residual norm, the norm itself and the two cell counters) lives in a
// file-scope array instead of the stream-ordered pool.  On the host the name
// `scratch` is only a stand-in; the array's device address comes from
// hipGetSymbolAddress, once per device with that device current, and only
// that address is ever handed to kernels.
static constexpr size_t kStaticScratchBytes = 16384;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device (resolved on first use).
int static_scratch(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        g_err = "no current HIP device";
        return MGR_E_HIP;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            g_err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return MGR_E_HIP;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return MGR_OK;
}
}  // namespace

extern "C" {

int mgr_ncp_eval_noalloc(const mgr_csr *L, const double *henry, const double *f, double *u, const double *du,
                         double alpha, double *R, int32_t *labels, double *rnorm, int64_t *nactive,
                         int64_t *nchanged, void *stream) {
    if (check_ncp_csr(L) != MGR_OK) return MGR_E_INVALID;
    if (!henry || !f || !u || !R || !labels) {
        g_err = "null argument";
        return MGR_E_INVALID;
    }
    const int64_t n = L->n, ncell = n / 3;
    const int nblk = red_blocks(n);
    // layout: the norm's partial sums, then the norm, then the two counters
    const size_t need = ((size_t)nblk + 1) * sizeof(double) + 2 * sizeof(int);
    if (need > kStaticScratchBytes || nblk > kRedBlocks) {
        g_err = "mgr_ncp_eval_noalloc: needs " + std::to_string(need) + " bytes of static scratch, capacity " +
                std::to_string(kStaticScratchBytes);
        return MGR_E_INVALID;
    }
    void *base = nullptr;
    if (const int rc = static_scratch(&base); rc != MGR_OK) return rc;
    double *part = static_cast<double *>(base);
    double *norm = part + nblk;
    int *cnt = reinterpret_cast<int *>(norm + 1);
    const hipStream_t s = (hipStream_t)stream;
    if (du) launch_axpy_inplace(n, alpha, du, u, s);
    launch_fill_i32(cnt, 0, 2, s);  // a fill kernel: the counters start at zero on every call
    launch_ncp_eval(ncell, L->row_ptr, L->col_idx, L->values, henry, f, u, R, labels, cnt, cnt + 1, s);
    launch_norm_part(n, R, part, s);
    launch_norm_fin(nblk, part, norm, s);
    double rn = 0.0;
    int na[2] = {0, 0};
    hipError_t e = hipMemcpyAsync(&rn, norm, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(na, cnt, 2 * sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) {
        g_err = std::string("mgr_ncp_eval_noalloc: ") + hipGetErrorString(e);
        return MGR_E_HIP;
    }
    if (rnorm) *rnorm = rn;
    if (nactive) *nactive = na[0];
    if (nchanged) *nchanged = na[1];
    return std::isfinite(rn) ? MGR_OK : MGR_E_BREAKDOWN;
}

int mgr_ncp_jacobian(const mgr_csr *L, const double *henry, const int32_t *labels, int32_t *row_ptr,
                     int32_t *col_idx, double *values, int64_t capacity, int64_t *nnz, void *stream) {
    if (check_ncp_csr(L) != MGR_OK) return MGR_E_INVALID;
    if (!henry || !labels || !row_ptr || !col_idx || !values) {
        g_err = "null argument";
        return MGR_E_INVALID;
    }
    mgr_handle t;
    t.stream = (hipStream_t)stream;
    mgr_handle *h = &t;
    ScratchScope scope(h);
    try {
        const int64_t n = L->n;
        Tmp<int32_t> cnt(h, n);
        launch_ncp_jac_count(n, L->row_ptr, labels, cnt.p, h->stream);
        const int64_t total = scan(h, cnt.p, row_ptr, n);
        if (nnz) *nnz = total;
        if (total > capacity) throw_err(h, MGR_E_INVALID, "Jacobian needs " + std::to_string(total) +
                                                              " entries, capacity " + std::to_string(capacity));
        launch_ncp_jac_fill(n, L->row_ptr, L->col_idx, L->values, henry, labels, row_ptr, col_idx, values,
                            h->stream);
        sync(h);
        return MGR_OK;
    } catch (...) {
        return abi_status(nullptr);
    }
}

int mgr_set_kernel_timing(mgr_handle *h, int on) {
    if (!h) return MGR_E_INVALID;
    h->timing = on != 0;
    for (auto &t : h->tm) {
        t.used = 0;
        t.bytes = 0;
        t.launches = 0;
    }
    return MGR_OK;
}

int mgr_kernel_time(mgr_handle *h, int kernel, double *total_ms, int64_t *launches, double *bytes_total) {
    if (!h || kernel < 0 || kernel > 2) return MGR_E_INVALID;
    try {
        sync(h);
        mgr_handle::Timer &t = h->tm[kernel];
        double tot = 0.0;
        for (size_t i = 0; i + 1 < t.used; i += 2) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, t.ev[i], t.ev[i + 1]));
            tot += ms;
        }
        if (total_ms) *total_ms = tot;
        if (launches) *launches = t.launches;
        if (bytes_total) *bytes_total = t.bytes;
        t.used = 0;
        t.bytes = 0;
        t.launches = 0;
        return MGR_OK;
    } catch (...) {
        return abi_status(h);
    }
}

}  // extern "C"
