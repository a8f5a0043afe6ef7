// Solve-phase kernels: CSR SpMV variants for the coarser MGR levels, R, P and
// the AMG levels, the relaxations of the MGR V-cycle and the coarsest dense
// solve.  Templated on the value type (double, or float for the mixed-precision
// hierarchy).  The stream kernel sums each row in ascending column order in one
// thread; the multi-lane kernels reduce strided partial sums across lanes, which
// reorders the additions only.
#include "mgr_impl.h"

namespace mgr {
namespace {

__device__ inline int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }

// Workgroups are dealt to the 8 XCDs round-robin.  Renumber them so that each
// XCD takes G consecutive row blocks before moving on (G blocks of kXcdGroupRows
// rows in all: one 128 x 128 grid plane, whose neighbours' x values then stay in
// that XCD's L2); a tail shorter than 8 groups keeps the plain order.
constexpr int64_t kXcdGroupRows = 16384;
template <int64_t G>
__device__ inline int64_t xcd_grouped_block() {
    const int64_t b = blockIdx.x, span = 8 * G;
    if (b >= (int64_t)gridDim.x / span * span) return b;
    const int64_t xcd = b % 8, i = b / 8;
    return ((i / G) * 8 + xcd) * G + i % G;
}

// CSR "stream" SpMV: a workgroup owns ROWS consecutive rows.  Their nonzeros are
// read as one contiguous, coalesced stream in passes of LDSN entries; in a
// pass each thread issues the column and value loads of all its entries before
// their dependent gathers of x, and stages the products v*x in LDS (other
// workgroups on the CU overlap a pass's loads with its row sums; issuing the
// next pass's loads early costs more in registers than it saves).  Then thread t
// sums row rb+t sequentially in ascending column order (a row's entries may span
// several passes, which run in ascending order).  No padding, any row-length mix,
// and the same summation order per row as a sequential CSR loop.  The matrix is
// streamed with non-temporal loads so that it does not evict x from the caches.
// Modes: 0 y = Ax; 1 y = r - Ax; 2 y += Ax; 3 y = x + (r - Ax)/d (Jacobi sweep);
// 4 y = Ax and y2 = y/d (a restriction that also forms the next level's first
// Jacobi iterate from zero, the division the separate pass would do).
// LDSN (entries per pass) follows the matrix's mean row length: short-row
// operators (P, R, the F-blocks) fill a 4096-entry pass only partly, and a
// smaller pass lets more workgroups share a CU.

// The per-row operands of the output step (the lanes kernel loads them before
// the row's sum so that their latency overlaps it).
// Mode 5 (y = e_F + A x, the prolongation that also writes the F-relaxation's
// correction, kept compact by F index, with zeros on the C points): r holds the
// compact correction and d carries the int32 F index map (-1 on C points).
// Mode 6: the same value added into the finer level's vector, y[m[row]] +=
// (e_F + A x), with the int32 map m carried by y2 (the W_p = 0 prolongation of
// the finer level done by this level's last launch).
template <typename T, int MODE>
struct RowIn {
    T a = 0, b = 0, c = 0;
    __device__ inline void load(int64_t row, const T *__restrict__ x, const T *__restrict__ r,
                                const T *__restrict__ d, const T *__restrict__ y) {
        if (MODE == 1) a = r[row];
        if (MODE == 2) a = y[row];
        if (MODE == 5 || MODE == 6) {
            const int f = reinterpret_cast<const int32_t *>(d)[row];
            a = f >= 0 ? r[f] : (T)0;
        }
        if (MODE == 3) {
            a = x[row];
            b = r[row];
        }
        if (MODE == 3 || MODE == 4) c = d[row];
    }
    __device__ inline void store(int64_t row, T acc, T *__restrict__ y, T *__restrict__ y2) const {
        if (MODE == 0) y[row] = acc;
        else if (MODE == 1) y[row] = a - acc;
        else if (MODE == 2 || MODE == 5) y[row] = a + acc;
        else if (MODE == 6) {
            const int64_t j = reinterpret_cast<const int32_t *>(y2)[row];
            const T v = a + acc;
            y[j] = y[j] + v;
        }
        else if (MODE == 3) y[row] = a + (b - acc) / c;
        else {
            y[row] = acc;
            y2[row] = acc / c;
        }
    }
};

template <typename T, int MODE, int ROWS, int NT, int LDSN>
__global__ void __launch_bounds__(NT) k_csr_stream(int64_t nrows, const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ ci, const T *__restrict__ v,
                                                   const T *__restrict__ x, const T *__restrict__ r,
                                                   const T *__restrict__ d, T *__restrict__ y,
                                                   T *__restrict__ y2) {
    static_assert(NT >= ROWS && LDSN % NT == 0, "stream kernel shape");
    constexpr int B = LDSN / NT;  // entries per thread per pass
    __shared__ T sh[LDSN];
    const int tid = threadIdx.x;
    const int64_t rb = xcd_grouped_block<kXcdGroupRows / ROWS>() * ROWS;
    const int64_t re = rb + ROWS < nrows ? rb + ROWS : nrows;
    // threads below ROWS own a row each; all NT threads load and multiply
    const int64_t row = rb + tid;
    const bool owner = tid < ROWS && row < re;
    const int p0 = rp[rb], p1 = rp[re];
    // the row's output operands: loaded up front in FP32 (the registers are
    // there), after the passes in FP64 (where they would cost a wave per SIMD)
    constexpr bool kEarlyRowIn = sizeof(T) == 4;
    int a = 0, b = 0;
    RowIn<T, MODE> in;
    if (owner) {
        a = rp[row];
        b = rp[row + 1];
        if (kEarlyRowIn) in.load(row, x, r, d, y);
    }
    T acc = 0;
    int j[B];
    T av[B];
    auto load_pass = [&](int base) {
        const int lim = base + LDSN < p1 ? base + LDSN : p1;
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int p = base + u * NT + tid;
            j[u] = p < lim ? __builtin_nontemporal_load(ci + p) : -1;
            av[u] = p < lim ? __builtin_nontemporal_load(v + p) : (T)0;
        }
    };
    for (int base = p0; base < p1; base += LDSN) {
        const int lim = base + LDSN < p1 ? base + LDSN : p1;
        load_pass(base);
        T xv[B];
#pragma unroll
        for (int u = 0; u < B; ++u) xv[u] = j[u] >= 0 ? x[j[u]] : (T)0;
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int p = base + u * NT + tid;
            if (p < lim) sh[p - base] = av[u] * xv[u];
        }
        __syncthreads();
        const int lo = a > base ? a : base, hi = b < lim ? b : lim;
        // the row's products in ascending order; eight LDS reads are issued
        // before their additions so that a long row waits for LDS once per eight
        // entries instead of once per entry
        int p = lo;
        for (; p + 8 <= hi; p += 8) {
            T s[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) s[u] = sh[p - base + u];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc = acc + s[u];
        }
        for (; p < hi; ++p) acc = acc + sh[p - base];
        __syncthreads();
    }
    if (owner) {
        if (!kEarlyRowIn) in.load(row, x, r, d, y);
        in.store(row, acc, y, y2);
    }
}

// The same products and row sums over a matrix's row-block jagged copy (Jag):
// the entries of a block of kJagRows rows are streamed in passes of LDSN as in
// the CSR stream kernel, but in slot order, so the lanes of a wavefront gather x
// at one stencil slot of consecutive rows.  Thread s owns the row of rank s and
// adds its products in ascending slot (= ascending column) order: the sums are
// those of the CSR stream kernel, bit for bit.  The block's slot table sits in
// LDS; a row's entry k is at st[k] + s, so the owner threads read consecutive
// LDS words.
//
// IX = uint16_t: the columns are 16-bit offsets from their slot's base sb[k].
// A thread's entries lie NT apart and a slot holds at most NT entries, so each
// entry's slot is past the previous one's: the thread walks the slot table
// forward, and over the block's full slots (NT entries each, the first `full`
// ones) the slot is the entry's index / NT.
template <typename T, typename IX, int MODE, int LDSN>
__global__ void __launch_bounds__(kJagRows) k_jag_stream(int64_t nrows, const int32_t *__restrict__ rp,
                                                         const IX *__restrict__ jci, const int32_t *__restrict__ sb,
                                                         const T *__restrict__ jv, const int32_t *__restrict__ jrows,
                                                         const int32_t *__restrict__ bst,
                                                         const int32_t *__restrict__ st, const T *__restrict__ x,
                                                         const T *__restrict__ r, const T *__restrict__ d,
                                                         T *__restrict__ y, T *__restrict__ y2) {
    constexpr int NT = kJagRows;
    constexpr int B = LDSN / NT;
    constexpr bool kOff = sizeof(IX) == 2;
    __shared__ T sh[LDSN];
    __shared__ int sst[kJagMaxSlots + 1];
    __shared__ int ssb[kOff ? kJagMaxSlots + 1 : 1];
    const int tid = threadIdx.x;
    const int64_t blk = xcd_grouped_block<kXcdGroupRows / kJagRows>();
    const int64_t rb = blk * NT;
    const int64_t re = rb + NT < nrows ? rb + NT : nrows;
    const int p0 = rp[rb];
    const int total = rp[re] - p0;
    const int t0 = bst[blk], nsl = bst[blk + 1] - t0;  // maxlen + 1 slot starts
    for (int k = tid; k < nsl; k += NT) {
        sst[k] = st[t0 + k];
        if (kOff) ssb[k] = sb[t0 + k];
    }
    const bool owner = rb + tid < re;
    const int64_t row = owner ? jrows[rb + tid] : 0;
    __syncthreads();
    // the number of leading slots holding more than t rows (= the row length of
    // rank t)
    auto slots_over = [&](int t) {
        int lo = 0, hi = nsl - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (sst[mid + 1] - sst[mid] > t) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    };
    const int len = owner ? slots_over(tid) : 0;
    const int full_end = kOff ? slots_over(NT - 1) * NT : 0;
    int ks = -1;  // slot of this thread's previous entry
    constexpr bool kEarlyRowIn = sizeof(T) == 4;
    RowIn<T, MODE> in;
    if (owner && kEarlyRowIn) in.load(row, x, r, d, y);
    T acc = 0;
    int kc = 0;
    for (int w0 = 0; w0 < total; w0 += LDSN) {
        const int w1 = w0 + LDSN < total ? w0 + LDSN : total;
        int j[B];
        T av[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int q = w0 + u * NT + tid;
            j[u] = q < w1 ? (int)__builtin_nontemporal_load(jci + p0 + q) : -1;
            av[u] = q < w1 ? __builtin_nontemporal_load(jv + p0 + q) : (T)0;
        }
        if (kOff) {
            // the slots' bases first (LDS only: they overlap the loads in flight),
            // then the columns
            int base[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int q = w0 + u * NT + tid;
                base[u] = 0;
                if (q < w1) {
                    int k;
                    if (q < full_end) {
                        k = q / NT;
                    } else {
                        // q < total = sst[nsl - 1] stops the walk at a slot
                        k = ks + 1 > full_end / NT ? ks + 1 : full_end / NT;
                        while (sst[k + 1] <= q) ++k;
                    }
                    ks = k;
                    base[u] = ssb[k];
                }
            }
#pragma unroll
            for (int u = 0; u < B; ++u)
                if (j[u] >= 0) j[u] += base[u];
        }
        T xv[B];
#pragma unroll
        for (int u = 0; u < B; ++u) xv[u] = j[u] >= 0 ? x[j[u]] : (T)0;
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int q = w0 + u * NT + tid;
            if (q < w1) sh[q - w0] = av[u] * xv[u];
        }
        __syncthreads();
        // this row's entries inside [w0, w1), in ascending slot order, eight at a time
        while (kc + 8 <= len && sst[kc + 7] + tid < w1) {
            int q[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) q[u] = sst[kc + u] + tid - w0;
            T v8[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v8[u] = sh[q[u]];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc = acc + v8[u];
            kc += 8;
        }
        while (kc < len && sst[kc] + tid < w1) {
            acc = acc + sh[sst[kc] + tid - w0];
            ++kc;
        }
        __syncthreads();
    }
    if (owner) {
        if (!kEarlyRowIn) in.load(row, x, r, d, y);
        in.store(row, acc, y, y2);
    }
}

// Jagged copy, first pass: cnt[b] = longest row of block b + 1.
__global__ void __launch_bounds__(kJagRows) k_jag_count(int64_t nrows, const int32_t *__restrict__ rp,
                                                        int32_t *__restrict__ cnt) {
    __shared__ int sm[kJagRows / kWave];
    const int64_t rb = (int64_t)blockIdx.x * kJagRows, i = rb + threadIdx.x;
    int len = i < nrows ? rp[i + 1] - rp[i] : 0;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const int y = __shfl_xor(len, o);
        len = y > len ? y : len;
    }
    if ((threadIdx.x & (kWave - 1)) == 0) sm[threadIdx.x / kWave] = len;
    __syncthreads();
    if (threadIdx.x == 0) {
        int m = 0;
        for (int w = 0; w < kJagRows / kWave; ++w) m = sm[w] > m ? sm[w] : m;
        cnt[blockIdx.x] = m + 1;
    }
}

// Jagged copy, second pass (bst = exclusive scan of the counts): ranks (longer
// rows first, ties by row), slot tables st[k] = sum over the block's rows of
// min(len, k), and the entries in slot order.  With jco (the 16-bit form) each
// slot's smallest column goes to sb[k] (parallel to st) and each entry's column
// as its offset from it; an offset beyond 65535 sets *bad (the copy is then
// unusable and the caller builds the 32-bit form).
__global__ void __launch_bounds__(kJagRows) k_jag_fill(int64_t nrows, const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ ci, const double *__restrict__ v,
                                                       const int32_t *__restrict__ bst, int32_t *__restrict__ st,
                                                       int32_t *__restrict__ jrows, int32_t *__restrict__ jci,
                                                       uint16_t *__restrict__ jco, int32_t *__restrict__ sb,
                                                       double *__restrict__ jv, int *__restrict__ bad) {
    __shared__ int slen[kJagRows];
    __shared__ int sst[kJagMaxSlots + 1];
    __shared__ int smin[kJagMaxSlots + 1];
    const int t = threadIdx.x;
    const int64_t rb = (int64_t)blockIdx.x * kJagRows, i = rb + t;
    const int nr = nrows - rb < kJagRows ? (int)(nrows - rb) : kJagRows;
    const int len = t < nr ? rp[i + 1] - rp[i] : -1;
    slen[t] = len;
    __syncthreads();
    int rank = 0;
    for (int u = 0; u < nr; ++u) {
        const int lu = slen[u];
        rank += (lu > len) || (lu == len && u < t);
    }
    const int t0 = bst[blockIdx.x], nsl = bst[blockIdx.x + 1] - t0;
    for (int k = t; k < nsl; k += kJagRows) {
        int sum = 0;
        for (int u = 0; u < nr; ++u) sum += slen[u] < k ? slen[u] : k;
        sst[k] = sum;
        st[t0 + k] = sum;
        smin[k] = INT_MAX;
    }
    __syncthreads();
    const int p0 = rp[rb], a = t < nr ? rp[i] : 0;
    if (jco) {
        for (int k = 0; k < len; ++k) atomicMin(&smin[k], ci[a + k]);
        __syncthreads();
        // the last table entry (the block's total) has no slot: base 0
        for (int k = t; k < nsl; k += kJagRows) sb[t0 + k] = k + 1 < nsl ? smin[k] : 0;
    }
    if (t >= nr) return;
    jrows[rb + rank] = (int32_t)i;
    for (int k = 0; k < len; ++k) {
        const int q = p0 + sst[k] + rank;
        const int c = ci[a + k];
        if (jco) {
            const unsigned off = (unsigned)(c - smin[k]);
            if (off > 0xffffu) *bad = 1;
            jco[q] = (uint16_t)off;
        } else {
            jci[q] = c;
        }
        jv[q] = v[a + k];
    }
}

// Row-list kernels on the compact copy of a level's F rows (row f of AF is row
// rows[f] of the level matrix, all its columns): LANES threads per row, each
// summing a strided share, then a fixed xor-tree across the lanes.
// t[f] = r[i] - (A e)[i], i = rows[f]
template <typename T, int LANES>
__global__ void __launch_bounds__(256) k_csr_rows_res(int64_t nr, const int32_t *__restrict__ rows,
                                                      const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                      const T *__restrict__ v, const T *__restrict__ e,
                                                      const T *__restrict__ r, T *__restrict__ t) {
    const int64_t gid = gtid();
    const int64_t f = gid / LANES;
    const int sub = (int)(gid % LANES);
    T s = 0;
    if (f < nr)
        for (int p = rp[f] + sub; p < rp[f + 1]; p += LANES) s = s + v[p] * e[ci[p]];
#pragma unroll
    for (int o = LANES / 2; o > 0; o >>= 1) s = s + __shfl_xor(s, o);
    if (f < nr && sub == 0) t[f] = r[rows[f]] - s;
}

// F-relaxation in place, e[i] += dinv[f] (r[i] - (A e)[i]) for i = flist[f]; valid
// when A_FF is diagonal (no F row reads another F point, so the update of e[i]
// races with no other row's reads).  e is read and written: no restrict.
template <typename T, int LANES>
__global__ void __launch_bounds__(256) k_frelax_inplace(int64_t nF, const int32_t *__restrict__ flist,
                                                        const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ ci, const T *__restrict__ v,
                                                        const T *__restrict__ dinv, const T *__restrict__ r,
                                                        T *e) {
    const int64_t gid = gtid();
    const int64_t f = gid / LANES;
    const int sub = (int)(gid % LANES);
    T s = 0;
    if (f < nF)
        for (int p = rp[f] + sub; p < rp[f + 1]; p += LANES) s = s + v[p] * e[ci[p]];
#pragma unroll
    for (int o = LANES / 2; o > 0; o >>= 1) s = s + __shfl_xor(s, o);
    if (f < nF && sub == 0) {
        const int64_t i = flist[f];
        e[i] = e[i] + dinv[f] * (r[i] - s);
    }
}

// CSR SpMV for the small levels, where 256-row workgroups would leave most CUs
// idle: LANES threads per row with strided shares and a fixed xor-tree, so the
// loads of a row are issued at once and the latency chain is short.  Modes as
// the stream kernel.
template <typename T, int MODE, int LANES>
__global__ void __launch_bounds__(256) k_csr_lanes(int64_t nrows, const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ ci, const T *__restrict__ v,
                                                   const T *__restrict__ x, const T *__restrict__ r,
                                                   const T *__restrict__ d, T *__restrict__ y, T *__restrict__ y2) {
    const int64_t gid = gtid();
    const int64_t row = gid / LANES;
    const int sub = (int)(gid % LANES);
    T s = 0;
    RowIn<T, MODE> in;
    if (row < nrows && sub == 0) in.load(row, x, r, d, y);
    if (row < nrows) {
        // two strides per trip, both gathers issued before either product is
        // added (the additions keep the stride order)
        const int pe = rp[row + 1];
        for (int p = rp[row] + sub; p < pe; p += 2 * LANES) {
            const int q = p + LANES;
            const int c0 = ci[p];
            const T v0 = v[p];
            const int c1 = q < pe ? ci[q] : c0;
            const T v1 = q < pe ? v[q] : (T)0;
            const T x0 = x[c0], x1 = x[c1];
            s = s + v0 * x0;
            if (q < pe) s = s + v1 * x1;
        }
    }
#pragma unroll
    for (int o = LANES / 2; o > 0; o >>= 1) s = s + __shfl_xor(s, o);
    if (row < nrows && sub == 0) in.store(row, s, y, y2);
}

// e = B^{-1} r per cell (ADD: e += B^{-1} r)
template <typename T, bool ADD>
__global__ void k_block_apply3(int64_t ncell, const T *__restrict__ B, const T *__restrict__ r, T *__restrict__ e) {
    const int64_t c = gtid();
    if (c >= ncell) return;
    const T r0 = r[3 * c], r1 = r[3 * c + 1], r2 = r[3 * c + 2];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const T d = B[(3 * q) * ncell + c] * r0 + B[(3 * q + 1) * ncell + c] * r1 + B[(3 * q + 2) * ncell + c] * r2;
        e[3 * c + q] = ADD ? e[3 * c + q] + d : d;
    }
}

template <typename T, bool ADD>
__global__ void k_block_apply1(int64_t ncell, const T *__restrict__ B, const T *__restrict__ r, T *__restrict__ e) {
    const int64_t c = gtid();
    if (c < ncell) e[c] = ADD ? e[c] + B[c] * r[c] : B[c] * r[c];
}

template <typename T>
__global__ void k_frelax_first(int64_t n, const int32_t *__restrict__ fmap, const T *__restrict__ dinv,
                               const T *__restrict__ r, T *__restrict__ e) {
    const int64_t i = gtid();
    if (i >= n) return;
    const int f = fmap[i];
    e[i] = f >= 0 ? dinv[f] * r[i] : (T)0;
}

// The mixed-precision cycle's FP64 boundary folded into its first and last
// level-0 steps.  In: rf = (float) r64, then e = B^{-1} rf per 3x3 cell block
// (the products and sums of k_block_apply3).  Out: the W_p = 0 prolongation
// e_C += e_c and z = (double) e in one pass over the level's rows.
__global__ void k_block_apply3_in64(int64_t ncell, const float *__restrict__ B, const double *__restrict__ r64,
                                    float *__restrict__ rf, float *__restrict__ e) {
    const int64_t c = gtid();
    if (c >= ncell) return;
    const float r0 = (float)r64[3 * c], r1 = (float)r64[3 * c + 1], r2 = (float)r64[3 * c + 2];
    rf[3 * c] = r0;
    rf[3 * c + 1] = r1;
    rf[3 * c + 2] = r2;
#pragma unroll
    for (int q = 0; q < 3; ++q)
        e[3 * c + q] = B[(3 * q) * ncell + c] * r0 + B[(3 * q + 1) * ncell + c] * r1 + B[(3 * q + 2) * ncell + c] * r2;
}

__global__ void k_scatter_add_out64(int64_t n, const int32_t *__restrict__ cmap, const float *__restrict__ ec,
                                    const float *__restrict__ e, double *__restrict__ z) {
    const int64_t i = gtid();
    if (i >= n) return;
    const int c = cmap[i];
    const float v = c >= 0 ? e[i] + ec[c] : e[i];
    z[i] = (double)v;
}

// The Jacobi F-relaxation from e = 0 kept compact: eF[f] = dinv[f] r[flist[f]]
template <typename T>
__global__ void k_frelax_first_compact(int64_t nF, const int32_t *__restrict__ flist, const T *__restrict__ dinv,
                                       const T *__restrict__ r, T *__restrict__ eF) {
    const int64_t f = gtid();
    if (f >= nF) return;
    eF[f] = dinv[f] * r[flist[f]];
}

// The prolongation with P the injection of the C points (W_p = 0) and the
// F-relaxation's correction kept compact: e[i] = eF[fmap[i]] on F points,
// 0 + e_c[cmap[i]] on C points
template <typename T>
__global__ void k_prolong_inject_compact(int64_t n, const int32_t *__restrict__ fmap,
                                         const int32_t *__restrict__ cmap, const T *__restrict__ eF,
                                         const T *__restrict__ ec, T *__restrict__ e) {
    const int64_t i = gtid();
    if (i >= n) return;
    const int f = fmap[i];
    e[i] = f >= 0 ? eF[f] : (T)0 + ec[cmap[i]];
}

template <typename T>
__global__ void k_frelax_scatter(int64_t nF, const int32_t *__restrict__ flist, const T *__restrict__ dinv,
                                 const T *__restrict__ t, T *__restrict__ e) {
    const int64_t f = gtid();
    if (f >= nF) return;
    const int64_t i = flist[f];
    e[i] = e[i] + dinv[f] * t[f];
}

template <typename T>
__global__ void k_div(int64_t n, const T *__restrict__ r, const T *__restrict__ d, T *__restrict__ x) {
    const int64_t i = gtid();
    if (i < n) x[i] = r[i] / d[i];
}

template <typename T>
__global__ void k_gather(int64_t n, const int32_t *__restrict__ idx, const T *__restrict__ src, T *__restrict__ dst) {
    const int64_t i = gtid();
    if (i < n) dst[i] = src[idx[i]];
}

// t[f] = r[idx[f]] and x0[f] = t[f] / d[f] (the gathered right-hand side and the
// first Jacobi iterate from zero of the hierarchy it feeds)
template <typename T>
__global__ void k_gather_div(int64_t n, const int32_t *__restrict__ idx, const T *__restrict__ src,
                             const T *__restrict__ d, T *__restrict__ dst, T *__restrict__ x0) {
    const int64_t i = gtid();
    if (i >= n) return;
    const T v = src[idx[i]];
    dst[i] = v;
    x0[i] = v / d[i];
}

// e[i] = 0 + d[map[i]] where map[i] >= 0, else 0 (the zero fill and the scatter
// of the F-point correction in one pass)
template <typename T>
__global__ void k_scatter_set(int64_t n, const int32_t *__restrict__ map, const T *__restrict__ d,
                              T *__restrict__ e) {
    const int64_t i = gtid();
    if (i >= n) return;
    const int f = map[i];
    e[i] = f >= 0 ? (T)0 + d[f] : (T)0;
}

template <typename T>
__global__ void k_scatter_add(int64_t n, const int32_t *__restrict__ idx, const T *__restrict__ d, T *__restrict__ e) {
    const int64_t i = gtid();
    if (i >= n) return;
    const int64_t j = idx[i];
    e[j] = e[j] + d[i];
}

// forward/back substitution with the coarsest LU (FP64 throughout); one workgroup
template <typename T>
__global__ void __launch_bounds__(256) k_lu_solve(int64_t n, const double *__restrict__ lu,
                                                  const int32_t *__restrict__ perm, const T *__restrict__ b,
                                                  T *__restrict__ x) {
    extern __shared__ double y[];
    const int tid = threadIdx.x;
    for (int64_t i = tid; i < n; i += blockDim.x) y[i] = (double)b[perm[i]];
    __syncthreads();
    for (int64_t k = 0; k < n; ++k) {
        const double yk = y[k];
        for (int64_t i = k + 1 + tid; i < n; i += blockDim.x) y[i] = y[i] - lu[i * n + k] * yk;
        __syncthreads();
    }
    for (int64_t k = n - 1; k >= 0; --k) {
        if (tid == 0) y[k] = y[k] / lu[k * n + k];
        __syncthreads();
        const double yk = y[k];
        for (int64_t i = tid; i < k; i += blockDim.x) y[i] = y[i] - lu[i * n + k] * yk;
        __syncthreads();
    }
    for (int64_t i = tid; i < n; i += blockDim.x) x[i] = (T)y[i];
}

// Broadcast of lane k's double to the whole wavefront (k uniform): two
// v_readlane, no LDS round trip as a shuffle would take.
__device__ inline double lane_bcast(double v, int k) {
    const long long u = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, k);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), k);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// the same substitutions for n <= 64 in one wavefront: four wavefronts copy the
// factors to LDS, then lane i of the first holds y[i] and y[k] is broadcast
// from lane k, so the substitutions need no workgroup barrier (same operations
// in the same order as the workgroup kernel)
template <typename T>
__global__ void __launch_bounds__(256) k_lu_solve_wave(int n, const double *__restrict__ lu,
                                                       const int32_t *__restrict__ perm, const T *__restrict__ b,
                                                       T *__restrict__ x) {
    __shared__ double L[kWave * kWave];
    const int t = threadIdx.x;
    double y = t < n ? (double)b[perm[t]] : 0.0;
#pragma unroll 4
    for (int q = t; q < n * n; q += 256) L[q] = lu[q];
    __syncthreads();
    if (t >= kWave) return;
    const int l = t;
    for (int k = 0; k < n; ++k) {
        const double yk = lane_bcast(y, k);
        if (l > k && l < n) y = y - L[l * n + k] * yk;
    }
    for (int k = n - 1; k >= 0; --k) {
        if (l == k) y = y / L[k * n + k];
        const double yk = lane_bcast(y, k);
        if (l < k) y = y - L[l * n + k] * yk;
    }
    if (l < n) x[l] = (T)y;
}

// ---- the bottom of an AMG V-cycle in one workgroup ----
// out(i, (A x)_i) for every row i of a tail-level matrix held in LDS against a
// vector in LDS, with all threads of the workgroup: L lanes per row (the
// largest power of two up to 32 with L * rows <= threads), each summing a
// strided share of the row, then a fixed xor-tree across its lanes (the lanes
// kernel's order).  Consecutive lanes read consecutive words of a row, which
// keeps the LDS reads free of bank conflicts.
template <typename T, typename F>
__device__ inline void tail_spmv(int nrows, const int32_t *rp, const int32_t *ci, const T *v, const T *xl, F out) {
    int L = 1;
    while (L < 32 && 2 * L * nrows <= kTailThreads) L *= 2;
    for (int base = 0; base < nrows * L; base += kTailThreads) {
        const int g = base + (int)threadIdx.x;
        const int row = g / L, sub = g % L;
        T acc = 0;
        if (row < nrows) {
            const int e = rp[row + 1];
            for (int p = rp[row] + sub; p < e; p += L) {
                const T pr = v[p] * xl[ci[p]];
                acc = acc + pr;
            }
        }
        for (int o = L / 2; o > 0; o >>= 1) acc = acc + __shfl_xor(acc, o);
        if (row < nrows && sub == 0) out(row, acc);
    }
}

// LDS offset (in T, from the start of the vectors) of tail level k's vectors
// r, xa, xb, t (k == nlev: the coarsest level's r and x)
template <typename T>
__device__ inline int tail_off(const TailDesc<T> &d, int k) {
    int o = 0;
    for (int j = 0; j < k; ++j) o += 4 * d.n[j];
    return o;
}

// The V-cycle of amg_cycle from level k0 down to the dense coarsest level and
// back, in one workgroup: the same steps and roundings (Jacobi iterate from
// zero r / l1, pre - 1 more l1-Jacobi sweeps, residual, restriction with the
// next level's first iterate, LU solve, prolongation, post sweeps).  The
// levels' matrices, l1 and the LU factors are first copied into LDS from their
// packed device copy, 16 bytes per load and eight loads per thread in flight;
// the work vectors live in LDS too, several lanes per row.
// A level's iterate ping-pongs between xa and xb; which one is final follows
// from the number of sweeps.
template <typename T>
__global__ void __launch_bounds__(kTailThreads) k_amg_tail(const TailDesc<T> d) {
    __shared__ __align__(16) unsigned char lds[kTailLdsBytes];
    const int tid = threadIdx.x;
    {
        uint4 *dst = reinterpret_cast<uint4 *>(lds);
        for (int q0 = 0; q0 < d.pack16; q0 += 8 * kTailThreads) {
            uint4 b0, b1, b2, b3, b4, b5, b6, b7;
            const int q = q0 + tid;
            const int last = d.pack16 - 1;
            // every load in bounds (clamped), the stores guarded
            b0 = d.pack[min(q, last)];
            b1 = d.pack[min(q + kTailThreads, last)];
            b2 = d.pack[min(q + 2 * kTailThreads, last)];
            b3 = d.pack[min(q + 3 * kTailThreads, last)];
            b4 = d.pack[min(q + 4 * kTailThreads, last)];
            b5 = d.pack[min(q + 5 * kTailThreads, last)];
            b6 = d.pack[min(q + 6 * kTailThreads, last)];
            b7 = d.pack[min(q + 7 * kTailThreads, last)];
            if (q < d.pack16) dst[q] = b0;
            if (q + kTailThreads < d.pack16) dst[q + kTailThreads] = b1;
            if (q + 2 * kTailThreads < d.pack16) dst[q + 2 * kTailThreads] = b2;
            if (q + 3 * kTailThreads < d.pack16) dst[q + 3 * kTailThreads] = b3;
            if (q + 4 * kTailThreads < d.pack16) dst[q + 4 * kTailThreads] = b4;
            if (q + 5 * kTailThreads < d.pack16) dst[q + 5 * kTailThreads] = b5;
            if (q + 6 * kTailThreads < d.pack16) dst[q + 6 * kTailThreads] = b6;
            if (q + 7 * kTailThreads < d.pack16) dst[q + 7 * kTailThreads] = b7;
        }
    }
    auto I = [&](int off) { return reinterpret_cast<const int32_t *>(lds + off); };
    auto V = [&](int off) { return reinterpret_cast<const T *>(lds + off); };
    T *vec = reinterpret_cast<T *>(lds + d.vec);
    const int K = d.nlev, nc = d.nc;
    {
        const int n = d.n[0];
        T *r = vec, *xa = vec + n;
        for (int i = tid; i < n; i += kTailThreads) {
            r[i] = d.r_in[i];
            if (d.x0_ready) xa[i] = d.x0_in[i];
        }
    }
    __syncthreads();
    const int sw_pre = d.pre > 0 ? d.pre - 1 : 0;
    // down
    for (int k = 0; k < K; ++k) {
        const int n = d.n[k];
        const int32_t *arp = I(d.arp[k]), *aci = I(d.aci[k]);
        const T *av = V(d.av[k]), *l1 = V(d.l1[k]);
        T *r = vec + tail_off(d, k), *xa = r + n, *xb = xa + n, *t = xb + n;
        T *cur = xa, *oth = xb;
        if (d.pre > 0) {
            const bool have_x0 = k == 0 ? d.x0_ready != 0 : true;
            if (!have_x0) {
                for (int i = tid; i < n; i += kTailThreads) xa[i] = r[i] / l1[i];
                __syncthreads();
            }
            for (int it = 1; it < d.pre; ++it) {
                T *c = cur, *o = oth;
                tail_spmv(n, arp, aci, av, c, [&](int i, T acc) { o[i] = c[i] + (r[i] - acc) / l1[i]; });
                __syncthreads();
                cur = o;
                oth = c;
            }
        } else {
            for (int i = tid; i < n; i += kTailThreads) xa[i] = (T)0;
            __syncthreads();
        }
        {
            T *c = cur;
            tail_spmv(n, arp, aci, av, c, [&](int i, T acc) { t[i] = r[i] - acc; });
        }
        __syncthreads();
        const bool next_coarse = k + 1 == K;
        const int nn = next_coarse ? nc : d.n[k + 1];
        T *rn = vec + tail_off(d, k + 1);
        const T *l1n = next_coarse ? nullptr : V(d.l1[k + 1]);
        const bool div = d.pre > 0 && !next_coarse;
        tail_spmv(nn, I(d.rrp[k]), I(d.rci[k]), V(d.rv[k]), t, [&](int j, T acc) {
            rn[j] = acc;
            if (div) rn[nn + j] = acc / l1n[j];
        });
        __syncthreads();
    }
    // coarsest: the substitutions of k_lu_solve_wave in the first wavefront
    {
        const double *LU = reinterpret_cast<const double *>(lds + d.lu);
        const int32_t *perm = I(d.perm);
        T *rK = vec + tail_off(d, K), *xK = rK + nc;
        if (tid < kWave) {
            const int l = tid;
            double y = l < nc ? (double)rK[perm[l]] : 0.0;
            for (int k = 0; k < nc; ++k) {
                const double yk = lane_bcast(y, k);
                if (l > k && l < nc) y = y - LU[l * nc + k] * yk;
            }
            for (int k = nc - 1; k >= 0; --k) {
                if (l == k) y = y / LU[k * nc + k];
                const double yk = lane_bcast(y, k);
                if (l < k) y = y - LU[l * nc + k] * yk;
            }
            if (l < nc) xK[l] = (T)y;
        }
        __syncthreads();
    }
    // up
    const T *xnext = vec + tail_off(d, K) + nc;
    for (int k = K - 1; k >= 0; --k) {
        const int n = d.n[k];
        const int32_t *arp = I(d.arp[k]), *aci = I(d.aci[k]);
        const T *av = V(d.av[k]), *l1 = V(d.l1[k]);
        T *r = vec + tail_off(d, k), *xa = r + n, *xb = xa + n;
        T *cur = (sw_pre % 2 == 0) ? xa : xb;
        T *oth = (cur == xa) ? xb : xa;
        {
            T *c = cur;
            tail_spmv(n, I(d.prp[k]), I(d.pci[k]), V(d.pv[k]), xnext, [&](int i, T acc) { c[i] = c[i] + acc; });
        }
        __syncthreads();
        for (int it = 0; it < d.post; ++it) {
            T *c = cur, *o = oth;
            tail_spmv(n, arp, aci, av, c, [&](int i, T acc) { o[i] = c[i] + (r[i] - acc) / l1[i]; });
            __syncthreads();
            cur = o;
            oth = c;
        }
        xnext = cur;
    }
    for (int i = tid; i < d.n[0]; i += kTailThreads) d.x_out[i] = xnext[i];
}

}  // namespace

constexpr int BT = 256;

template <typename T, int ROWS, int NT, int LDSN>
static void csr_rows(int mode, const DCsr &A, const T *vals, const T *x, const T *r, const T *d, T *y, T *y2,
                     hipStream_t s, KEvents ev) {
    const unsigned g = nblocks(A.nrows, ROWS);
#define MGR_STREAM(M)                                                                                               \
    do {                                                                                                            \
        if (ev.start)                                                                                               \
            hipExtLaunchKernelGGL(k_csr_stream<T, M, ROWS, NT, LDSN>, dim3(g), dim3(NT), 0, s, ev.start, ev.stop, 0, \
                                  A.nrows, A.rp, A.ci, vals, x, r, d, y, y2);                                       \
        else                                                                                                        \
            k_csr_stream<T, M, ROWS, NT, LDSN><<<g, NT, 0, s>>>(A.nrows, A.rp, A.ci, vals, x, r, d, y, y2);         \
    } while (0)
    switch (mode) {
    case 0: MGR_STREAM(0); break;
    case 1: MGR_STREAM(1); break;
    case 2: MGR_STREAM(2); break;
    case 3: MGR_STREAM(3); break;
    case 4: MGR_STREAM(4); break;
    case 5: MGR_STREAM(5); break;
    default: MGR_STREAM(6); break;
    }
#undef MGR_STREAM
}

template <typename T>
static const T *jag_vals(const Jag &J);
template <>
const double *jag_vals<double>(const Jag &J) { return J.v; }
template <>
const float *jag_vals<float>(const Jag &J) { return J.vf; }

template <typename T>
static void jag_rows(int mode, const DCsr &A, const T *x, const T *r, const T *d, T *y, T *y2, hipStream_t s,
                     KEvents ev) {
    const Jag &J = *A.jag;
    const unsigned g = (unsigned)J.nblk;
    // passes of 4864 FP64 entries (19 per thread): with the 2 KB slot table the
    // workgroup takes 40 KB of LDS, four per CU (5120 would leave three: +5 %
    // on the coarse-grid sweep); 4096 with the 16-bit columns' second 2 KB table
    // (slot bases).  FP32 8192, and 4096 with the 16-bit columns (whose slot
    // bases take 32 more registers at 8192: three waves per SIMD, sweep +60 %)
#define MGR_JAG(IX, LDSN, M, CI)                                                                                   \
    do {                                                                                                           \
        if (ev.start)                                                                                              \
            hipExtLaunchKernelGGL(k_jag_stream<T, IX, M, LDSN>, dim3(g), dim3(kJagRows), 0, s, ev.start, ev.stop, 0, \
                                  A.nrows, A.rp, CI, J.sb, jag_vals<T>(J), J.rows, J.bst, J.st, x, r, d, y, y2);   \
        else                                                                                                       \
            k_jag_stream<T, IX, M, LDSN><<<g, kJagRows, 0, s>>>(A.nrows, A.rp, CI, J.sb, jag_vals<T>(J), J.rows,   \
                                                                J.bst, J.st, x, r, d, y, y2);                     \
    } while (0)
#define MGR_JAG_MODES(IX, LDSN, CI)                 \
    switch (mode) {                                 \
    case 0: MGR_JAG(IX, LDSN, 0, CI); break;        \
    case 1: MGR_JAG(IX, LDSN, 1, CI); break;        \
    case 2: MGR_JAG(IX, LDSN, 2, CI); break;        \
    case 3: MGR_JAG(IX, LDSN, 3, CI); break;        \
    case 4: MGR_JAG(IX, LDSN, 4, CI); break;        \
    case 5: MGR_JAG(IX, LDSN, 5, CI); break;        \
    default: MGR_JAG(IX, LDSN, 6, CI); break;       \
    }
    if (J.co) {
        MGR_JAG_MODES(uint16_t, 4096, J.co)
    } else {
        MGR_JAG_MODES(int32_t, (sizeof(T) == 4 ? 8192 : 4864), J.ci)
    }
#undef MGR_JAG_MODES
#undef MGR_JAG
}

template <typename T, int MODE>
static void csr_lanes(const DCsr &A, int lanes, const T *vals, const T *x, const T *r, const T *d, T *y, T *y2,
                      hipStream_t s, KEvents ev) {
    const unsigned g = nblocks(A.nrows * lanes, BT);
#define MGR_LANES(L)                                                                                                 \
    do {                                                                                                             \
        if (ev.start)                                                                                                \
            hipExtLaunchKernelGGL(k_csr_lanes<T, MODE, L>, dim3(g), dim3(BT), 0, s, ev.start, ev.stop, 0, A.nrows,   \
                                  A.rp, A.ci, vals, x, r, d, y, y2);                                                 \
        else                                                                                                         \
            k_csr_lanes<T, MODE, L><<<g, BT, 0, s>>>(A.nrows, A.rp, A.ci, vals, x, r, d, y, y2);                     \
    } while (0)
    switch (lanes) {
    case 2: MGR_LANES(2); break;
    case 4: MGR_LANES(4); break;
    case 8: MGR_LANES(8); break;
    case 16: MGR_LANES(16); break;
    default: MGR_LANES(32); break;
    }
#undef MGR_LANES
}

// Levels of at least kCsrStreamMinRows rows take 256-row stream workgroups (or
// the jagged kernel); levels of kCsrStreamSmallRows up to that take the stream
// kernel with row blocks sized so that a block's entries about fill one pass
// (64 rows of >= 24 entries, 128 rows of >= 12), which issues a level's loads
// in one wave of workgroups (AMG level 2 of the 128^3 coarse grid, 123 k rows of
// 38 entries: 25 -> 17 us per sweep against the lanes kernel); smaller levels
// take the lanes-per-row kernel, whose launches are latency-bound anyway.  The
// cut, at 1 M rows, gives the long-row levels of 0.1-1 M rows (the AMG level 1
// of the 128^3 coarse grid, 0.70 M rows of 34 entries, and the F-block AMG's
// levels 1 and 2) the smaller blocks: their 256-row grids (the jagged copies
// included) filled 0.5-2.7 waves of resident workgroups; V-cycle -34 us.  The
// coarse grid itself (2.1 M rows) keeps the jagged kernel (128-row stream
// blocks: 148 against 138 us per sweep).
constexpr int64_t kCsrStreamMinRows = 1048576;
constexpr int64_t kCsrStreamSmallRows = 8192;
// mean row lengths below which the stream kernel takes 1024- and 2048-entry passes
// (above: 5120 entries in FP64, 20 per thread, 40 KB of LDS: 4 workgroups per CU;
// 8192 in FP32)
constexpr double kStreamShortRow = 3.0;
constexpr double kStreamMidRow = 8.0;

// Large levels: 256-row stream workgroups, or the jagged kernel where the matrix
// has a jagged copy; mid-size levels: stream workgroups of fewer rows (all with
// sequential row sums).  Small levels: several lanes per row.
template <typename T>
static void csr_any(int mode, const DCsr &A, const T *vals, const T *x, const T *r, const T *d, T *y, T *y2,
                    hipStream_t s, KEvents ev = {}) {
    if (A.nrows <= 0) return;
    const double avg = (double)A.nnz / (double)A.nrows;
    if (A.nrows >= kCsrStreamMinRows) {
        if (A.jag && avg >= kStreamMidRow) {
            jag_rows<T>(mode, A, x, r, d, y, y2, s, ev);
            return;
        }
        if (avg < kStreamShortRow) csr_rows<T, 256, 256, 1024>(mode, A, vals, x, r, d, y, y2, s, ev);
        else if (avg < kStreamMidRow) csr_rows<T, 256, 256, 2048>(mode, A, vals, x, r, d, y, y2, s, ev);
        else if (sizeof(T) == 4) csr_rows<T, 256, 256, 8192>(mode, A, vals, x, r, d, y, y2, s, ev);
        else csr_rows<T, 256, 256, 5120>(mode, A, vals, x, r, d, y, y2, s, ev);
        return;
    }
    if (A.nrows >= kCsrStreamSmallRows) {
        if (avg >= 24) csr_rows<T, 64, 256, 4864>(mode, A, vals, x, r, d, y, y2, s, ev);
        else if (avg >= 12) csr_rows<T, 128, 256, 4864>(mode, A, vals, x, r, d, y, y2, s, ev);
        else csr_rows<T, 256, 256, 2048>(mode, A, vals, x, r, d, y, y2, s, ev);
        return;
    }
    const int lanes = avg < 3 ? 2 : avg < 6 ? 4 : avg < 12 ? 8 : avg < 24 ? 16 : 32;
    switch (mode) {
    case 0: csr_lanes<T, 0>(A, lanes, vals, x, r, d, y, y2, s, ev); break;
    case 1: csr_lanes<T, 1>(A, lanes, vals, x, r, d, y, y2, s, ev); break;
    case 2: csr_lanes<T, 2>(A, lanes, vals, x, r, d, y, y2, s, ev); break;
    case 3: csr_lanes<T, 3>(A, lanes, vals, x, r, d, y, y2, s, ev); break;
    case 4: csr_lanes<T, 4>(A, lanes, vals, x, r, d, y, y2, s, ev); break;
    case 5: csr_lanes<T, 5>(A, lanes, vals, x, r, d, y, y2, s, ev); break;
    default: csr_lanes<T, 6>(A, lanes, vals, x, r, d, y, y2, s, ev); break;
    }
}

bool csr_long_rows(const DCsr &A) {
    return A.nrows >= kCsrStreamMinRows && (double)A.nnz >= kStreamMidRow * (double)A.nrows;
}

void launch_jag_count(const DCsr &A, int32_t *cnt, hipStream_t s) {
    const unsigned g = nblocks(A.nrows, kJagRows);
    if (g) k_jag_count<<<g, kJagRows, 0, s>>>(A.nrows, A.rp, cnt);
}

void launch_jag_fill(const DCsr &A, Jag &J, int *bad, hipStream_t s) {
    if (J.nblk)
        k_jag_fill<<<(unsigned)J.nblk, kJagRows, 0, s>>>(A.nrows, A.rp, A.ci, A.v, J.bst, J.st, J.rows, J.ci, J.co,
                                                         J.sb, J.v, bad);
}

template <typename T>
void launch_amg_tail(const TailDesc<T> &d, hipStream_t s) {
    k_amg_tail<T><<<1, kTailThreads, 0, s>>>(d);
}

template <typename T>
void launch_csr(int mode, const DCsr &A, const T *vals, const T *x, const T *r, const T *d, T *y, hipStream_t s,
                KEvents ev) {
    csr_any<T>(mode, A, vals, x, r, d, y, nullptr, s, ev);
}

template <typename T>
void launch_csr_prolong_into(const DCsr &A, const T *vals, const T *x, const T *eF, const int32_t *fmap,
                             const int32_t *map, T *y, hipStream_t s) {
    csr_any<T>(6, A, vals, x, eF, reinterpret_cast<const T *>(fmap), y,
               reinterpret_cast<T *>(const_cast<int32_t *>(map)), s);
}

template <typename T>
void launch_csr_restrict_div(const DCsr &A, const T *vals, const T *x, const T *d, T *y, T *y2, hipStream_t s) {
    csr_any<T>(4, A, vals, x, nullptr, d, y, y2, s);
}

template <typename T>
void launch_csr_rows_residual(const DCsr &A, int lanes, const T *vals, int64_t nrows, const int32_t *rows,
                              const T *e, const T *r, T *t, hipStream_t s) {
    if (nrows <= 0) return;
    const int L = lanes;
    unsigned g = nblocks(nrows * L, BT);
    switch (L) {
    case 1: k_csr_rows_res<T, 1><<<g, BT, 0, s>>>(nrows, rows, A.rp, A.ci, vals, e, r, t); break;
    case 2: k_csr_rows_res<T, 2><<<g, BT, 0, s>>>(nrows, rows, A.rp, A.ci, vals, e, r, t); break;
    case 4: k_csr_rows_res<T, 4><<<g, BT, 0, s>>>(nrows, rows, A.rp, A.ci, vals, e, r, t); break;
    case 8: k_csr_rows_res<T, 8><<<g, BT, 0, s>>>(nrows, rows, A.rp, A.ci, vals, e, r, t); break;
    case 16: k_csr_rows_res<T, 16><<<g, BT, 0, s>>>(nrows, rows, A.rp, A.ci, vals, e, r, t); break;
    default: k_csr_rows_res<T, 32><<<g, BT, 0, s>>>(nrows, rows, A.rp, A.ci, vals, e, r, t); break;
    }
}

template <typename T>
void launch_frelax_inplace(const DCsr &A, int lanes, const T *vals, int64_t nF, const int32_t *flist,
                           const T *dinv, const T *r, T *e, hipStream_t s) {
    if (nF <= 0) return;
    const int L = lanes;
    unsigned g = nblocks(nF * L, BT);
    switch (L) {
    case 1: k_frelax_inplace<T, 1><<<g, BT, 0, s>>>(nF, flist, A.rp, A.ci, vals, dinv, r, e); break;
    case 2: k_frelax_inplace<T, 2><<<g, BT, 0, s>>>(nF, flist, A.rp, A.ci, vals, dinv, r, e); break;
    case 4: k_frelax_inplace<T, 4><<<g, BT, 0, s>>>(nF, flist, A.rp, A.ci, vals, dinv, r, e); break;
    case 8: k_frelax_inplace<T, 8><<<g, BT, 0, s>>>(nF, flist, A.rp, A.ci, vals, dinv, r, e); break;
    case 16: k_frelax_inplace<T, 16><<<g, BT, 0, s>>>(nF, flist, A.rp, A.ci, vals, dinv, r, e); break;
    default: k_frelax_inplace<T, 32><<<g, BT, 0, s>>>(nF, flist, A.rp, A.ci, vals, dinv, r, e); break;
    }
}

template <typename T>
void launch_block_apply(int64_t ncell, int bs, const T *binv, const T *r, T *e, bool add, hipStream_t s) {
    if (ncell <= 0) return;
    const unsigned g = nblocks(ncell, BT);
    if (bs == 3) {
        if (add) k_block_apply3<T, true><<<g, BT, 0, s>>>(ncell, binv, r, e);
        else k_block_apply3<T, false><<<g, BT, 0, s>>>(ncell, binv, r, e);
    } else {
        if (add) k_block_apply1<T, true><<<g, BT, 0, s>>>(ncell, binv, r, e);
        else k_block_apply1<T, false><<<g, BT, 0, s>>>(ncell, binv, r, e);
    }
}

template <typename T>
void launch_frelax_first(int64_t n, const int32_t *fmap, const T *dinv, const T *r, T *e, hipStream_t s) {
    if (n > 0) k_frelax_first<T><<<nblocks(n, BT), BT, 0, s>>>(n, fmap, dinv, r, e);
}

void launch_block_apply3_in64(int64_t ncell, const float *binv, const double *r64, float *rf, float *e,
                              hipStream_t s) {
    if (ncell > 0) k_block_apply3_in64<<<nblocks(ncell, BT), BT, 0, s>>>(ncell, binv, r64, rf, e);
}

void launch_scatter_add_out64(int64_t n, const int32_t *cmap, const float *ec, const float *e, double *z,
                              hipStream_t s) {
    if (n > 0) k_scatter_add_out64<<<nblocks(n, BT), BT, 0, s>>>(n, cmap, ec, e, z);
}

template <typename T>
void launch_frelax_first_compact(int64_t nF, const int32_t *flist, const T *dinv, const T *r, T *eF, hipStream_t s) {
    if (nF > 0) k_frelax_first_compact<T><<<nblocks(nF, BT), BT, 0, s>>>(nF, flist, dinv, r, eF);
}

template <typename T>
void launch_prolong_inject_compact(int64_t n, const int32_t *fmap, const int32_t *cmap, const T *eF, const T *ec,
                                   T *e, hipStream_t s) {
    if (n > 0) k_prolong_inject_compact<T><<<nblocks(n, BT), BT, 0, s>>>(n, fmap, cmap, eF, ec, e);
}

template <typename T>
void launch_frelax_scatter(int64_t nF, const int32_t *flist, const T *dinv, const T *t, T *e, hipStream_t s) {
    if (nF > 0) k_frelax_scatter<T><<<nblocks(nF, BT), BT, 0, s>>>(nF, flist, dinv, t, e);
}

template <typename T>
void launch_div(int64_t n, const T *r, const T *d, T *x, hipStream_t s) {
    if (n > 0) k_div<T><<<nblocks(n, BT), BT, 0, s>>>(n, r, d, x);
}

template <typename T>
void launch_gather(int64_t n, const int32_t *idx, const T *src, T *dst, hipStream_t s) {
    if (n > 0) k_gather<T><<<nblocks(n, BT), BT, 0, s>>>(n, idx, src, dst);
}

template <typename T>
void launch_scatter_add(int64_t n, const int32_t *idx, const T *d, T *e, hipStream_t s) {
    if (n > 0) k_scatter_add<T><<<nblocks(n, BT), BT, 0, s>>>(n, idx, d, e);
}

template <typename T>
void launch_gather_div(int64_t n, const int32_t *idx, const T *src, const T *d, T *dst, T *x0, hipStream_t s) {
    if (n > 0) k_gather_div<T><<<nblocks(n, BT), BT, 0, s>>>(n, idx, src, d, dst, x0);
}

template <typename T>
void launch_scatter_set(int64_t n, const int32_t *map, const T *d, T *e, hipStream_t s) {
    if (n > 0) k_scatter_set<T><<<nblocks(n, BT), BT, 0, s>>>(n, map, d, e);
}

template <typename T>
void launch_lu_solve(int64_t n, const double *lu, const int32_t *perm, const T *b, T *x, hipStream_t s) {
    if (n <= 0) return;
    if (n <= kWave) k_lu_solve_wave<T><<<1, 256, 0, s>>>((int)n, lu, perm, b, x);
    else k_lu_solve<T><<<1, BT, (size_t)n * sizeof(double), s>>>(n, lu, perm, b, x);
}

#define MGR_INSTANTIATE(T)                                                                                      \
    template void launch_amg_tail<T>(const TailDesc<T> &, hipStream_t);                                       \
    template void launch_csr<T>(int, const DCsr &, const T *, const T *, const T *, const T *, T *, hipStream_t,    \
                                KEvents);                                                                           \
    template void launch_csr_restrict_div<T>(const DCsr &, const T *, const T *, const T *, T *, T *, hipStream_t); \
    template void launch_csr_prolong_into<T>(const DCsr &, const T *, const T *, const T *, const int32_t *,     \
                                             const int32_t *, T *, hipStream_t);                                \
    template void launch_csr_rows_residual<T>(const DCsr &, int, const T *, int64_t, const int32_t *, const T *, \
                                              const T *, T *, hipStream_t);                                     \
    template void launch_frelax_inplace<T>(const DCsr &, int, const T *, int64_t, const int32_t *, const T *,   \
                                           const T *, T *, hipStream_t);                                        \
    template void launch_block_apply<T>(int64_t, int, const T *, const T *, T *, bool, hipStream_t);            \
    template void launch_frelax_first<T>(int64_t, const int32_t *, const T *, const T *, T *, hipStream_t);     \
    template void launch_frelax_first_compact<T>(int64_t, const int32_t *, const T *, const T *, T *,           \
                                                 hipStream_t);                                                  \
    template void launch_prolong_inject_compact<T>(int64_t, const int32_t *, const int32_t *, const T *,        \
                                                   const T *, T *, hipStream_t);                                \
    template void launch_frelax_scatter<T>(int64_t, const int32_t *, const T *, const T *, T *, hipStream_t);   \
    template void launch_div<T>(int64_t, const T *, const T *, T *, hipStream_t);                               \
    template void launch_gather<T>(int64_t, const int32_t *, const T *, T *, hipStream_t);                      \
    template void launch_scatter_add<T>(int64_t, const int32_t *, const T *, T *, hipStream_t);                 \
    template void launch_gather_div<T>(int64_t, const int32_t *, const T *, const T *, T *, T *, hipStream_t);   \
    template void launch_scatter_set<T>(int64_t, const int32_t *, const T *, T *, hipStream_t);                 \
    template void launch_lu_solve<T>(int64_t, const double *, const int32_t *, const T *, T *, hipStream_t);

MGR_INSTANTIATE(double)
MGR_INSTANTIATE(float)

}  // namespace mgr
