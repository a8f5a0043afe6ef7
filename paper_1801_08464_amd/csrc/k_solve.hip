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
template <typename T, int MODE>
struct RowIn {
    T a = 0, b = 0, c = 0;
    __device__ inline void load(int64_t row, const T *__restrict__ x, const T *__restrict__ r,
                                const T *__restrict__ d, const T *__restrict__ y) {
        if (MODE == 1) a = r[row];
        if (MODE == 2) a = y[row];
        if (MODE == 3) {
            a = x[row];
            b = r[row];
        }
        if (MODE == 3 || MODE == 4) c = d[row];
    }
    __device__ inline void store(int64_t row, T acc, T *__restrict__ y, T *__restrict__ y2) const {
        if (MODE == 0) y[row] = acc;
        else if (MODE == 1) y[row] = a - acc;
        else if (MODE == 2) y[row] = a + acc;
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
template <typename T, int MODE, int LDSN>
__global__ void __launch_bounds__(kJagRows) k_jag_stream(int64_t nrows, const int32_t *__restrict__ rp,
                                                         const int32_t *__restrict__ jci, const T *__restrict__ jv,
                                                         const int32_t *__restrict__ jrows,
                                                         const int32_t *__restrict__ bst,
                                                         const int32_t *__restrict__ st, const T *__restrict__ x,
                                                         const T *__restrict__ r, const T *__restrict__ d,
                                                         T *__restrict__ y, T *__restrict__ y2) {
    constexpr int NT = kJagRows;
    constexpr int B = LDSN / NT;
    __shared__ T sh[LDSN];
    __shared__ int sst[kJagMaxSlots + 1];
    const int tid = threadIdx.x;
    const int64_t blk = xcd_grouped_block<kXcdGroupRows / kJagRows>();
    const int64_t rb = blk * NT;
    const int64_t re = rb + NT < nrows ? rb + NT : nrows;
    const int p0 = rp[rb];
    const int total = rp[re] - p0;
    const int t0 = bst[blk], nsl = bst[blk + 1] - t0;  // maxlen + 1 slot starts
    for (int k = tid; k < nsl; k += NT) sst[k] = st[t0 + k];
    const bool owner = rb + tid < re;
    const int64_t row = owner ? jrows[rb + tid] : 0;
    __syncthreads();
    // the owner's row length: the number of slots holding more than tid rows
    int len = 0;
    if (owner) {
        int lo = 0, hi = nsl - 1;  // slots [0, hi) all have count > tid iff ...
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (sst[mid + 1] - sst[mid] > tid) lo = mid + 1;
            else hi = mid;
        }
        len = lo;
    }
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
            j[u] = q < w1 ? __builtin_nontemporal_load(jci + p0 + q) : -1;
            av[u] = q < w1 ? __builtin_nontemporal_load(jv + p0 + q) : (T)0;
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
// min(len, k), and the entries in slot order.
__global__ void __launch_bounds__(kJagRows) k_jag_fill(int64_t nrows, const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ ci, const double *__restrict__ v,
                                                       const int32_t *__restrict__ bst, int32_t *__restrict__ st,
                                                       int32_t *__restrict__ jrows, int32_t *__restrict__ jci,
                                                       double *__restrict__ jv) {
    __shared__ int slen[kJagRows];
    __shared__ int sst[kJagMaxSlots + 1];
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
    }
    __syncthreads();
    if (t >= nr) return;
    jrows[rb + rank] = (int32_t)i;
    const int p0 = rp[rb], a = rp[i];
    for (int k = 0; k < len; ++k) {
        const int q = p0 + sst[k] + rank;
        jci[q] = ci[a + k];
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

}  // namespace

constexpr int BT = 256;

template <typename T, int ROWS, int NT, int LDSN>
static void csr_rows(int mode, const DCsr &A, const T *vals, const T *x, const T *r, const T *d, T *y, T *y2,
                     hipStream_t s) {
    const unsigned g = nblocks(A.nrows, ROWS);
#define MGR_STREAM(M) k_csr_stream<T, M, ROWS, NT, LDSN><<<g, NT, 0, s>>>(A.nrows, A.rp, A.ci, vals, x, r, d, y, y2)
    switch (mode) {
    case 0: MGR_STREAM(0); break;
    case 1: MGR_STREAM(1); break;
    case 2: MGR_STREAM(2); break;
    case 3: MGR_STREAM(3); break;
    default: MGR_STREAM(4); break;
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
static void jag_rows(int mode, const DCsr &A, const T *x, const T *r, const T *d, T *y, T *y2, hipStream_t s) {
    const Jag &J = *A.jag;
    // passes of 4864 FP64 entries (19 per thread): with the 2 KB slot table the
    // workgroup takes 40 KB of LDS, four per CU (5120 would leave three: +5 %
    // on the coarse-grid sweep); FP32 8192
    constexpr int LDSN = sizeof(T) == 4 ? 8192 : 4864;
    const unsigned g = (unsigned)J.nblk;
#define MGR_JAG(M)                                                                                          \
    k_jag_stream<T, M, LDSN><<<g, kJagRows, 0, s>>>(A.nrows, A.rp, J.ci, jag_vals<T>(J), J.rows, J.bst, J.st, x, \
                                                    r, d, y, y2)
    switch (mode) {
    case 0: MGR_JAG(0); break;
    case 1: MGR_JAG(1); break;
    case 2: MGR_JAG(2); break;
    case 3: MGR_JAG(3); break;
    default: MGR_JAG(4); break;
    }
#undef MGR_JAG
}

template <typename T, int MODE>
static void csr_lanes(const DCsr &A, int lanes, const T *vals, const T *x, const T *r, const T *d, T *y, T *y2,
                      hipStream_t s) {
    const unsigned g = nblocks(A.nrows * lanes, BT);
#define MGR_LANES(L) k_csr_lanes<T, MODE, L><<<g, BT, 0, s>>>(A.nrows, A.rp, A.ci, vals, x, r, d, y, y2)
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
// take the lanes-per-row kernel, whose launches are latency-bound anyway.
constexpr int64_t kCsrStreamMinRows = 131072;
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
                    hipStream_t s) {
    if (A.nrows <= 0) return;
    const double avg = (double)A.nnz / (double)A.nrows;
    if (A.nrows >= kCsrStreamMinRows) {
        if (A.jag && avg >= kStreamMidRow) {
            jag_rows<T>(mode, A, x, r, d, y, y2, s);
            return;
        }
        if (avg < kStreamShortRow) csr_rows<T, 256, 256, 1024>(mode, A, vals, x, r, d, y, y2, s);
        else if (avg < kStreamMidRow) csr_rows<T, 256, 256, 2048>(mode, A, vals, x, r, d, y, y2, s);
        else if (sizeof(T) == 4) csr_rows<T, 256, 256, 8192>(mode, A, vals, x, r, d, y, y2, s);
        else csr_rows<T, 256, 256, 5120>(mode, A, vals, x, r, d, y, y2, s);
        return;
    }
    if (A.nrows >= kCsrStreamSmallRows) {
        if (avg >= 24) csr_rows<T, 64, 256, 4864>(mode, A, vals, x, r, d, y, y2, s);
        else if (avg >= 12) csr_rows<T, 128, 256, 4864>(mode, A, vals, x, r, d, y, y2, s);
        else csr_rows<T, 256, 256, 2048>(mode, A, vals, x, r, d, y, y2, s);
        return;
    }
    const int lanes = avg < 3 ? 2 : avg < 6 ? 4 : avg < 12 ? 8 : avg < 24 ? 16 : 32;
    switch (mode) {
    case 0: csr_lanes<T, 0>(A, lanes, vals, x, r, d, y, y2, s); break;
    case 1: csr_lanes<T, 1>(A, lanes, vals, x, r, d, y, y2, s); break;
    case 2: csr_lanes<T, 2>(A, lanes, vals, x, r, d, y, y2, s); break;
    case 3: csr_lanes<T, 3>(A, lanes, vals, x, r, d, y, y2, s); break;
    default: csr_lanes<T, 4>(A, lanes, vals, x, r, d, y, y2, s); break;
    }
}

bool csr_long_rows(const DCsr &A) {
    return A.nrows >= kCsrStreamMinRows && (double)A.nnz >= kStreamMidRow * (double)A.nrows;
}

void launch_jag_count(const DCsr &A, int32_t *cnt, hipStream_t s) {
    const unsigned g = nblocks(A.nrows, kJagRows);
    if (g) k_jag_count<<<g, kJagRows, 0, s>>>(A.nrows, A.rp, cnt);
}

void launch_jag_fill(const DCsr &A, Jag &J, hipStream_t s) {
    if (J.nblk) k_jag_fill<<<(unsigned)J.nblk, kJagRows, 0, s>>>(A.nrows, A.rp, A.ci, A.v, J.bst, J.st, J.rows, J.ci, J.v);
}

template <typename T>
void launch_csr(int mode, const DCsr &A, const T *vals, const T *x, const T *r, const T *d, T *y, hipStream_t s) {
    csr_any<T>(mode, A, vals, x, r, d, y, nullptr, s);
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
    template void launch_csr<T>(int, const DCsr &, const T *, const T *, const T *, const T *, T *, hipStream_t); \
    template void launch_csr_restrict_div<T>(const DCsr &, const T *, const T *, const T *, T *, T *, hipStream_t); \
    template void launch_csr_rows_residual<T>(const DCsr &, int, const T *, int64_t, const int32_t *, const T *, \
                                              const T *, T *, hipStream_t);                                     \
    template void launch_frelax_inplace<T>(const DCsr &, int, const T *, int64_t, const int32_t *, const T *,   \
                                           const T *, T *, hipStream_t);                                        \
    template void launch_block_apply<T>(int64_t, int, const T *, const T *, T *, bool, hipStream_t);            \
    template void launch_frelax_first<T>(int64_t, const int32_t *, const T *, const T *, T *, hipStream_t);     \
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
