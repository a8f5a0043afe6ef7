// Setup-phase kernels of the MGR hierarchy and the classical AMG below it.
//
// Every floating-point result here is produced by the same sequence of IEEE
// operations (one rounding per product, sum or quotient; no contraction) that
// the method's definition fixes, so the hierarchy is bit-for-bit reproducible:
// sums run in ascending column/index order, SpGEMM accumulates each output
// entry over ascending k, and the PMIS rounds are synchronous with integer
// keys.
#include <climits>

#include "mgr_impl.h"

namespace mgr {
namespace {

__device__ inline int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }

__device__ inline double row_diag(const int32_t *rp, const int32_t *ci, const double *v, int64_t i) {
    for (int p = rp[i]; p < rp[i + 1]; ++p)
        if (ci[p] == i) return v[p];
    return 0.0;
}

// ---------------- validation ----------------
// Counters and flags over a whole pass are reduced per workgroup, then one
// atomic per workgroup: same-address device atomics serialise across the XCDs
// (one per wavefront cost ~250 us per 2 M rows), so these kernels stride over
// their rows with at most kReduceBlocks workgroups.
constexpr int kReduceBlocks = 1024;
constexpr int kReduceBT = 256;

__device__ inline int block_sum_i32(int v, int *sh) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) sh[threadIdx.x / kWave] = v;
    __syncthreads();
    int t = 0;
    for (int k = 0; k < kReduceBT / kWave; ++k) t += sh[k];
    return t;
}

__device__ inline unsigned block_or_u32(unsigned v, int *sh) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v |= (unsigned)__shfl_xor((int)v, o);
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) sh[threadIdx.x / kWave] = (int)v;
    __syncthreads();
    unsigned t = 0;
    for (int k = 0; k < kReduceBT / kWave; ++k) t |= (unsigned)sh[k];
    return t;
}

// err[0] |= 1 on a bad row; err[1] = max label; err[2] |= 1 on a label outside [0, 31]
__global__ void __launch_bounds__(kReduceBT) k_validate(int64_t n, int64_t nnz, const int32_t *rp,
                                                        const int32_t *ci, const int32_t *lab, int *err) {
    __shared__ int sh[kReduceBT / kWave];
    bool bad = false, badlab = false;
    unsigned bits = 0;  // the labels present
    for (int64_t i = gtid(); i < n; i += (int64_t)gridDim.x * kReduceBT) {
        const int a = rp[i], b = rp[i + 1];
        bool rbad = a < 0 || b < a || (int64_t)b > nnz;
        if (!rbad) {
            // no early exit: the column loads of a row do not wait for each other
            int prev = -1;
            for (int p = a; p < b; ++p) {
                const int c = ci[p];
                rbad = rbad || c <= prev || (int64_t)c >= n;  // c <= prev also catches c < 0
                prev = c;
            }
        }
        bad = bad || rbad;
        if (lab) {
            const int L = lab[i];
            if (L < 0 || L > 31) badlab = true;
            else bits |= 1u << L;
        }
    }
    const unsigned f = block_or_u32((bad ? 1u : 0u) | (badlab ? 2u : 0u), sh);
    const unsigned lb = block_or_u32(bits, sh);
    if (threadIdx.x == 0) {
        if (f & 1u) atomicOr(&err[0], 1);
        if (f & 2u) atomicOr(&err[2], 1);
        if (lb) atomicMax(&err[1], 31 - __builtin_clz(lb));
    }
}

// ---------------- cell-sliced ELL of the level-0 operator ----------------
__global__ void k_rowlen(int64_t n, const int32_t *rp, int32_t *len) {
    int64_t i = gtid();
    if (i < n) len[i] = rp[i + 1] - rp[i];
}

// width of (slice s, component v) = longest row of that component in the slice
__global__ void k_csell_width(int64_t nslice, int bs, int64_t ncell, const int32_t *rowlen, int32_t *width) {
    int64_t g = gtid();
    if (g >= nslice * bs) return;
    int64_t s = g / bs;
    int v = (int)(g % bs);
    int w = 0;
    for (int l = 0; l < kWave; ++l) {
        int64_t c = s * kWave + l;
        if (c >= ncell) break;
        int x = rowlen[c * bs + v];
        w = x > w ? x : w;
    }
    width[g] = w;
}

__global__ void k_csell_fill(int64_t ncell, int bs, const int32_t *rp, const int32_t *ci, const double *v,
                             const int32_t *off, const int32_t *width, int32_t *col, double *val) {
    int64_t i = gtid();
    if (i >= ncell * bs) return;
    int64_t c = i / bs;
    int comp = (int)(i % bs);
    int64_t s = c / kWave;
    int lane = (int)(c % kWave);
    int64_t o = off[s * bs + comp];
    int w = width[s * bs + comp];
    int a = rp[i], len = rp[i + 1] - a;
    for (int t = 0; t < len && t < w; ++t) {
        int64_t idx = (o + t) * kWave + lane;
        col[idx] = ci[a + t];
        val[idx] = v[a + t];
    }
}

// one wavefront per slot of 64 lanes: the slot's smallest column (padding
// excluded), then each lane's offset from it
__global__ void k_csell_pack16(int64_t nslot, const int32_t *__restrict__ col, int32_t *__restrict__ sb,
                               uint16_t *__restrict__ co, int *bad) {
    const int64_t slot = gtid() / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (slot >= nslot) return;  // uniform per wavefront
    const int c = col[slot * kWave + lane];
    int m = c >= 0 ? c : INT_MAX;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const int y = __shfl_xor(m, o);
        m = y < m ? y : m;
    }
    if (lane == 0) sb[slot] = m == INT_MAX ? 0 : m;
    const unsigned off = c >= 0 ? (unsigned)(c - m) : 0xffffu;
    if (c >= 0 && off >= 0xffffu) *bad = 1;
    co[slot * kWave + lane] = (uint16_t)off;
}

// ---------------- global relaxation: cell-block inverses ----------------
// planes: binv[(r*3+q)*ncell + c] = (B_c^{-1})_{rq}; det by cofactor expansion
// along row 0 and inv_ij = cof_ji * (1/det).  err[3] = smallest singular cell.
__global__ void k_block_inverse(int64_t ncell, int bs, const int32_t *rp, const int32_t *ci, const double *v,
                                double *binv, int *err) {
    int64_t c = gtid();
    if (c >= ncell) return;
    double a[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    int64_t lo = (int64_t)bs * c, hi = lo + bs;
    for (int r = 0; r < bs; ++r) {
        int64_t i = lo + r;
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            int64_t j = ci[p];
            if (j >= lo && j < hi) a[r][j - lo] = v[p];
        }
    }
    if (bs == 1) {
        if (a[0][0] == 0.0) {
            atomicMin(&err[3], (int)c);
            binv[c] = 0.0;
        } else {
            binv[c] = 1.0 / a[0][0];
        }
        return;
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
    if (det == 0.0 || !isfinite(det)) atomicMin(&err[3], (int)c);
    double id = 1.0 / det;
    binv[0 * ncell + c] = c00 * id;
    binv[1 * ncell + c] = c10 * id;
    binv[2 * ncell + c] = c20 * id;
    binv[3 * ncell + c] = c01 * id;
    binv[4 * ncell + c] = c11 * id;
    binv[5 * ncell + c] = c21 * id;
    binv[6 * ncell + c] = c02 * id;
    binv[7 * ncell + c] = c12 * id;
    binv[8 * ncell + c] = c22 * id;
}

// ---------------- MGR level construction ----------------
__global__ void k_level_flags(int64_t n, const int32_t *lab, int l, int32_t *isF, int32_t *isC) {
    int64_t i = gtid();
    if (i >= n) return;
    isF[i] = lab[i] == l;
    isC[i] = lab[i] > l;
}

__global__ void k_level_maps(int64_t n, const int32_t *lab, int l, const int32_t *fpos, const int32_t *cpos,
                             int32_t *fmap, int32_t *cmap, int32_t *flist, int32_t *clist) {
    int64_t i = gtid();
    if (i >= n) return;
    if (lab[i] == l) {
        fmap[i] = fpos[i];
        cmap[i] = -1;
        flist[fpos[i]] = (int32_t)i;
    } else {
        fmap[i] = -1;
        cmap[i] = cpos[i];
        clist[cpos[i]] = (int32_t)i;
    }
}

// dinv_f = 1 / a_ii (i = flist[f]); err[3] = smallest level-local row with a zero diagonal.
// offdiag |= 1 if some F row couples to another F point (A_FF not diagonal).
// (grid-stride over at most kReduceBlocks workgroups: the off-diagonal flag is
// reduced per workgroup)
__global__ void __launch_bounds__(kReduceBT) k_fdiag_inverse(int64_t nF, const int32_t *flist, const int32_t *rp,
                                                             const int32_t *ci, const double *v, double *dinv,
                                                             int *err, int *offdiag, const int32_t *fmap) {
    __shared__ int sh[kReduceBT / kWave];
    bool off = false;
    for (int64_t f = gtid(); f < nF; f += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = flist[f];
        double d = 0.0;
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            const int64_t j = ci[p];
            if (j == i) d = v[p];
            else if (fmap[j] >= 0) off = true;
        }
        if (d == 0.0) {
            atomicMin(&err[3], (int)i);
            dinv[f] = 0.0;
        } else {
            dinv[f] = 1.0 / d;
        }
    }
    if (block_or_u32(off ? 1u : 0u, sh) && threadIdx.x == 0) atomicOr(offdiag, 1);
}

// R = [W_r, I_C]: rows = C points, columns = level-local indices
__global__ void k_r_count(int64_t nC, const int32_t *clist, const int32_t *rp, const int32_t *ci,
                          const int32_t *fmap, int rp_type, int32_t *cnt) {
    int64_t c = gtid();
    if (c >= nC) return;
    int64_t u = clist[c];
    int k = 1;
    if (rp_type != 1)
        for (int p = rp[u]; p < rp[u + 1]; ++p) k += fmap[ci[p]] >= 0;
    cnt[c] = k;
}

__global__ void k_r_fill(int64_t nC, const int32_t *clist, const int32_t *rp, const int32_t *ci, const double *v,
                         const int32_t *fmap, const double *dinv, int rp_type, const int32_t *Rrp, int32_t *Rci,
                         double *Rv) {
    int64_t c = gtid();
    if (c >= nC) return;
    int u = clist[c];
    int q = Rrp[c];
    bool placed = false;
    if (rp_type != 1) {
        for (int p = rp[u]; p < rp[u + 1]; ++p) {
            int j = ci[p];
            if (!placed && j > u) {
                Rci[q] = u;
                Rv[q] = 1.0;
                q++;
                placed = true;
            }
            int f = fmap[j];
            if (f < 0) continue;
            Rci[q] = j;
            Rv[q] = -(v[p] * dinv[f]);
            q++;
        }
    }
    if (!placed) {
        Rci[q] = u;
        Rv[q] = 1.0;
    }
}

__global__ void k_gather_i32(int64_t n, const int32_t *idx, const int32_t *src, int32_t *dst) {
    int64_t i = gtid();
    if (i < n) dst[i] = src[idx[i]];
}

// ---------------- SpGEMM: one wavefront per output row ----------------
// Lane l holds the entries t = l, l+64, ... of row i of A (ascending k) and a
// cursor into row k of B.  Each step takes the smallest head column j over the
// wavefront; the contributions to C_ij are summed in ascending t (= ascending
// k) by walking the ballot mask, starting from 0.0.  Patterns are symbolic.
constexpr int kSpgChunks = 8;

template <int G>
__device__ inline int group_min_i32(int v) {
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
        int o = __shfl_xor(v, off);
        v = o < v ? o : v;
    }
    return v;
}

// G lanes (an aligned group of the wavefront) per output row.  Each lane keeps,
// per chunk, the head column and (fill pass) the head value of its B row, loaded
// together so a merge step waits on one load.  Output t of the row is held by
// lane t mod G and the group writes G outputs at a time (coalesced).  NCH chunks
// per lane (rows of up to G * NCH entries): the fill pass takes the fewest that
// hold the operand's longest row, since its registers per chunk set how many
// wavefronts a SIMD holds, and the merge waits on loads.
template <bool FILL, int G, int NCH>
__global__ void __launch_bounds__(256) k_spgemm(int64_t m, const int32_t *__restrict__ Arp,
                                                const int32_t *__restrict__ Aci, const double *__restrict__ Av,
                                                const int32_t *__restrict__ Brp, const int32_t *__restrict__ Bci,
                                                const double *__restrict__ Bv, int32_t *cnt_or_Crp,
                                                int32_t *__restrict__ Cci, double *__restrict__ Cv, int *err) {
    const int glane = threadIdx.x & (G - 1);
    const int gbase = (threadIdx.x & (kWave - 1)) & ~(G - 1);
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x / G) + (threadIdx.x / G);
    if (row >= m) return;  // uniform per group
    const int a0 = Arp[row];
    const int len = Arp[row + 1] - a0;
    if (len > G * NCH) {  // too long for this group size: flagged, counted as empty
        if (glane == 0) {
            atomicOr(err, 1);
            if (!FILL) cnt_or_Crp[row] = 0;
        }
        return;
    }
    const unsigned long long gmask = G == 64 ? ~0ull : ((1ull << G) - 1);
    const int nch = (len + G - 1) / G;
    int p[NCH], e[NCH], hd[NCH];
    double av[NCH], hv[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        p[c] = 0;
        e[c] = 0;
        hd[c] = INT_MAX;
        av[c] = 0.0;
        hv[c] = 0.0;
        int t = c * G + glane;
        if (c < nch && t < len) {
            int k = Aci[a0 + t];
            if (FILL) av[c] = Av[a0 + t];
            p[c] = Brp[k];
            e[c] = Brp[k + 1];
            if (p[c] < e[c]) {
                hd[c] = Bci[p[c]];
                if (FILL) hv[c] = Bv[p[c]];
            }
        }
    }
    int out = FILL ? cnt_or_Crp[row] : 0;
    int count = 0;
    int my_j = 0;
    double my_v = 0.0;
    for (;;) {
        int mn = INT_MAX;
#pragma unroll
        for (int c = 0; c < NCH; ++c)
            if (c < nch) mn = hd[c] < mn ? hd[c] : mn;
        mn = group_min_i32<G>(mn);
        if (mn == INT_MAX) break;
        if (FILL) {
            double acc = 0.0;
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                if (c < nch) {
                    bool hit = hd[c] == mn;
                    double prod = hit ? av[c] * hv[c] : 0.0;
                    unsigned long long mask = (__ballot(hit) >> gbase) & gmask;
                    while (mask) {
                        int l = __builtin_ctzll(mask);
                        acc = acc + __shfl(prod, gbase + l);
                        mask &= mask - 1;
                    }
                }
            }
            const int slot = count & (G - 1);
            if (glane == slot) {
                my_j = mn;
                my_v = acc;
            }
            if (slot == G - 1) {
                Cci[out + count - (G - 1) + glane] = my_j;
                Cv[out + count - (G - 1) + glane] = my_v;
            }
        }
        count++;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            if (c < nch && hd[c] == mn) {
                p[c]++;
                if (p[c] < e[c]) {
                    hd[c] = Bci[p[c]];
                    if (FILL) hv[c] = Bv[p[c]];
                } else {
                    hd[c] = INT_MAX;
                }
            }
        }
    }
    if (FILL) {
        // the last count mod G outputs
        const int rem = count & (G - 1);
        if (glane < rem) {
            Cci[out + count - rem + glane] = my_j;
            Cv[out + count - rem + glane] = my_v;
        }
    }
    if (!FILL && glane == 0) cnt_or_Crp[row] = count;
}

// sum and maximum of the lengths of rows list[0..m) (or rows 0..m when list is null):
// a fixed grid strides over the rows, reduces per workgroup, and issues one
// integer atomic per workgroup (so few atomics meet at one address)
constexpr int kLenStatBlocks = 512;
constexpr int kLenStatBT = 256;
__global__ void __launch_bounds__(kLenStatBT) k_row_len_stats(int64_t m, const int32_t *list, const int32_t *rp, int *sum,
                                                      int *mx) {
    __shared__ int ss[kLenStatBT / kWave], sm[kLenStatBT / kWave];
    int s = 0, x = 0;
    for (int64_t q = gtid(); q < m; q += (int64_t)gridDim.x * kLenStatBT) {
        const int64_t i = list ? list[q] : q;
        const int len = rp[i + 1] - rp[i];
        s += len;
        x = len > x ? len : x;
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        s += __shfl_xor(s, o);
        const int y = __shfl_xor(x, o);
        x = y > x ? y : x;
    }
    const int wv = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        ss[wv] = s;
        sm[wv] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kLenStatBT / kWave; ++k) {
            s += ss[k];
            x = sm[k] > x ? sm[k] : x;
        }
        if (sum) atomicAdd(sum, s);
        atomicMax(mx, x);
    }
}

// ---------------- stable transpose ----------------
__global__ void k_transpose_count(int64_t nrows, const int32_t *rp, const int32_t *ci, int32_t *cnt) {
    int64_t i = gtid();
    if (i >= nrows) return;
    for (int p = rp[i]; p < rp[i + 1]; ++p) atomicAdd(&cnt[ci[p]], 1);
}

__global__ void k_transpose_fill(int64_t nrows, const int32_t *rp, const int32_t *ci, const double *v, int32_t *next,
                                 int32_t *Tci, double *Tv) {
    int64_t i = gtid();
    if (i >= nrows) return;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        int slot = atomicAdd(&next[ci[p]], 1);
        Tci[slot] = (int32_t)i;
        if (Tv) Tv[slot] = v[p];
    }
}

// ---------------- classical strength of connection ----------------
// j in S_i iff j != i, m_i > 0 and -s_i a_ij >= theta m_i, s_i = sign of a_ii (+ for 0)
// G lanes per row: the diagonal by ballot, m_i by a group max (exact in any
// order), the strong entries counted by a group sum and (FILL) written in
// ascending column order through ballot prefix counts.
template <bool FILL, int G>
__global__ void __launch_bounds__(256) k_strength(int64_t n, const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci, const double *__restrict__ v,
                                                  double theta, int32_t *cnt_or_Srp, int32_t *__restrict__ Sci,
                                                  uint8_t *__restrict__ sflag) {
    const int glane = threadIdx.x & (G - 1);
    const int gbase = (threadIdx.x & (kWave - 1)) & ~(G - 1);
    const unsigned long long gmask = G == 64 ? ~0ull : ((1ull << G) - 1);
    const unsigned long long below = glane == 0 ? 0ull : ((1ull << glane) - 1);
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x / G) + (threadIdx.x / G);
    if (i >= n) return;  // uniform per group
    const int a = rp[i], b = rp[i + 1];
    double dl = 0.0;
    bool has = false;
    for (int p = a + glane; p < b; p += G)
        if (ci[p] == i) {
            dl = v[p];
            has = true;
        }
    const unsigned long long md = (__ballot(has) >> gbase) & gmask;
    const double d = md ? __shfl(dl, gbase + __builtin_ctzll(md)) : 0.0;
    const bool pos = d >= 0.0;
    double m = -INFINITY;
    for (int p = a + glane; p < b; p += G) {
        if (ci[p] == i) continue;
        const double t = pos ? -v[p] : v[p];
        if (t > m) m = t;
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
        const double o = __shfl_xor(m, off);
        m = o > m ? o : m;
    }
    const double thr = theta * m;
    const int q = FILL ? cnt_or_Srp[i] : 0;
    int cnt = 0;
    for (int p0 = a; p0 < b; p0 += G) {
        const int p = p0 + glane;
        bool strong = false;
        int j = -1;
        if (p < b) {
            j = ci[p];
            if (j != i && m > 0.0) {
                const double t = pos ? -v[p] : v[p];
                strong = t >= thr;
            }
        }
        const unsigned long long ms = (__ballot(strong) >> gbase) & gmask;
        if (FILL) {
            if (strong) Sci[q + cnt + __popcll(ms & below)] = j;
            if (p < b) sflag[p] = strong ? 1 : 0;
        }
        cnt += __popcll(ms);
    }
    if (!FILL && glane == 0) cnt_or_Srp[i] = cnt;
}

// ---------------- PMIS ----------------
__device__ inline uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

__global__ void k_pmis_init(int64_t n, const int32_t *STrp, int32_t *state) {
    int64_t i = gtid();
    if (i >= n) return;
    state[i] = (STrp[i + 1] - STrp[i]) == 0 ? -1 : 0;
}

__device__ inline bool key_gt(int li, uint64_t hi, int64_t i, int lj, uint64_t hj, int64_t j) {
    if (li != lj) return li > lj;
    if (hi != hj) return hi > hj;
    return i > j;
}

// newc[i] = 1 iff i is undecided and its key (lambda, hash, index) exceeds the
// key of every undecided point in S_i and S_i^T (state of the round's start)
__global__ void k_pmis_select(int64_t n, const int32_t *Srp, const int32_t *Sci, const int32_t *STrp,
                              const int32_t *STci, const int32_t *state, uint64_t seed, int32_t *newc) {
    int64_t i = gtid();
    if (i >= n) return;
    if (state[i] != 0) {
        newc[i] = 0;
        return;
    }
    int li = STrp[i + 1] - STrp[i];
    uint64_t hi = splitmix64(seed ^ (uint64_t)i);
    bool ok = true;
    for (int p = Srp[i]; p < Srp[i + 1] && ok; ++p) {
        int64_t j = Sci[p];
        if (state[j] == 0 && !key_gt(li, hi, i, STrp[j + 1] - STrp[j], splitmix64(seed ^ (uint64_t)j), j)) ok = false;
    }
    for (int p = STrp[i]; p < STrp[i + 1] && ok; ++p) {
        int64_t j = STci[p];
        if (state[j] == 0 && !key_gt(li, hi, i, STrp[j + 1] - STrp[j], splitmix64(seed ^ (uint64_t)j), j)) ok = false;
    }
    newc[i] = ok ? 1 : 0;
}

// new C points become C; undecided points that strongly depend on a new C point become F.
// counters[0] += undecided left, counters[1] += new C points (reduced per workgroup,
// one atomic each).
__global__ void __launch_bounds__(kReduceBT) k_pmis_update(int64_t n, const int32_t *Srp, const int32_t *Sci,
                                                           const int32_t *newc, int32_t *state, int *counters) {
    __shared__ int sh[kReduceBT / kWave];
    int und = 0, nc = 0;
    for (int64_t i = gtid(); i < n; i += (int64_t)gridDim.x * kReduceBT) {
        if (newc[i]) {
            state[i] = 1;
            ++nc;
        } else if (state[i] == 0) {
            bool f = false;
            for (int p = Srp[i]; p < Srp[i + 1]; ++p)
                if (newc[Sci[p]]) {
                    f = true;
                    break;
                }
            if (f) state[i] = -1;
            else ++und;
        }
    }
    const int cu = block_sum_i32(und, sh), cc = block_sum_i32(nc, sh);
    if (threadIdx.x == 0) {
        if (cu) atomicAdd(&counters[0], cu);
        if (cc) atomicAdd(&counters[1], cc);
    }
}

__global__ void k_cf_flags(int64_t n, const int32_t *state, int32_t *isC) {
    int64_t i = gtid();
    if (i < n) isC[i] = state[i] == 1;
}

// ---------------- classical interpolation ----------------
__global__ void k_interp_count(int64_t n, const int32_t *rp, const int32_t *ci, const uint8_t *sflag,
                               const int32_t *cf, int32_t *cnt) {
    int64_t i = gtid();
    if (i >= n) return;
    if (cf[i] == 1) {
        cnt[i] = 1;
        return;
    }
    int c = 0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) c += (sflag[p] && cf[ci[p]] == 1);
    cnt[i] = c;
}

__device__ inline int find_col(const int32_t *cols, int len, int key) {
    int lo = 0, hi = len - 1;
    while (lo <= hi) {
        int mid = (lo + hi) >> 1;
        int x = cols[mid];
        if (x == key) return mid;
        if (x < key) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

// For F-point i (C_i strong C neighbours, F_i strong F neighbours, W_i the rest):
// atil = a_ii + sum_W a_in; for k in F_i ascending: den = sum_{m in C_i} abar_km
// (abar_km = a_km when a_km a_kk < 0, else 0); den == 0 lumps a_ik into atil,
// otherwise num_j += (a_ik abar_kj) / den; w_ij = -((a_ij + num_j) / atil).
constexpr int kInterpMaxC = 256;  // strong C neighbours per row held in LDS by the wavefront form

__global__ void k_interp_fill(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                              const uint8_t *sflag, const int32_t *cf, const int32_t *cmap, const int32_t *Prp,
                              int32_t *Pci, double *Pv) {
    int64_t i = gtid();
    if (i >= n) return;
    int base = Prp[i], nci = Prp[i + 1] - base;
    // C rows and rows within the wavefront kernel's limit are written there
    if (cf[i] == 1 || nci <= kInterpMaxC) return;
    int a = rp[i], b = rp[i + 1];
    int t = 0;
    for (int p = a; p < b; ++p) {
        int j = ci[p];
        if (sflag[p] && cf[j] == 1) {
            Pci[base + t] = cmap[j];
            Pv[base + t] = 0.0;
            t++;
        }
    }
    double atil = 0.0;
    for (int p = a; p < b; ++p)
        if (ci[p] == i) atil = v[p];
    for (int p = a; p < b; ++p) {
        if (ci[p] == i) continue;
        if (!sflag[p]) atil = atil + v[p];
    }
    for (int p = a; p < b; ++p) {
        int k = ci[p];
        if (k == i || !sflag[p] || cf[k] != -1) continue;
        double aik = v[p];
        double akk = row_diag(rp, ci, v, k);
        double den = 0.0;
        for (int q = rp[k]; q < rp[k + 1]; ++q) {
            int mcol = ci[q];
            if (cf[mcol] != 1 || find_col(Pci + base, nci, cmap[mcol]) < 0) continue;
            double akm = v[q];
            double abar = (akm * akk < 0.0) ? akm : 0.0;
            den = den + abar;
        }
        if (den == 0.0) {
            atil = atil + aik;
        } else {
            for (int q = rp[k]; q < rp[k + 1]; ++q) {
                int mcol = ci[q];
                if (cf[mcol] != 1) continue;
                int pos = find_col(Pci + base, nci, cmap[mcol]);
                if (pos < 0) continue;
                double akm = v[q];
                double abar = (akm * akk < 0.0) ? akm : 0.0;
                double prod = aik * abar;
                Pv[base + pos] = Pv[base + pos] + prod / den;
            }
        }
    }
    t = 0;
    for (int p = a; p < b; ++p) {
        int j = ci[p];
        if (!(sflag[p] && cf[j] == 1)) continue;
        double s = v[p] + Pv[base + t];
        Pv[base + t] = (atil == 0.0) ? 0.0 : -(s / atil);
        t++;
    }
}

// The same interpolation with one group of G lanes per F row (the thread-per-row
// form above serialises every distance-two lookup of a row in one lane).  The
// row's strong C neighbours (ascending, at most MAXC of them), their a_ij and
// the running num_j live in LDS.  Strong F neighbours k are taken in ascending
// order; the lanes load row k together, find each column's place in the C list
// by binary search, and the sums (atil over the weak entries, den over row k)
// walk the group's ballot masks in ascending lane order, chunk after chunk, so
// every sum runs in the order above whatever G is.  G = 16 serves the rows with
// at most 32 strong C neighbours (most rows: a wavefront per row would leave
// most lanes idle; G = 8 where the matrix's rows are short), G = 64 those with
// up to kInterpMaxC; longer rows are left to k_interp_fill.

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kInterpSmallC = 32;  // strong C neighbours per row of the 16-lane form
// chunks of G entries of a strong F neighbour's row held in registers (longer
// rows take three passes over memory instead)
constexpr int kInterpRowChunks = 4;

template <int G>
struct InterpGroup {
    int lane, gbase;
    unsigned long long gmask;
    __device__ InterpGroup() {
        lane = threadIdx.x & (G - 1);
        gbase = (threadIdx.x & (kWave - 1)) & ~(G - 1);
        gmask = G == kWave ? ~0ull : ((1ull << G) - 1);
    }
    // the group's lanes where pred holds, as a G-bit mask
    __device__ unsigned long long ballot(bool pred) const { return (__ballot(pred) >> gbase) & gmask; }
    template <typename T>
    __device__ T shfl(T val, int l) const {
        return __shfl(val, gbase + l);
    }
    // acc + the values of the lanes in mask, added one at a time in ascending lane order
    __device__ double ordered_add(double acc, unsigned long long mask, double val) const {
        while (mask) {
            const int l = __builtin_ctzll(mask);
            acc = acc + __shfl(val, gbase + l);
            mask &= mask - 1;
        }
        return acc;
    }
};

// The sort of a transpose's rows (the slots were taken in arbitrary order;
// source rows are unique, so sorting by source row gives the one stable order)
// with a group of kSortLanes lanes per row: rows of up to kSortMaxLen entries
// are staged in LDS and each entry is written at its rank (the number of
// smaller keys in the row); a longer row is sorted by insertion in the group's
// first lane.
constexpr int kSortLanes = 8;
constexpr int kSortMaxLen = 64;
__global__ void __launch_bounds__(256) k_transpose_sort_grp(int64_t ncols, const int32_t *__restrict__ Trp,
                                                            int32_t *__restrict__ Tci, double *__restrict__ Tv) {
    constexpr int RPB = 256 / kSortLanes;
    __shared__ int sk[RPB][kSortMaxLen];
    __shared__ double sv[RPB][kSortMaxLen];
    const int lane = threadIdx.x & (kSortLanes - 1), w = threadIdx.x / kSortLanes;
    const int64_t j = (int64_t)blockIdx.x * RPB + w;
    if (j >= ncols) return;  // uniform per group
    const int a = Trp[j], len = Trp[j + 1] - a;
    if (len <= 1) return;
    if (len > kSortMaxLen) {
        if (lane == 0) {
            for (int p = a + 1; p < a + len; ++p) {
                const int key = Tci[p];
                const double val = Tv ? Tv[p] : 0.0;
                int q = p - 1;
                while (q >= a && Tci[q] > key) {
                    Tci[q + 1] = Tci[q];
                    if (Tv) Tv[q + 1] = Tv[q];
                    q--;
                }
                Tci[q + 1] = key;
                if (Tv) Tv[q + 1] = val;
            }
        }
        return;
    }
    int *k = sk[w];
    double *kv = sv[w];
    for (int e = lane; e < len; e += kSortLanes) {
        k[e] = Tci[a + e];
        if (Tv) kv[e] = Tv[a + e];
    }
    wave_sync();  // the group lies in one wavefront
    for (int e = lane; e < len; e += kSortLanes) {
        const int key = k[e];
        int r = 0;
        for (int f = 0; f < len; ++f) r += k[f] < key;
        Tci[a + r] = key;
        if (Tv) Tv[a + r] = kv[e];
    }
}

// ---------------- row selections: P = [W_p; I_C], A_FF, the F columns ----------------
// A group of G lanes takes one row and its entries G at a time (coalesced
// loads).  A kept entry's place is the row's start plus the number of kept
// entries before it, counted by an ordered ballot over the group, so every
// output row is in ascending column order, as a sequential loop writes it.
// keep(p, col) decides entry p and sets its output column; emit(p, col, pos)
// writes it.  Returns the row's count (the same in every lane of the group).
template <int G, typename Keep, typename Emit>
__device__ inline int group_select(const InterpGroup<G> &grp, int a, int b, int q, Keep keep, Emit emit) {
    const unsigned long long below = (1ull << grp.lane) - 1ull;
    for (int c0 = a; c0 < b; c0 += G) {
        const int p = c0 + grp.lane;
        int col = -1;
        const bool k = p < b && keep(p, col);
        const unsigned long long m = grp.ballot(k);
        if (k) emit(p, col, q + __popcll(m & below));
        q += __popcll(m);
    }
    return q;
}

// P = [W_p; I_C]: rows of the level, columns = C points.  FILL false: the row
// counts into cnt; true: the entries at Prp.
template <int G, bool FILL>
__global__ void __launch_bounds__(256) k_p_sel(int64_t n, const int32_t *__restrict__ rp,
                                               const int32_t *__restrict__ ci, const double *__restrict__ v,
                                               const int32_t *__restrict__ cmap, const int32_t *__restrict__ fmap,
                                               const double *__restrict__ dinv, int rp_type,
                                               const int32_t *__restrict__ Prp, int32_t *__restrict__ cnt,
                                               int32_t *__restrict__ Pci, double *__restrict__ Pv) {
    const InterpGroup<G> grp;
    const int64_t i = (int64_t)blockIdx.x * (256 / G) + threadIdx.x / G;
    if (i >= n) return;  // uniform per group
    const int ci_self = cmap[i];
    if (ci_self >= 0 || rp_type == 2) {  // a C row (unit row), or W_p = 0
        if (grp.lane == 0) {
            if (!FILL) cnt[i] = ci_self >= 0 ? 1 : 0;
            else if (ci_self >= 0) {
                Pci[Prp[i]] = ci_self;
                Pv[Prp[i]] = 1.0;
            }
        }
        return;
    }
    auto keep = [&](int p, int &col) {
        col = cmap[ci[p]];
        return col >= 0;
    };
    if (FILL) {
        const double di = dinv[fmap[i]];
        group_select(grp, rp[i], rp[i + 1], Prp[i], keep, [&](int p, int col, int pos) {
            Pci[pos] = col;
            Pv[pos] = -(v[p] * di);
        });
    } else {
        const int c = group_select(grp, rp[i], rp[i + 1], 0, keep, [](int, int, int) {});
        if (grp.lane == 0) cnt[i] = c;
    }
}

// A_FF: rows flist, the F columns renumbered by fmap (fmap null: every column,
// unrenumbered: the compact copy of the F rows)
template <int G, bool FILL>
__global__ void __launch_bounds__(256) k_ff_sel(int64_t nF, const int32_t *__restrict__ flist,
                                                const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                const double *__restrict__ v, const int32_t *__restrict__ fmap,
                                                const int32_t *__restrict__ Frp, int32_t *__restrict__ cnt,
                                                int32_t *__restrict__ Fci, double *__restrict__ Fv) {
    const InterpGroup<G> grp;
    const int64_t f = (int64_t)blockIdx.x * (256 / G) + threadIdx.x / G;
    if (f >= nF) return;  // uniform per group
    const int64_t i = flist[f];
    auto keep = [&](int p, int &col) {
        const int j = ci[p];
        col = fmap ? fmap[j] : j;
        return col >= 0;
    };
    if (FILL) {
        group_select(grp, rp[i], rp[i + 1], Frp[f], keep, [&](int p, int col, int pos) {
            Fci[pos] = col;
            Fv[pos] = v[p];
        });
    } else {
        const int c = fmap ? group_select(grp, rp[i], rp[i + 1], 0, keep, [](int, int, int) {}) : rp[i + 1] - rp[i];
        if (grp.lane == 0) cnt[f] = c;
    }
}

// The F columns of A (fmap >= 0) in every row.  When the error vector vanishes
// on the C points, the residual r - A e reads only these entries; the skipped
// products are exact zeros, so the row sums are unchanged.  fnum: the columns as
// F indices (fmap[j]) instead of level rows.
template <int G, bool FILL>
__global__ void __launch_bounds__(256) k_fcol_sel(int64_t n, const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci, const double *__restrict__ v,
                                                  const int32_t *__restrict__ fmap, const int32_t *__restrict__ Frp,
                                                  int32_t *__restrict__ cnt, int32_t *__restrict__ Fci,
                                                  double *__restrict__ Fv, int fnum) {
    const InterpGroup<G> grp;
    const int64_t i = (int64_t)blockIdx.x * (256 / G) + threadIdx.x / G;
    if (i >= n) return;  // uniform per group
    auto keep = [&](int p, int &col) {
        const int j = ci[p];
        const int f = fmap[j];
        col = fnum ? f : j;
        return f >= 0;
    };
    if (FILL) {
        group_select(grp, rp[i], rp[i + 1], Frp[i], keep, [&](int p, int col, int pos) {
            Fci[pos] = col;
            Fv[pos] = v[p];
        });
    } else {
        const int c = group_select(grp, rp[i], rp[i + 1], 0, keep, [](int, int, int) {});
        if (grp.lane == 0) cnt[i] = c;
    }
}

template <int G, int MAXC, int LO>
__global__ void __launch_bounds__(256) k_interp_fill_grp(
    int64_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci, const double *__restrict__ v,
    const uint8_t *__restrict__ sflag, const int32_t *__restrict__ cf, const int32_t *__restrict__ cmap,
    const int32_t *__restrict__ Prp, int32_t *__restrict__ Pci, double *__restrict__ Pv) {
    constexpr int RPB = 256 / G;  // rows per workgroup
    __shared__ int s_cols[RPB][MAXC];
    __shared__ double s_num[RPB][MAXC];
    __shared__ double s_aij[RPB][MAXC];
    const InterpGroup<G> grp;
    const int lane = grp.lane, w = threadIdx.x / G;
    const int64_t i = (int64_t)blockIdx.x * RPB + w;
    if (i >= n) return;
    const int base = Prp[i], nci = Prp[i + 1] - base;
    if (cf[i] == 1) {
        if (LO == 0 && lane == 0) {  // C rows: written by the first form only
            Pci[base] = cmap[i];
            Pv[base] = 1.0;
        }
        return;
    }
    if (nci == 0 || nci <= LO || nci > MAXC) return;
    int *cols = s_cols[w];
    double *num = s_num[w], *aij = s_aij[w];
    const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    const int a = rp[i], b = rp[i + 1];
    // Row i's entries, G at a time: from registers when the row fits in
    // kInterpRowChunks chunks (loaded once for the three passes below), else
    // from memory in each pass.  Each pass's body sees one chunk: the entry's
    // presence, column, value, strength flag and the column's C/F mark.
    const bool rowreg = b - a <= G * kInterpRowChunks;  // the same for the whole group
    int rj[kInterpRowChunks], rcf[kInterpRowChunks];
    double rv[kInterpRowChunks];
    bool rs[kInterpRowChunks];
    if (rowreg) {
#pragma unroll
        for (int u = 0; u < kInterpRowChunks; ++u) {
            const int p = a + u * G + lane;
            const bool ok = p < b;
            rj[u] = ok ? ci[p] : -1;
            rv[u] = ok ? v[p] : 0.0;
            rs[u] = ok && sflag[p];
            rcf[u] = ok ? cf[rj[u]] : 0;
        }
    }
    auto each_chunk = [&](auto &&body) {
        if (rowreg) {
#pragma unroll
            for (int u = 0; u < kInterpRowChunks; ++u)
                if (a + u * G < b) body(a + u * G + lane < b, rj[u], rv[u], rs[u], rcf[u]);
        } else {
            for (int c0 = a; c0 < b; c0 += G) {
                const int p = c0 + lane;
                const bool ok = p < b;
                const int j = ok ? ci[p] : -1;
                body(ok, j, ok ? v[p] : 0.0, ok && sflag[p], ok ? cf[j] : 0);
            }
        }
    };
    // the strong C neighbours (ascending) and the diagonal
    int nc = 0;
    double aii = 0.0;
    each_chunk([&](bool ok, int j, double vv, bool sf, int cfj) {
        const bool sc = ok && sf && cfj == 1;
        const unsigned long long m = grp.ballot(sc);
        if (sc) {
            const int pos = nc + __popcll(m & below);
            cols[pos] = cmap[j];
            aij[pos] = vv;
            num[pos] = 0.0;
            Pci[base + pos] = cmap[j];
        }
        nc += __popcll(m);
        const unsigned long long md = grp.ballot(ok && j == i);
        if (md) aii = grp.shfl(vv, __builtin_ctzll(md));
    });
    wave_sync();
    // atil = a_ii + the weak entries, ascending
    double atil = aii;
    each_chunk([&](bool ok, int j, double vv, bool sf, int) {
        const bool weak = ok && j != i && !sf;
        atil = grp.ordered_add(atil, grp.ballot(weak), vv);
    });
    // the strong F neighbours k, ascending
    each_chunk([&](bool ok, int j, double vv, bool sf, int cfj) {
        unsigned long long mk = grp.ballot(ok && j != i && sf && cfj == -1);
        while (mk) {
            const int l = __builtin_ctzll(mk);
            mk &= mk - 1;
            const int k = grp.shfl(j, l);
            const double aik = grp.shfl(vv, l);
            const int ka = rp[k], kb = rp[k + 1];
            if (kb - ka <= G * kInterpRowChunks) {
                // row k in registers: its columns and values loaded once (all
                // chunks together), its C positions found once; the same sums
                // in the same order as the passes below
                int qc[kInterpRowChunks], qp[kInterpRowChunks];
                double qv[kInterpRowChunks];
#pragma unroll
                for (int u = 0; u < kInterpRowChunks; ++u) {
                    const int q = ka + u * G + lane;
                    qc[u] = q < kb ? ci[q] : -1;
                    qv[u] = q < kb ? v[q] : 0.0;
                }
                double akk = 0.0;
#pragma unroll
                for (int u = 0; u < kInterpRowChunks; ++u) {
                    const unsigned long long md = grp.ballot(qc[u] == k);
                    if (md) akk = grp.shfl(qv[u], __builtin_ctzll(md));
                }
#pragma unroll
                for (int u = 0; u < kInterpRowChunks; ++u)
                    qp[u] = (qc[u] >= 0 && cf[qc[u]] == 1) ? find_col(cols, nc, cmap[qc[u]]) : -1;
                double den = 0.0;
#pragma unroll
                for (int u = 0; u < kInterpRowChunks; ++u) {
                    const double abar = (qv[u] * akk < 0.0) ? qv[u] : 0.0;
                    den = grp.ordered_add(den, grp.ballot(qp[u] >= 0), abar);
                }
                if (den == 0.0) {
                    atil = atil + aik;
                    continue;
                }
#pragma unroll
                for (int u = 0; u < kInterpRowChunks; ++u) {
                    if (qp[u] >= 0) {
                        const double abar = (qv[u] * akk < 0.0) ? qv[u] : 0.0;
                        const double prod = aik * abar;
                        num[qp[u]] = num[qp[u]] + prod / den;
                    }
                }
                wave_sync();
                continue;
            }
            double akk = 0.0;
            for (int d0 = ka; d0 < kb; d0 += G) {
                const int q = d0 + lane;
                const bool okq = q < kb;
                const unsigned long long md = grp.ballot(okq && ci[q] == k);
                if (md) akk = grp.shfl(okq ? v[q] : 0.0, __builtin_ctzll(md));
            }
            double den = 0.0;
            for (int d0 = ka; d0 < kb; d0 += G) {
                const int q = d0 + lane;
                const bool okq = q < kb;
                const int mcol = okq ? ci[q] : 0;
                const int pos = (okq && cf[mcol] == 1) ? find_col(cols, nc, cmap[mcol]) : -1;
                const double akm = okq ? v[q] : 0.0;
                const double abar = (akm * akk < 0.0) ? akm : 0.0;
                den = grp.ordered_add(den, grp.ballot(pos >= 0), abar);
            }
            if (den == 0.0) {
                atil = atil + aik;
                continue;
            }
            for (int d0 = ka; d0 < kb; d0 += G) {
                const int q = d0 + lane;
                const bool okq = q < kb;
                const int mcol = okq ? ci[q] : 0;
                const int pos = (okq && cf[mcol] == 1) ? find_col(cols, nc, cmap[mcol]) : -1;
                if (pos >= 0) {
                    const double akm = v[q];
                    const double abar = (akm * akk < 0.0) ? akm : 0.0;
                    const double prod = aik * abar;
                    num[pos] = num[pos] + prod / den;
                }
            }
            wave_sync();
        }
    });
    wave_sync();
    for (int t = lane; t < nc; t += G) {
        const double sum = aij[t] + num[t];
        Pv[base + t] = (atil == 0.0) ? 0.0 : -(sum / atil);
    }
}

// l1 row norms (ascending column order); err[3] = smallest empty row
__global__ void k_l1(int64_t n, const int32_t *rp, const double *v, double *l1, int *err) {
    int64_t i = gtid();
    if (i >= n) return;
    double s = 0.0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) s = s + fabs(v[p]);
    if (s == 0.0) atomicMin(&err[3], (int)i);
    l1[i] = s;
}

// ---------------- coarsest level: dense LU with partial pivoting ----------------
// One workgroup.  Pivot = first row of largest |a_ik| (ties -> lowest row).
constexpr int kLuBT = 256;
__global__ void __launch_bounds__(kLuBT) k_dense_lu(int64_t n, const int32_t *rp, const int32_t *ci,
                                                    const double *v, double *lu, int32_t *perm, int *err) {
    __shared__ double sv[kLuBT];
    __shared__ int si[kLuBT];
    __shared__ int piv_s, fail_s;
    const int tid = threadIdx.x;
    for (int64_t idx = tid; idx < n * n; idx += kLuBT) lu[idx] = 0.0;
    __syncthreads();
    for (int64_t i = tid; i < n; i += kLuBT) {
        perm[i] = (int32_t)i;
        for (int p = rp[i]; p < rp[i + 1]; ++p) lu[i * n + ci[p]] = v[p];
    }
    __syncthreads();
    for (int64_t k = 0; k < n; ++k) {
        double best = -1.0;
        int bi = (int)n;
        for (int64_t i = k + tid; i < n; i += kLuBT) {
            double a = fabs(lu[i * n + k]);
            if (a > best) {
                best = a;
                bi = (int)i;
            }
        }
        sv[tid] = best;
        si[tid] = bi;
        __syncthreads();
        for (int off = kLuBT / 2; off > 0; off >>= 1) {
            if (tid < off) {
                double ob = sv[tid + off];
                int oi = si[tid + off];
                if (ob > sv[tid] || (ob == sv[tid] && oi < si[tid])) {
                    sv[tid] = ob;
                    si[tid] = oi;
                }
            }
            __syncthreads();
        }
        if (tid == 0) {
            piv_s = si[0];
            fail_s = !(sv[0] > 0.0);
        }
        __syncthreads();
        if (fail_s) {
            if (tid == 0) atomicOr(&err[4], 1);
            return;
        }
        const int64_t piv = piv_s;
        if (piv != k) {
            for (int64_t j = tid; j < n; j += kLuBT) {
                double x = lu[k * n + j];
                lu[k * n + j] = lu[piv * n + j];
                lu[piv * n + j] = x;
            }
            if (tid == 0) {
                int32_t x = perm[k];
                perm[k] = perm[piv];
                perm[piv] = x;
            }
        }
        __syncthreads();
        const double pv = lu[k * n + k];
        for (int64_t i = k + 1 + tid; i < n; i += kLuBT) lu[i * n + k] = lu[i * n + k] / pv;
        __syncthreads();
        const int64_t w = n - k - 1;
        for (int64_t idx = tid; idx < w * w; idx += kLuBT) {
            int64_t i = k + 1 + idx / w, j = k + 1 + idx % w;
            lu[i * n + j] = lu[i * n + j] - lu[i * n + k] * lu[k * n + j];
        }
        __syncthreads();
    }
}

__global__ void k_pattern_outer(int64_t n, const int32_t *rp, const int32_t *ci, const double *lam, const double *x,
                                double *d) {
    int64_t i = gtid();
    if (i >= n) return;
    double li = lam[i];
    for (int p = rp[i]; p < rp[i + 1]; ++p) d[p] = -(li * x[ci[p]]);
}

}  // namespace

constexpr int BT = 256;

void launch_validate(int64_t n, int64_t nnz, const int32_t *rp, const int32_t *ci, const int32_t *lab, int *err,
                     hipStream_t s) {
    const int64_t g = nblocks(n, kReduceBT);
    if (n > 0) k_validate<<<(unsigned)(g < kReduceBlocks ? g : kReduceBlocks), kReduceBT, 0, s>>>(n, nnz, rp, ci, lab, err);
}
void launch_csell_count(int64_t ncell, int bs, const int32_t *rp, int32_t *rowlen, hipStream_t s) {
    int64_t n = ncell * bs;
    if (n > 0) k_rowlen<<<nblocks(n, BT), BT, 0, s>>>(n, rp, rowlen);
}
void launch_csell_width(int64_t nslice, int bs, int64_t ncell, const int32_t *rowlen, int32_t *width,
                        hipStream_t s) {
    if (nslice > 0) k_csell_width<<<nblocks(nslice * bs, BT), BT, 0, s>>>(nslice, bs, ncell, rowlen, width);
}
void launch_csell_fill(int64_t ncell, int bs, const int32_t *rp, const int32_t *ci, const double *v,
                       const int32_t *off, const int32_t *width, int32_t *col, double *val, hipStream_t s) {
    if (ncell > 0) k_csell_fill<<<nblocks(ncell * bs, BT), BT, 0, s>>>(ncell, bs, rp, ci, v, off, width, col, val);
}
void launch_csell_pack16(int64_t nslot, const int32_t *col, int32_t *sb, uint16_t *co, int *bad, hipStream_t s) {
    if (nslot > 0) k_csell_pack16<<<nblocks(nslot * kWave, BT), BT, 0, s>>>(nslot, col, sb, co, bad);
}
void launch_block_inverse(int64_t ncell, int bs, const int32_t *rp, const int32_t *ci, const double *v, double *binv,
                          int *err, hipStream_t s) {
    if (ncell > 0) k_block_inverse<<<nblocks(ncell, BT), BT, 0, s>>>(ncell, bs, rp, ci, v, binv, err);
}
void launch_level_flags(int64_t n, const int32_t *lab, int l, int32_t *isF, int32_t *isC, hipStream_t s) {
    if (n > 0) k_level_flags<<<nblocks(n, BT), BT, 0, s>>>(n, lab, l, isF, isC);
}
void launch_level_maps(int64_t n, const int32_t *lab, int l, const int32_t *fpos, const int32_t *cpos, int32_t *fmap,
                       int32_t *cmap, int32_t *flist, int32_t *clist, hipStream_t s) {
    if (n > 0) k_level_maps<<<nblocks(n, BT), BT, 0, s>>>(n, lab, l, fpos, cpos, fmap, cmap, flist, clist);
}
void launch_fdiag_inverse(int64_t nF, const int32_t *flist, const int32_t *rp, const int32_t *ci, const double *v,
                          double *dinv, int *err, int *offdiag_flag, const int32_t *fmap, hipStream_t s) {
    if (nF > 0) {
        const unsigned g = nblocks(nF, kReduceBT);
        k_fdiag_inverse<<<g < kReduceBlocks ? g : kReduceBlocks, kReduceBT, 0, s>>>(nF, flist, rp, ci, v, dinv, err,
                                                                                    offdiag_flag, fmap);
    }
}
// lanes per row of the row selections, from the mean row length of the matrix
int select_lanes(int64_t nrows, int64_t nnz) {
    const double avg = nrows > 0 ? (double)nnz / (double)nrows : 0.0;
    return avg < 6.0 ? 4 : avg < 12.0 ? 8 : avg < 24.0 ? 16 : 32;
}
#define MGR_SEL(KERNEL, FILL, LANES, N, ...)                                                        \
    do {                                                                                           \
        switch (LANES) {                                                                           \
        case 4: KERNEL<4, FILL><<<nblocks(N, 256 / 4), 256, 0, s>>>(__VA_ARGS__); break;          \
        case 8: KERNEL<8, FILL><<<nblocks(N, 256 / 8), 256, 0, s>>>(__VA_ARGS__); break;          \
        case 16: KERNEL<16, FILL><<<nblocks(N, 256 / 16), 256, 0, s>>>(__VA_ARGS__); break;       \
        default: KERNEL<32, FILL><<<nblocks(N, 256 / 32), 256, 0, s>>>(__VA_ARGS__); break;       \
        }                                                                                          \
    } while (0)
void launch_p_count(int lanes, int64_t n, const int32_t *rp, const int32_t *ci, const int32_t *cmap, int rp_type,
                    int32_t *cnt, hipStream_t s) {
    if (n > 0)
        MGR_SEL(k_p_sel, false, lanes, n, n, rp, ci, nullptr, cmap, nullptr, nullptr, rp_type, nullptr, cnt, nullptr,
                nullptr);
}
void launch_p_fill(int lanes, int64_t n, const int32_t *rp, const int32_t *ci, const double *v, const int32_t *cmap,
                   const int32_t *fmap, const double *dinv, int rp_type, const int32_t *Prp, int32_t *Pci, double *Pv,
                   hipStream_t s) {
    if (n > 0)
        MGR_SEL(k_p_sel, true, lanes, n, n, rp, ci, v, cmap, fmap, dinv, rp_type, Prp, nullptr, Pci, Pv);
}
void launch_r_count(int64_t nC, const int32_t *clist, const int32_t *rp, const int32_t *ci, const int32_t *fmap,
                    int rp_type, int32_t *cnt, hipStream_t s) {
    if (nC > 0) k_r_count<<<nblocks(nC, BT), BT, 0, s>>>(nC, clist, rp, ci, fmap, rp_type, cnt);
}
void launch_r_fill(int64_t nC, const int32_t *clist, const int32_t *rp, const int32_t *ci, const double *v,
                   const int32_t *fmap, const double *dinv, int rp_type, const int32_t *Rrp, int32_t *Rci,
                   double *Rv, hipStream_t s) {
    if (nC > 0)
        k_r_fill<<<nblocks(nC, BT), BT, 0, s>>>(nC, clist, rp, ci, v, fmap, dinv, rp_type, Rrp, Rci, Rv);
}
void launch_gather_i32(int64_t n, const int32_t *idx, const int32_t *src, int32_t *dst, hipStream_t s) {
    if (n > 0) k_gather_i32<<<nblocks(n, BT), BT, 0, s>>>(n, idx, src, dst);
}
void launch_ff_count(int lanes, int64_t nF, const int32_t *flist, const int32_t *rp, const int32_t *ci,
                     const int32_t *fmap, int32_t *cnt, hipStream_t s) {
    if (nF > 0) MGR_SEL(k_ff_sel, false, lanes, nF, nF, flist, rp, ci, nullptr, fmap, nullptr, cnt, nullptr, nullptr);
}
void launch_ff_fill(int lanes, int64_t nF, const int32_t *flist, const int32_t *rp, const int32_t *ci, const double *v,
                    const int32_t *fmap, const int32_t *Frp, int32_t *Fci, double *Fv, hipStream_t s) {
    if (nF > 0) MGR_SEL(k_ff_sel, true, lanes, nF, nF, flist, rp, ci, v, fmap, Frp, nullptr, Fci, Fv);
}
void launch_fcol_count(int lanes, int64_t n, const int32_t *rp, const int32_t *ci, const int32_t *fmap, int32_t *cnt,
                       hipStream_t s) {
    if (n > 0) MGR_SEL(k_fcol_sel, false, lanes, n, n, rp, ci, nullptr, fmap, nullptr, cnt, nullptr, nullptr, 0);
}
void launch_fcol_fill(int lanes, int64_t n, const int32_t *rp, const int32_t *ci, const double *v, const int32_t *fmap,
                      const int32_t *Frp, int32_t *Fci, double *Fv, bool fnum, hipStream_t s) {
    if (n > 0) MGR_SEL(k_fcol_sel, true, lanes, n, n, rp, ci, v, fmap, Frp, nullptr, Fci, Fv, fnum ? 1 : 0);
}
#undef MGR_SEL
int spgemm_max_row() { return kWave * kSpgChunks; }
void launch_row_len_stats(int64_t m, const int32_t *list, const int32_t *rp, int *sum, int *mx, hipStream_t s) {
    if (m <= 0) return;
    const unsigned g0 = nblocks(m, kLenStatBT);
    const unsigned g = g0 < (unsigned)kLenStatBlocks ? g0 : (unsigned)kLenStatBlocks;
    k_row_len_stats<<<g, kLenStatBT, 0, s>>>(m, list, rp, sum, mx);
}
template <bool FILL, int G, int NCH>
static void spgemm_g(int64_t m, const int32_t *Arp, const int32_t *Aci, const double *Av, const int32_t *Brp,
                     const int32_t *Bci, const double *Bv, int32_t *c, int32_t *Cci, double *Cv, int *err,
                     hipStream_t s) {
    k_spgemm<FILL, G, NCH><<<nblocks(m, BT / G), BT, 0, s>>>(m, Arp, Aci, Av, Brp, Bci, Bv, c, Cci, Cv, err);
}
template <int G>
static void spgemm_fill_g(int nch, int64_t m, const int32_t *Arp, const int32_t *Aci, const double *Av,
                          const int32_t *Brp, const int32_t *Bci, const double *Bv, int32_t *c, int32_t *Cci,
                          double *Cv, int *err, hipStream_t s) {
    switch (nch) {
    case 1: spgemm_g<true, G, 1>(m, Arp, Aci, Av, Brp, Bci, Bv, c, Cci, Cv, err, s); break;
    case 2: spgemm_g<true, G, 2>(m, Arp, Aci, Av, Brp, Bci, Bv, c, Cci, Cv, err, s); break;
    case 4: spgemm_g<true, G, 4>(m, Arp, Aci, Av, Brp, Bci, Bv, c, Cci, Cv, err, s); break;
    default: spgemm_g<true, G, kSpgChunks>(m, Arp, Aci, Av, Brp, Bci, Bv, c, Cci, Cv, err, s); break;
    }
}
void launch_spgemm(int pass, int group, int nch, int64_t m, const int32_t *Arp, const int32_t *Aci, const double *Av,
                   const int32_t *Brp, const int32_t *Bci, const double *Bv, int32_t *cnt_or_Crp, int32_t *Cci,
                   double *Cv, int *err, hipStream_t s) {
    if (m <= 0) return;
#define MGR_SPG(G)                                                                                                \
    do {                                                                                                          \
        if (pass == 0) spgemm_g<false, G, kSpgChunks>(m, Arp, Aci, Av, Brp, Bci, Bv, cnt_or_Crp, Cci, Cv, err, s); \
        else spgemm_fill_g<G>(nch, m, Arp, Aci, Av, Brp, Bci, Bv, cnt_or_Crp, Cci, Cv, err, s);                    \
    } while (0)
    switch (group) {
    case 4: MGR_SPG(4); break;
    case 8: MGR_SPG(8); break;
    case 16: MGR_SPG(16); break;
    case 32: MGR_SPG(32); break;
    default: MGR_SPG(64); break;
    }
#undef MGR_SPG
}
void launch_transpose_count(int64_t nrows, const int32_t *rp, const int32_t *ci, int32_t *cnt, hipStream_t s) {
    if (nrows > 0) k_transpose_count<<<nblocks(nrows, BT), BT, 0, s>>>(nrows, rp, ci, cnt);
}
void launch_transpose_fill(int64_t nrows, const int32_t *rp, const int32_t *ci, const double *v, int32_t *next,
                           int32_t *Tci, double *Tv, hipStream_t s) {
    if (nrows > 0) k_transpose_fill<<<nblocks(nrows, BT), BT, 0, s>>>(nrows, rp, ci, v, next, Tci, Tv);
}
void launch_transpose_sort(int64_t ncols, const int32_t *Trp, int32_t *Tci, double *Tv, hipStream_t s) {
    if (ncols > 0) k_transpose_sort_grp<<<nblocks(ncols, 256 / kSortLanes), 256, 0, s>>>(ncols, Trp, Tci, Tv);
}
template <int G>
static void strength_g(int pass, int64_t n, const int32_t *rp, const int32_t *ci, const double *v, double theta,
                       int32_t *cnt_or_Srp, int32_t *Sci, uint8_t *sflag, hipStream_t s) {
    const unsigned g = nblocks(n, BT / G);
    if (pass == 0) k_strength<false, G><<<g, BT, 0, s>>>(n, rp, ci, v, theta, cnt_or_Srp, Sci, sflag);
    else k_strength<true, G><<<g, BT, 0, s>>>(n, rp, ci, v, theta, cnt_or_Srp, Sci, sflag);
}
void launch_strength(int pass, int64_t n, int64_t nnz, const int32_t *rp, const int32_t *ci, const double *v,
                     double theta, int32_t *cnt_or_Srp, int32_t *Sci, uint8_t *sflag, hipStream_t s) {
    if (n <= 0) return;
    const double avg = (double)nnz / (double)n;
    if (avg < 12) strength_g<8>(pass, n, rp, ci, v, theta, cnt_or_Srp, Sci, sflag, s);
    else if (avg < 32) strength_g<16>(pass, n, rp, ci, v, theta, cnt_or_Srp, Sci, sflag, s);
    else strength_g<32>(pass, n, rp, ci, v, theta, cnt_or_Srp, Sci, sflag, s);
}
void launch_pmis_init(int64_t n, const int32_t *STrp, int32_t *state, hipStream_t s) {
    if (n > 0) k_pmis_init<<<nblocks(n, BT), BT, 0, s>>>(n, STrp, state);
}
void launch_pmis_select(int64_t n, const int32_t *Srp, const int32_t *Sci, const int32_t *STrp, const int32_t *STci,
                        const int32_t *state, uint64_t seed, int32_t *newc, hipStream_t s) {
    if (n > 0) k_pmis_select<<<nblocks(n, BT), BT, 0, s>>>(n, Srp, Sci, STrp, STci, state, seed, newc);
}
void launch_pmis_update(int64_t n, const int32_t *Srp, const int32_t *Sci, const int32_t *newc, int32_t *state,
                        int *counters, hipStream_t s) {
    const int64_t g = nblocks(n, kReduceBT);
    if (n > 0)
        k_pmis_update<<<(unsigned)(g < kReduceBlocks ? g : kReduceBlocks), kReduceBT, 0, s>>>(n, Srp, Sci, newc, state,
                                                                                             counters);
}
void launch_cf_flags(int64_t n, const int32_t *state, int32_t *isC, hipStream_t s) {
    if (n > 0) k_cf_flags<<<nblocks(n, BT), BT, 0, s>>>(n, state, isC);
}
void launch_interp_count(int64_t n, const int32_t *rp, const int32_t *ci, const uint8_t *sflag, const int32_t *cf,
                         int32_t *cnt, hipStream_t s) {
    if (n > 0) k_interp_count<<<nblocks(n, BT), BT, 0, s>>>(n, rp, ci, sflag, cf, cnt);
}
void launch_interp_fill(int64_t n, int64_t nnz, const int32_t *rp, const int32_t *ci, const double *v,
                        const uint8_t *sflag, const int32_t *cf, const int32_t *cmap, const int32_t *Prp, int32_t *Pci,
                        double *Pv, hipStream_t s) {
    if (n <= 0) return;
    // the group follows the mean row length: 8 lanes below 12 entries (the F
    // blocks of the MGR levels), 16 below 28 (the coarse grid: 32 lanes took
    // 3.3 against 3.1 ms there), 32 above (its first AMG levels: 1.74 against
    // 1.94 ms on the first)
    if (nnz < 12 * n)
        k_interp_fill_grp<8, kInterpSmallC, 0><<<nblocks(n, 256 / 8), 256, 0, s>>>(n, rp, ci, v, sflag, cf, cmap,
                                                                                   Prp, Pci, Pv);
    else if (nnz < 28 * n)
        k_interp_fill_grp<16, kInterpSmallC, 0><<<nblocks(n, 256 / 16), 256, 0, s>>>(n, rp, ci, v, sflag, cf, cmap,
                                                                                     Prp, Pci, Pv);
    else
        k_interp_fill_grp<32, kInterpSmallC, 0><<<nblocks(n, 256 / 32), 256, 0, s>>>(n, rp, ci, v, sflag, cf, cmap,
                                                                                     Prp, Pci, Pv);
    k_interp_fill_grp<kWave, kInterpMaxC, kInterpSmallC><<<nblocks(n, 256 / kWave), 256, 0, s>>>(
        n, rp, ci, v, sflag, cf, cmap, Prp, Pci, Pv);
    k_interp_fill<<<nblocks(n, BT), BT, 0, s>>>(n, rp, ci, v, sflag, cf, cmap, Prp, Pci, Pv);
}
void launch_l1(int64_t n, const int32_t *rp, const double *v, double *l1, int *err, hipStream_t s) {
    if (n > 0) k_l1<<<nblocks(n, BT), BT, 0, s>>>(n, rp, v, l1, err);
}
void launch_dense_lu(int64_t n, const int32_t *rp, const int32_t *ci, const double *v, double *lu, int32_t *perm,
                     int *err, hipStream_t s) {
    if (n > 0) k_dense_lu<<<1, kLuBT, 0, s>>>(n, rp, ci, v, lu, perm, err);
}
void launch_pattern_outer(int64_t n, const int32_t *rp, const int32_t *ci, const double *lam, const double *x,
                          double *d, hipStream_t s) {
    if (n > 0) k_pattern_outer<<<nblocks(n, BT), BT, 0, s>>>(n, rp, ci, lam, x, d);
}

}  // namespace mgr
