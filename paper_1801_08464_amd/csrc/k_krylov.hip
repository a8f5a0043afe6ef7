// Krylov kernels of restarted GMRES: fused multi-dot and multi-AXPY passes over
// the Arnoldi basis, the Givens update of the Hessenberg column and the small
// triangular solve.  Restart lengths up to 32 use classical Gram-Schmidt twice
// with the second pass lagged by one step (two reads of the basis per step);
// longer ones classical Gram-Schmidt with a DGKS re-orthogonalisation pass when
// the norm drops below 1/sqrt(2) of its value before the pass.
// Reductions are two-stage (fixed grid of per-block partials, then one block
// summing the partials in order), so results do not depend on scheduling.
#include <stdexcept>

#include "mgr_impl.h"

namespace mgr {
namespace {

constexpr int BT = 256;
constexpr int kMaxV = 64;  // restart length limit (basis vectors per pass)

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// sum over the block of one value per thread; result valid in thread 0
__device__ inline double block_sum(double v, double *sh) {
    v = wave_sum(v);
    const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
    __syncthreads();
    if (l == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < BT / kWave; ++k) r += sh[k];
    return r;
}

// Basis-width template parameter: EXACT kernels are instantiated for nv == NV, so
// their unrolled loops carry no per-vector branch and the loads of all basis
// vectors are issued back to back (a branch per vector makes the compiler wait
// for each load before the next).  The NV = 64 kernels serve wider bases with a
// runtime guard.
template <int NV, bool EXACT>
__device__ inline bool has(int i, int nv) {
    return EXACT || i < nv;
}

// Per-block partials of NV+1 running sums (entry NV holds <w, w>): wavefront
// sums, then one synchronisation and a fixed-order sum over the 4 wavefronts.
template <int NV, bool EXACT>
__device__ inline void write_partials(const double (&acc)[NV + 1], int nv, double (*sh)[NV + 1], double *part) {
    const int wv = threadIdx.x / kWave, l = threadIdx.x % kWave;
#pragma unroll
    for (int i = 0; i <= NV; ++i) {
        if (has<NV, EXACT>(i, nv) || i == NV) {  // uniform over the block
            const double v = wave_sum(acc[i]);
            if (l == 0) sh[wv][i] = v;
        }
    }
    __syncthreads();
    const int t = threadIdx.x;
    if (EXACT) nv = NV;
    if (t <= nv) {
        const int i = t == nv ? NV : t;
        double s = sh[0][i];
#pragma unroll
        for (int k = 1; k < BT / kWave; ++k) s = s + sh[k][i];
        part[(int64_t)blockIdx.x * (nv + 1) + t] = s;
    }
}

// Basis vectors read once per pass with non-temporal loads: the 1.6 GB basis
// does not fit the caches, and streaming it past them keeps w, u_j and the
// next step's vectors cached.
typedef double ntd2 __attribute__((ext_vector_type(2)));
__device__ inline double2 ldnt(const double *base, int i, int64_t ld, int64_t q) {
    const ntd2 v = __builtin_nontemporal_load(reinterpret_cast<const ntd2 *>(base + (int64_t)i * ld) + q);
    return make_double2(v.x, v.y);
}
__device__ inline const double2 *vec2(const double *base, int i, int64_t ld) {
    return reinterpret_cast<const double2 *>(base + (int64_t)i * ld);
}

// part[b*(nv+1) + i] = sum over this block's elements of w*V_i (i < nv), and w*w at i = nv
template <int NV, bool EXACT>
__global__ void __launch_bounds__(BT) k_mdot(int64_t n2, int64_t ld, int nv, const double *__restrict__ V,
                                             const double *__restrict__ w, double *__restrict__ part) {
    __shared__ double sh[BT / kWave][NV + 1];
    double acc[NV + 1];
#pragma unroll
    for (int i = 0; i <= NV; ++i) acc[i] = 0.0;
    const double2 *w2 = reinterpret_cast<const double2 *>(w);
    const int64_t stride = (int64_t)gridDim.x * BT;
    for (int64_t q = (int64_t)blockIdx.x * BT + threadIdx.x; q < n2; q += stride) {
        const double2 wq = w2[q];
#pragma unroll
        for (int i = 0; i < NV; ++i)
            if (has<NV, EXACT>(i, nv)) {
                const double2 vq = vec2(V, i, ld)[q];
                acc[i] = acc[i] + wq.x * vq.x;
                acc[i] = acc[i] + wq.y * vq.y;
            }
        acc[NV] = acc[NV] + wq.x * wq.x;
        acc[NV] = acc[NV] + wq.y * wq.y;
    }
    write_partials<NV, EXACT>(acc, nv, sh, part);
}

// w -= sum_i h[i] V_i, then the partials of <w, V_i> and <w, w> for the updated w
// (the projection of the first Gram-Schmidt pass fused with the dot products of
// the second: V is read once for both)
template <int NV, bool EXACT>
__global__ void __launch_bounds__(BT) k_maxpy_dot(int64_t n2, int64_t ld, int nv, const double *__restrict__ V,
                                                  const double *__restrict__ h, double *__restrict__ w,
                                                  double *__restrict__ part) {
    __shared__ double sh[BT / kWave][NV + 1];
    double hh[NV], acc[NV + 1];
#pragma unroll
    for (int i = 0; i < NV; ++i) hh[i] = has<NV, EXACT>(i, nv) ? h[i] : 0.0;
#pragma unroll
    for (int i = 0; i <= NV; ++i) acc[i] = 0.0;
    double2 *w2 = reinterpret_cast<double2 *>(w);
    const int64_t stride = (int64_t)gridDim.x * BT;
    for (int64_t q = (int64_t)blockIdx.x * BT + threadIdx.x; q < n2; q += stride) {
        double2 wq = w2[q];
        double2 vq[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i)
            if (has<NV, EXACT>(i, nv)) {
                vq[i] = vec2(V, i, ld)[q];
                wq.x = wq.x - hh[i] * vq[i].x;
                wq.y = wq.y - hh[i] * vq[i].y;
            }
        w2[q] = wq;
#pragma unroll
        for (int i = 0; i < NV; ++i)
            if (has<NV, EXACT>(i, nv)) {
                acc[i] = acc[i] + wq.x * vq[i].x;
                acc[i] = acc[i] + wq.y * vq[i].y;
            }
        acc[NV] = acc[NV] + wq.x * wq.x;
        acc[NV] = acc[NV] + wq.y * wq.y;
    }
    write_partials<NV, EXACT>(acc, nv, sh, part);
}

// w -= sum_i h[i] V_i ; part[b] = partial of <w, w> after the update
template <int NV, bool EXACT>
__global__ void __launch_bounds__(BT) k_maxpy_norm(int64_t n2, int64_t ld, int nv, const double *__restrict__ V,
                                                   const double *__restrict__ h, double *__restrict__ w,
                                                   double *__restrict__ part, const int *guard) {
    if (guard && *guard == 0) return;
    __shared__ double sh[BT / kWave];
    double hh[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) hh[i] = has<NV, EXACT>(i, nv) ? h[i] : 0.0;
    double acc = 0.0;
    double2 *w2 = reinterpret_cast<double2 *>(w);
    const int64_t stride = (int64_t)gridDim.x * BT;
    for (int64_t q = (int64_t)blockIdx.x * BT + threadIdx.x; q < n2; q += stride) {
        double2 wq = w2[q];
#pragma unroll
        for (int i = 0; i < NV; ++i)
            if (has<NV, EXACT>(i, nv)) {
                const double2 vq = vec2(V, i, ld)[q];
                wq.x = wq.x - hh[i] * vq.x;
                wq.y = wq.y - hh[i] * vq.y;
            }
        w2[q] = wq;
        acc = acc + wq.x * wq.x;
        acc = acc + wq.y * wq.y;
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

template <int NV, bool EXACT>
__global__ void __launch_bounds__(BT) k_zaxpy(int64_t n, int64_t ld, int nv, const double *__restrict__ Z,
                                              const double *__restrict__ y, double *__restrict__ x) {
    double yy[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) yy[i] = has<NV, EXACT>(i, nv) ? y[i] : 0.0;
    const int64_t stride = (int64_t)gridDim.x * BT;
    for (int64_t q = (int64_t)blockIdx.x * BT + threadIdx.x; q < n; q += stride) {
        double s = x[q];
#pragma unroll
        for (int i = 0; i < NV; ++i)
            if (has<NV, EXACT>(i, nv)) s = s + yy[i] * Z[(int64_t)i * ld + q];
        x[q] = s;
    }
}

__global__ void __launch_bounds__(BT) k_norm_part(int64_t n, const double *__restrict__ a, double *__restrict__ part) {
    __shared__ double sh[BT / kWave];
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * BT;
    for (int64_t q = (int64_t)blockIdx.x * BT + threadIdx.x; q < n; q += stride) acc = acc + a[q] * a[q];
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_scale_dev(int64_t n, const double *__restrict__ a, const double *__restrict__ sc, int divide,
                            double *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double c = sc[0];
    y[i] = divide ? a[i] / c : a[i] * c;
}

__global__ void k_axpby(int64_t n, double a, const double *__restrict__ x, double b, double *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = a * x[i] + b * y[i];
}

// stage 0: h_i = sum of partials (i <= j) -> H(:,j) and hcur; WN0 = <w,w> before the update
// stage 1: after the fused update-and-dot pass: h2_i = <w, V_i>, WN = <w,w>, and
//          guard = 1 if WN < WN0 / 2 (the DGKS test: a second projection is needed)
// stage 3: only when guard: WN = <w,w> after the second update, H(:,j) += h2
// Stages 0 and 1 run one block per reduced value (blockIdx.x = i); every sum runs
// in a fixed thread/tree order, so the result does not depend on scheduling.
__global__ void __launch_bounds__(BT) k_arnoldi_fin(int stage, int j, int m, int nblk, const double *__restrict__ part,
                                                    double *__restrict__ dsc, int *guard) {
    if (stage == 3 && *guard == 0) return;
    __shared__ double sh[BT / kWave];
    const int t = threadIdx.x;
    const int i = blockIdx.x;
    const int nv = j + 1;
    if (stage == 0 || stage == 1) {
        double s = 0.0;
        for (int b = t; b < nblk; b += BT) s += part[(int64_t)b * (nv + 1) + i];
        s = block_sum(s, sh);
        if (t == 0) {
            if (stage == 0) {
                if (i < nv) {
                    dsc[Dsc::H(i, j, m)] = s;
                    dsc[Dsc::hcur(i, m)] = s;
                } else {
                    dsc[Dsc::WN0] = s;
                }
            } else {
                if (i < nv) {
                    dsc[Dsc::h2(i, m)] = s;
                } else {
                    dsc[Dsc::WN] = s;
                    *guard = (s < 0.5 * dsc[Dsc::WN0]) ? 1 : 0;
                }
            }
        }
    } else {
        double s = 0.0;
        for (int b = t; b < nblk; b += BT) s += part[b];
        s = block_sum(s, sh);
        if (t == 0) dsc[Dsc::WN] = s;
        if (t < nv) dsc[Dsc::H(t, j, m)] += dsc[Dsc::h2(t, m)];
    }
}

// apply the previous rotations to column j, build rotation j, update g
__global__ void k_givens(int j, int m, double *dsc) {
    if (threadIdx.x != 0) return;
    const double hn = sqrt(dsc[Dsc::WN]);
    for (int i = 0; i < j; ++i) {
        const double a = dsc[Dsc::H(i, j, m)], b = dsc[Dsc::H(i + 1, j, m)];
        const double c = dsc[Dsc::cs(i, m)], s = dsc[Dsc::sn(i, m)];
        dsc[Dsc::H(i, j, m)] = c * a + s * b;
        dsc[Dsc::H(i + 1, j, m)] = -s * a + c * b;
    }
    const double a = dsc[Dsc::H(j, j, m)];
    const double den = sqrt(a * a + hn * hn);
    double c = 1.0, s = 0.0;
    if (den != 0.0) {
        c = a / den;
        s = hn / den;
    }
    dsc[Dsc::cs(j, m)] = c;
    dsc[Dsc::sn(j, m)] = s;
    dsc[Dsc::H(j, j, m)] = c * a + s * hn;
    dsc[Dsc::H(j + 1, j, m)] = 0.0;
    const double gj = dsc[Dsc::g(j, m)];
    dsc[Dsc::g(j + 1, m)] = -s * gj;
    dsc[Dsc::g(j, m)] = c * gj;
    dsc[Dsc::GABS] = fabs(-s * gj);
    dsc[Dsc::HN] = hn;
}

// y = H(0:k,0:k)^{-1} g(0:k)
__global__ void k_trisolve(int k, int m, double *dsc) {
    if (threadIdx.x != 0) return;
    for (int i = k - 1; i >= 0; --i) {
        double s = dsc[Dsc::g(i, m)];
        for (int q = i + 1; q < k; ++q) s = s - dsc[Dsc::H(i, q, m)] * dsc[Dsc::y(q, m)];
        dsc[Dsc::y(i, m)] = s / dsc[Dsc::H(i, i, m)];
    }
}

__global__ void __launch_bounds__(BT) k_norm_fin(int nblk, const double *__restrict__ part, double *out) {
    __shared__ double sh[BT / kWave];
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += BT) s += part[b];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[0] = sqrt(s);
}


// ---- Arnoldi with lagged re-orthogonalisation ----
// Classical Gram-Schmidt applied twice to every basis vector, the second pass of
// vector j merged with the first pass of the operator image of vector j, so each
// step reads the basis twice instead of three times.  At step j, columns
// 0..j-1 hold the final orthonormal v_i and column j holds u_j, the previous
// step's image after one projection, with norm s_j (u_0 = v_0, s_0 = 1).  The
// preconditioner and the operator are applied to u_j itself: z_j and w = A z_j
// carry the scale s_j, which the coefficients absorb.  One pass gives
// p_i = <V_i, w> (i <= j) and q_i = <V_i, u_j> (i <= j, q_j = <u_j, u_j>); with
// a = q/s_j (i < j) and beta^2 = q_j/s_j^2 - |a|^2, v_j = (u_j/s_j - V a)/beta,
// and the projection of w/s_j on v_0..v_j has h_i = p_i/s_j (i < j),
// h_j = (p_j/s_j^2 - <a, h>)/beta.  The second pass writes v_j over u_j and the
// projected remainder u_{j+1} into column j+1 with its norm s_{j+1}.  Column
// j-1 of the Hessenberg matrix, first taken with u_j as its last basis vector,
// gains s_j a above and s_j beta below the diagonal, and its Givens rotation is
// rebuilt before column j is rotated.

template <int K>
__device__ inline void write_partials_k(const double (&acc)[K], double (*sh)[K], double *part) {
    const int wv = threadIdx.x / kWave, l = threadIdx.x % kWave;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const double v = wave_sum(acc[i]);
        if (l == 0) sh[wv][i] = v;
    }
    __syncthreads();
    const int t = threadIdx.x;
    if (t < K) {
        double s = sh[0][t];
#pragma unroll
        for (int k = 1; k < BT / kWave; ++k) s = s + sh[k][t];
        part[(int64_t)blockIdx.x * K + t] = s;
    }
}

// part[b*2NV + i] = partial of <V_i, w> (i < NV), part[b*2NV + NV + i] = partial
// of <V_i, u> with u = V_{NV-1}
template <int NV>
__global__ void __launch_bounds__(BT) k_lag_dots(int64_t n2, int64_t ld, const double *__restrict__ V,
                                                 const double *__restrict__ w, double *__restrict__ part) {
    __shared__ double sh[BT / kWave][2 * NV];
    double acc[2 * NV];
#pragma unroll
    for (int i = 0; i < 2 * NV; ++i) acc[i] = 0.0;
    const double2 *w2 = reinterpret_cast<const double2 *>(w);
    const int64_t stride = (int64_t)gridDim.x * BT;
    for (int64_t q = (int64_t)blockIdx.x * BT + threadIdx.x; q < n2; q += stride) {
        const double2 wq = w2[q];
        const double2 uq = vec2(V, NV - 1, ld)[q];
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            const double2 vi = (i == NV - 1) ? uq : ldnt(V, i, ld, q);
            acc[i] = acc[i] + wq.x * vi.x;
            acc[i] = acc[i] + wq.y * vi.y;
            acc[NV + i] = acc[NV + i] + uq.x * vi.x;
            acc[NV + i] = acc[NV + i] + uq.y * vi.y;
        }
    }
    write_partials_k<2 * NV>(acc, sh, part);
}

// Rotations 0..c-1 (final) applied to col[0..c] (the unrotated column c, its
// subdiagonal in col[c+1]), then rotation c from the diagonal and subdiagonal;
// g(c), g(c+1) from g0 = g(c) before it.  One thread, operands in LDS.
__device__ inline void rotate_lds(int c, double *col, const double *cs, const double *sn, double g0, double *out) {
    const double hn = col[c + 1];
    for (int i = 0; i < c; ++i) {
        const double a = col[i], b = col[i + 1];
        col[i] = cs[i] * a + sn[i] * b;
        col[i + 1] = -sn[i] * a + cs[i] * b;
    }
    const double a = col[c];
    const double den = sqrt(a * a + hn * hn);
    double csc = 1.0, snc = 0.0;
    if (den != 0.0) {
        csc = a / den;
        snc = hn / den;
    }
    col[c] = csc * a + snc * hn;
    col[c + 1] = 0.0;
    out[0] = csc;
    out[1] = snc;
    out[2] = csc * g0;
    out[3] = -snc * g0;
}

// Stage the unrotated column c (rows 0..c+1) and rotations 0..c-1 in LDS
// (threads in parallel), rotate it (thread 0), write the rotated column, the
// rotation and g(c), g(c+1) back (threads in parallel).  Every thread of the
// block calls it; `raw` already holds column c when `have_raw`.
__device__ inline void rotate_column(int c, int m, double *dsc, double *raw, bool have_raw, double *cs, double *sn,
                                     double *out) {
    const int t = threadIdx.x;
    if (!have_raw)
        for (int i = t; i <= c + 1; i += blockDim.x) raw[i] = dsc[Dsc::Hraw(i, c, m)];
    for (int i = t; i < c; i += blockDim.x) {
        cs[i] = dsc[Dsc::cs(i, m)];
        sn[i] = dsc[Dsc::sn(i, m)];
    }
    __syncthreads();
    if (t == 0) rotate_lds(c, raw, cs, sn, dsc[Dsc::gpre(c, m)], out);
    __syncthreads();
    for (int i = t; i <= c + 1; i += blockDim.x) dsc[Dsc::H(i, c, m)] = raw[i];
    if (t == 0) {
        dsc[Dsc::cs(c, m)] = out[0];
        dsc[Dsc::sn(c, m)] = out[1];
        dsc[Dsc::g(c, m)] = out[2];
        dsc[Dsc::g(c + 1, m)] = out[3];
    }
}

// stage 0 (2(j+1) blocks): block i sums partial i into hcur (p) / h2 (q)
// stage 1 (one thread): the coefficient algebra of step j
__global__ void __launch_bounds__(BT) k_lag_coef(int stage, int j, int m, int nblk, const double *__restrict__ part,
                                                 double *__restrict__ dsc) {
    const int nv = j + 1;
    if (stage == 0) {
        __shared__ double sh[BT / kWave];
        const int i = blockIdx.x;
        double s = 0.0;
        for (int b = threadIdx.x; b < nblk; b += BT) s += part[(int64_t)b * (2 * nv) + i];
        s = block_sum(s, sh);
        if (threadIdx.x == 0) dsc[i < nv ? Dsc::hcur(i, m) : Dsc::h2(i - nv, m)] = s;
        return;
    }
    // stage 1: operands staged in LDS by all threads, the algebra on thread 0
    __shared__ double sp[kFusedMaxV], sq[kFusedMaxV], sa[kFusedMaxV], sh[kFusedMaxV];
    __shared__ double raw[kFusedMaxV + 2], cs[kFusedMaxV], sn[kFusedMaxV], out[4];
    __shared__ double scal[4];  // beta, s_j, broke
    const int t = threadIdx.x;
    for (int i = t; i < nv; i += blockDim.x) {
        sp[i] = dsc[Dsc::hcur(i, m)];
        sq[i] = dsc[Dsc::h2(i, m)];
    }
    if (j >= 1)
        for (int i = t; i <= j; i += blockDim.x) raw[i] = dsc[Dsc::Hraw(i, j - 1, m)];
    __syncthreads();
    if (t == 0) {
        double beta = 1.0, sj = 1.0, broke = 0.0;
        if (j >= 1) {
            sj = dsc[Dsc::sc(j, m)];
            const double is = 1.0 / sj;
            double aa = 0.0;
            for (int i = 0; i < j; ++i) {
                sa[i] = sq[i] * is;
                aa = aa + sa[i] * sa[i];
            }
            const double b2 = sq[j] * is * is - aa;
            if (!(b2 > 0.0) || !isfinite(b2)) {  // u_j lies in the span of v_0..v_{j-1}
                broke = 1.0;
            } else {
                beta = sqrt(b2);
                // column j-1 was taken with u_j as its last basis vector
                for (int i = 0; i < j; ++i) raw[i] += sj * sa[i];
                raw[j] = sj * beta;
            }
        }
        scal[0] = beta;
        scal[1] = sj;
        scal[2] = broke;
    }
    __syncthreads();
    const double beta = scal[0], sj = scal[1];
    if (scal[2] != 0.0) {
        if (t == 0) dsc[Dsc::BRK] = 1.0;
        return;
    }
    if (j >= 1) {
        for (int i = t; i <= j; i += blockDim.x) dsc[Dsc::Hraw(i, j - 1, m)] = raw[i];
        rotate_column(j - 1, m, dsc, raw, true, cs, sn, out);
    }
    if (t == 0) {
        const double is = 1.0 / sj;
        double ah = 0.0;
        for (int i = 0; i < j; ++i) {
            sh[i] = sp[i] * is;
            ah = ah + sa[i] * sh[i];
        }
        sh[j] = (sp[j] * is * is - ah) / beta;
        for (int i = 0; i < j; ++i) sa[i] = sa[i] / beta;
        dsc[Dsc::ALPHA] = is / beta;
        dsc[Dsc::INVS] = is;
        dsc[Dsc::BRK] = 0.0;
        if (j == 0) dsc[Dsc::sc(0, m)] = 1.0;
    }
    __syncthreads();
    for (int i = t; i <= j; i += blockDim.x) {
        dsc[Dsc::Hraw(i, j, m)] = sh[i];
        dsc[Dsc::ch(i, m)] = sh[i];
        if (i < j) dsc[Dsc::ca(i, m)] = sa[i];
    }
}

// v_j = alpha u_j - sum_{i<j} ca_i v_i over column j; u_{j+1} = w/s_j -
// sum_{i<=j} ch_i v_i into column j+1; part[b] = partial of |u_{j+1}|^2
template <int NV>
__global__ void __launch_bounds__(BT) k_lag_update(int64_t n2, int64_t ld, const double *__restrict__ V,
                                                   double *Uj, double *__restrict__ Un,
                                                   const double *__restrict__ w, const double *__restrict__ dsc,
                                                   int m, double *__restrict__ part) {
    if (dsc[Dsc::BRK] != 0.0) return;
    __shared__ double sh[BT / kWave];
    double ca[NV > 1 ? NV - 1 : 1], ch[NV];
#pragma unroll
    for (int i = 0; i + 1 < NV; ++i) ca[i] = dsc[Dsc::ca(i, m)];
#pragma unroll
    for (int i = 0; i < NV; ++i) ch[i] = dsc[Dsc::ch(i, m)];
    const double alpha = dsc[Dsc::ALPHA], invs = dsc[Dsc::INVS];
    const double2 *w2 = reinterpret_cast<const double2 *>(w);
    double2 *u2 = reinterpret_cast<double2 *>(Uj);
    double2 *n2p = reinterpret_cast<double2 *>(Un);
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * BT;
    for (int64_t q = (int64_t)blockIdx.x * BT + threadIdx.x; q < n2; q += stride) {
        const double2 uq = u2[q], wq0 = w2[q];
        double2 vj = make_double2(uq.x * alpha, uq.y * alpha);
        double2 wq = make_double2(wq0.x * invs, wq0.y * invs);
#pragma unroll
        for (int i = 0; i + 1 < NV; ++i) {
            const double2 vi = ldnt(V, i, ld, q);
            vj.x = vj.x - ca[i] * vi.x;
            vj.y = vj.y - ca[i] * vi.y;
            wq.x = wq.x - ch[i] * vi.x;
            wq.y = wq.y - ch[i] * vi.y;
        }
        wq.x = wq.x - ch[NV - 1] * vj.x;
        wq.y = wq.y - ch[NV - 1] * vj.y;
        u2[q] = vj;
        n2p[q] = wq;
        acc = acc + wq.x * wq.x;
        acc = acc + wq.y * wq.y;
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// s_{j+1} = |u_{j+1}|; column j taken with u_{j+1} as its last basis vector
// (subdiagonal s_{j+1}) and rotated; GABS = |g(j+1)|, HN = s_{j+1}
__global__ void __launch_bounds__(BT) k_lag_givens(int j, int m, int nblk, const double *__restrict__ part,
                                                   double *__restrict__ dsc) {
    if (dsc[Dsc::BRK] != 0.0) return;
    __shared__ double sh[BT / kWave];
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += BT) s += part[b];
    s = block_sum(s, sh);
    __shared__ double raw[kFusedMaxV + 2], cs[kFusedMaxV], sn[kFusedMaxV], out[4], hn_s;
    const int t = threadIdx.x;
    for (int i = t; i <= j; i += BT) raw[i] = dsc[Dsc::Hraw(i, j, m)];
    if (t == 0) {
        const double hn = sqrt(s);
        hn_s = hn;
        raw[j + 1] = hn;
        dsc[Dsc::sc(j + 1, m)] = hn;
        dsc[Dsc::Hraw(j + 1, j, m)] = hn;
        dsc[Dsc::gpre(j, m)] = dsc[Dsc::g(j, m)];
    }
    __syncthreads();
    rotate_column(j, m, dsc, raw, true, cs, sn, out);
    if (t == 0) {
        dsc[Dsc::GABS] = fabs(out[3]);
        dsc[Dsc::HN] = hn_s;
    }
}

__global__ void k_lag_yscale(int k, int m, double *dsc) {
    const int i = threadIdx.x;
    if (i < k) dsc[Dsc::y(i, m)] /= dsc[Dsc::sc(i, m)];
}

}  // namespace

static unsigned red_grid(int64_t n) {
    int64_t g = (n + BT - 1) / BT;
    if (g > kRedBlocks) g = kRedBlocks;
    return (unsigned)(g > 0 ? g : 1);
}

int64_t krylov_ld(int64_t n) { return (n + 63) / 64 * 64; }

// nv <= kFusedMaxV: the kernel instantiated for exactly nv vectors; wider
// bases: the guarded kMaxV kernel
#define MGR_NV_CASE(KERNEL, N, ...) \
    case N: KERNEL<N, true><<<g, BT, 0, s>>>(__VA_ARGS__); break;
#define MGR_NV_DISPATCH(KERNEL, nv, ...)                                                                 \
    do {                                                                                                 \
        switch (nv) {                                                                                    \
            MGR_NV_CASE(KERNEL, 1, __VA_ARGS__) MGR_NV_CASE(KERNEL, 2, __VA_ARGS__)                      \
            MGR_NV_CASE(KERNEL, 3, __VA_ARGS__) MGR_NV_CASE(KERNEL, 4, __VA_ARGS__)                      \
            MGR_NV_CASE(KERNEL, 5, __VA_ARGS__) MGR_NV_CASE(KERNEL, 6, __VA_ARGS__)                      \
            MGR_NV_CASE(KERNEL, 7, __VA_ARGS__) MGR_NV_CASE(KERNEL, 8, __VA_ARGS__)                      \
            MGR_NV_CASE(KERNEL, 9, __VA_ARGS__) MGR_NV_CASE(KERNEL, 10, __VA_ARGS__)                     \
            MGR_NV_CASE(KERNEL, 11, __VA_ARGS__) MGR_NV_CASE(KERNEL, 12, __VA_ARGS__)                    \
            MGR_NV_CASE(KERNEL, 13, __VA_ARGS__) MGR_NV_CASE(KERNEL, 14, __VA_ARGS__)                    \
            MGR_NV_CASE(KERNEL, 15, __VA_ARGS__) MGR_NV_CASE(KERNEL, 16, __VA_ARGS__)                    \
            MGR_NV_CASE(KERNEL, 17, __VA_ARGS__) MGR_NV_CASE(KERNEL, 18, __VA_ARGS__)                    \
            MGR_NV_CASE(KERNEL, 19, __VA_ARGS__) MGR_NV_CASE(KERNEL, 20, __VA_ARGS__)                    \
            MGR_NV_CASE(KERNEL, 21, __VA_ARGS__) MGR_NV_CASE(KERNEL, 22, __VA_ARGS__)                    \
            MGR_NV_CASE(KERNEL, 23, __VA_ARGS__) MGR_NV_CASE(KERNEL, 24, __VA_ARGS__)                    \
            MGR_NV_CASE(KERNEL, 25, __VA_ARGS__) MGR_NV_CASE(KERNEL, 26, __VA_ARGS__)                    \
            MGR_NV_CASE(KERNEL, 27, __VA_ARGS__) MGR_NV_CASE(KERNEL, 28, __VA_ARGS__)                    \
            MGR_NV_CASE(KERNEL, 29, __VA_ARGS__) MGR_NV_CASE(KERNEL, 30, __VA_ARGS__)                    \
            MGR_NV_CASE(KERNEL, 31, __VA_ARGS__) MGR_NV_CASE(KERNEL, 32, __VA_ARGS__)                    \
        default: KERNEL<kMaxV, false><<<g, BT, 0, s>>>(__VA_ARGS__); break;                              \
        }                                                                                                \
    } while (0)
static_assert(kFusedMaxV == 32, "the exact-width dispatch covers 1..32 vectors");

void launch_mdot(int64_t n, int64_t ld, int nv, const double *V, const double *w, double *part, hipStream_t s) {
    const int64_t n2 = (n + 1) / 2;
    const unsigned g = red_grid(n);
    MGR_NV_DISPATCH(k_mdot, nv, n2, ld, nv, V, w, part);
}

void launch_maxpy_dot(int64_t n, int64_t ld, int nv, const double *V, const double *h, double *w, double *part,
                      hipStream_t s) {
    const int64_t n2 = (n + 1) / 2;
    const unsigned g = red_grid(n);
    if (nv <= kFusedMaxV) {
        MGR_NV_DISPATCH(k_maxpy_dot, nv, n2, ld, nv, V, h, w, part);
    } else {
        // too wide to hold the basis values in registers: update, then dot
        k_maxpy_norm<kMaxV, false><<<g, BT, 0, s>>>(n2, ld, nv, V, h, w, part, nullptr);
        k_mdot<kMaxV, false><<<g, BT, 0, s>>>(n2, ld, nv, V, w, part);
    }
}

void launch_maxpy_norm(int64_t n, int64_t ld, int nv, const double *V, const double *h, double *w, double *part,
                       const int *guard, hipStream_t s) {
    const int64_t n2 = (n + 1) / 2;
    const unsigned g = red_grid(n);
    MGR_NV_DISPATCH(k_maxpy_norm, nv, n2, ld, nv, V, h, w, part, guard);
}

void launch_zaxpy(int64_t n, int64_t ld, int nv, const double *Z, const double *y, double *x, hipStream_t s) {
    if (nv <= 0) return;
    const unsigned g = red_grid(n);
    MGR_NV_DISPATCH(k_zaxpy, nv, n, ld, nv, Z, y, x);
}
#undef MGR_NV_DISPATCH
#undef MGR_NV_CASE

#define MGR_LAG_CASE(KERNEL, N, ...) \
    case N: KERNEL<N><<<g, BT, 0, s>>>(__VA_ARGS__); break;
#define MGR_LAG_DISPATCH(KERNEL, nv, ...)                                                               \
    do {                                                                                                \
        switch (nv) {                                                                                   \
            MGR_LAG_CASE(KERNEL, 1, __VA_ARGS__) MGR_LAG_CASE(KERNEL, 2, __VA_ARGS__)                   \
            MGR_LAG_CASE(KERNEL, 3, __VA_ARGS__) MGR_LAG_CASE(KERNEL, 4, __VA_ARGS__)                   \
            MGR_LAG_CASE(KERNEL, 5, __VA_ARGS__) MGR_LAG_CASE(KERNEL, 6, __VA_ARGS__)                   \
            MGR_LAG_CASE(KERNEL, 7, __VA_ARGS__) MGR_LAG_CASE(KERNEL, 8, __VA_ARGS__)                   \
            MGR_LAG_CASE(KERNEL, 9, __VA_ARGS__) MGR_LAG_CASE(KERNEL, 10, __VA_ARGS__)                  \
            MGR_LAG_CASE(KERNEL, 11, __VA_ARGS__) MGR_LAG_CASE(KERNEL, 12, __VA_ARGS__)                 \
            MGR_LAG_CASE(KERNEL, 13, __VA_ARGS__) MGR_LAG_CASE(KERNEL, 14, __VA_ARGS__)                 \
            MGR_LAG_CASE(KERNEL, 15, __VA_ARGS__) MGR_LAG_CASE(KERNEL, 16, __VA_ARGS__)                 \
            MGR_LAG_CASE(KERNEL, 17, __VA_ARGS__) MGR_LAG_CASE(KERNEL, 18, __VA_ARGS__)                 \
            MGR_LAG_CASE(KERNEL, 19, __VA_ARGS__) MGR_LAG_CASE(KERNEL, 20, __VA_ARGS__)                 \
            MGR_LAG_CASE(KERNEL, 21, __VA_ARGS__) MGR_LAG_CASE(KERNEL, 22, __VA_ARGS__)                 \
            MGR_LAG_CASE(KERNEL, 23, __VA_ARGS__) MGR_LAG_CASE(KERNEL, 24, __VA_ARGS__)                 \
            MGR_LAG_CASE(KERNEL, 25, __VA_ARGS__) MGR_LAG_CASE(KERNEL, 26, __VA_ARGS__)                 \
            MGR_LAG_CASE(KERNEL, 27, __VA_ARGS__) MGR_LAG_CASE(KERNEL, 28, __VA_ARGS__)                 \
            MGR_LAG_CASE(KERNEL, 29, __VA_ARGS__) MGR_LAG_CASE(KERNEL, 30, __VA_ARGS__)                 \
            MGR_LAG_CASE(KERNEL, 31, __VA_ARGS__) MGR_LAG_CASE(KERNEL, 32, __VA_ARGS__)                 \
        default: throw std::runtime_error("lagged Arnoldi: basis wider than 32 vectors");               \
        }                                                                                               \
    } while (0)

void launch_lag_dots(int64_t n, int64_t ld, int nv, const double *V, const double *w, double *part, hipStream_t s) {
    const int64_t n2 = (n + 1) / 2;
    const unsigned g = red_grid(n);
    MGR_LAG_DISPATCH(k_lag_dots, nv, n2, ld, V, w, part);
}

void launch_lag_coef(int j, int m, int nblk, const double *part, double *dsc, hipStream_t s) {
    k_lag_coef<<<2 * (j + 1), BT, 0, s>>>(0, j, m, nblk, part, dsc);
    k_lag_coef<<<1, 64, 0, s>>>(1, j, m, nblk, part, dsc);
}

void launch_lag_update(int64_t n, int64_t ld, int nv, double *V, const double *w, const double *dsc, int m,
                       double *part, hipStream_t s) {
    const int64_t n2 = (n + 1) / 2;
    const unsigned g = red_grid(n);
    double *Uj = V + (int64_t)(nv - 1) * ld, *Un = V + (int64_t)nv * ld;
    MGR_LAG_DISPATCH(k_lag_update, nv, n2, ld, V, Uj, Un, w, dsc, m, part);
}
#undef MGR_LAG_DISPATCH
#undef MGR_LAG_CASE

void launch_lag_givens(int j, int m, int nblk, const double *part, double *dsc, hipStream_t s) {
    k_lag_givens<<<1, BT, 0, s>>>(j, m, nblk, part, dsc);
}

void launch_lag_yscale(int k, int m, double *dsc, hipStream_t s) {
    if (k > 0) k_lag_yscale<<<1, 64, 0, s>>>(k, m, dsc);
}

void launch_norm_part(int64_t n, const double *a, double *part, hipStream_t s) {
    k_norm_part<<<red_grid(n), BT, 0, s>>>(n, a, part);
}

void launch_scale_dev(int64_t n, const double *a, const double *scal, int divide, double *y, hipStream_t s) {
    if (n > 0) k_scale_dev<<<nblocks(n, BT), BT, 0, s>>>(n, a, scal, divide, y);
}

void launch_axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t s) {
    if (n > 0) k_axpby<<<nblocks(n, BT), BT, 0, s>>>(n, a, x, b, y);
}

void launch_arnoldi_fin(int stage, int j, int m, int nblk, const double *part, double *dsc, int *guard,
                        hipStream_t s) {
    const unsigned g = (stage == 0 || stage == 1) ? (unsigned)(j + 2) : 1u;
    k_arnoldi_fin<<<g, BT, 0, s>>>(stage, j, m, nblk, part, dsc, guard);
}

void launch_givens(int j, int m, double *dsc, hipStream_t s) { k_givens<<<1, 64, 0, s>>>(j, m, dsc); }

void launch_trisolve(int k, int m, double *dsc, hipStream_t s) { k_trisolve<<<1, 64, 0, s>>>(k, m, dsc); }

void launch_norm_fin(int nblk, const double *part, double *out, hipStream_t s) {
    k_norm_fin<<<1, BT, 0, s>>>(nblk, part, out);
}

int red_blocks(int64_t n) { return (int)red_grid(n); }

}  // namespace mgr
