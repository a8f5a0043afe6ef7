// Krylov kernels of restarted GMRES: fused multi-dot and multi-AXPY passes over
// the Arnoldi basis (classical Gram-Schmidt with a DGKS re-orthogonalisation
// pass when the norm drops below 1/sqrt(2) of its value before the pass), the
// Givens update of the Hessenberg column and the small triangular solve.
// Reductions are two-stage (fixed grid of per-block partials, then one block
// summing the partials in order), so results do not depend on scheduling.
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

// part[b*(nv+1) + i] = sum over this block's elements of w*V_i (i < nv), and w*w at i = nv
template <int NV>
__global__ void __launch_bounds__(BT) k_mdot(int64_t n, int nv, const double *__restrict__ V,
                                             const double *__restrict__ w, double *__restrict__ part,
                                             const int *guard) {
    if (guard && *guard == 0) return;
    __shared__ double sh[BT / kWave];
    double acc[NV + 1];
#pragma unroll
    for (int i = 0; i <= NV; ++i) acc[i] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * BT;
    for (int64_t q = (int64_t)blockIdx.x * BT + threadIdx.x; q < n; q += stride) {
        const double wq = w[q];
#pragma unroll
        for (int i = 0; i < NV; ++i)
            if (i < nv) acc[i] = acc[i] + wq * V[(int64_t)i * n + q];
        acc[NV] = acc[NV] + wq * wq;
    }
    // fully unrolled so that acc stays in registers; the condition is uniform over the block
#pragma unroll
    for (int i = 0; i <= NV; ++i) {
        if (i < nv || i == NV) {
            double s = block_sum(acc[i], sh);
            if (threadIdx.x == 0) part[(int64_t)blockIdx.x * (nv + 1) + (i == NV ? nv : i)] = s;
        }
    }
}

// w -= sum_i h[i] V_i ; part[b] = partial of <w, w> after the update
template <int NV>
__global__ void __launch_bounds__(BT) k_maxpy_norm(int64_t n, int nv, const double *__restrict__ V,
                                                   const double *__restrict__ h, double *__restrict__ w,
                                                   double *__restrict__ part, const int *guard) {
    if (guard && *guard == 0) return;
    __shared__ double sh[BT / kWave];
    double hh[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) hh[i] = i < nv ? h[i] : 0.0;
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * BT;
    for (int64_t q = (int64_t)blockIdx.x * BT + threadIdx.x; q < n; q += stride) {
        double wq = w[q];
#pragma unroll
        for (int i = 0; i < NV; ++i)
            if (i < nv) wq = wq - hh[i] * V[(int64_t)i * n + q];
        w[q] = wq;
        acc = acc + wq * wq;
    }
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

template <int NV>
__global__ void __launch_bounds__(BT) k_zaxpy(int64_t n, int nv, const double *__restrict__ Z,
                                              const double *__restrict__ y, double *__restrict__ x) {
    double yy[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) yy[i] = i < nv ? y[i] : 0.0;
    const int64_t stride = (int64_t)gridDim.x * BT;
    for (int64_t q = (int64_t)blockIdx.x * BT + threadIdx.x; q < n; q += stride) {
        double s = x[q];
#pragma unroll
        for (int i = 0; i < NV; ++i)
            if (i < nv) s = s + yy[i] * Z[(int64_t)i * n + q];
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
// stage 1: WN = <w,w> after the update; guard = 1 if WN < WN0 / 2 (DGKS test)
// stage 2: second pass (only when guard): H(:,j) += h_i, hcur = h_i
// stage 3: WN = <w,w> after the second update
// One block per reduced value (blockIdx.x = i); each sums its nblk partials with a
// fixed thread/tree order, so the result does not depend on scheduling.
__global__ void __launch_bounds__(BT) k_arnoldi_fin(int stage, int j, int m, int nblk, const double *__restrict__ part,
                                                    double *__restrict__ dsc, int *guard) {
    if ((stage == 2 || stage == 3) && *guard == 0) return;
    __shared__ double sh[BT / kWave];
    const int t = threadIdx.x;
    const int i = blockIdx.x;
    if (stage == 0 || stage == 2) {
        const int nv = j + 1;
        double s = 0.0;
        for (int b = t; b < nblk; b += BT) s += part[(int64_t)b * (nv + 1) + i];
        s = block_sum(s, sh);
        if (t == 0) {
            if (i < nv) {
                if (stage == 0) dsc[Dsc::H(i, j, m)] = s;
                else dsc[Dsc::H(i, j, m)] += s;
                dsc[Dsc::hcur(i, m)] = s;
            } else if (stage == 0) {
                dsc[Dsc::WN0] = s;
            }
        }
    } else {
        double s = 0.0;
        for (int b = t; b < nblk; b += BT) s += part[b];
        s = block_sum(s, sh);
        if (t == 0) {
            dsc[Dsc::WN] = s;
            if (stage == 1) *guard = (s < 0.5 * dsc[Dsc::WN0]) ? 1 : 0;
        }
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

}  // namespace

static unsigned red_grid(int64_t n) {
    int64_t g = (n + BT - 1) / BT;
    if (g > kRedBlocks) g = kRedBlocks;
    return (unsigned)(g > 0 ? g : 1);
}

void launch_mdot(int64_t n, int nv, const double *V, const double *w, double *part, const int *guard,
                 hipStream_t s) {
    unsigned g = red_grid(n);
    if (nv <= 4) k_mdot<4><<<g, BT, 0, s>>>(n, nv, V, w, part, guard);
    else if (nv <= 8) k_mdot<8><<<g, BT, 0, s>>>(n, nv, V, w, part, guard);
    else if (nv <= 16) k_mdot<16><<<g, BT, 0, s>>>(n, nv, V, w, part, guard);
    else if (nv <= 32) k_mdot<32><<<g, BT, 0, s>>>(n, nv, V, w, part, guard);
    else k_mdot<kMaxV><<<g, BT, 0, s>>>(n, nv, V, w, part, guard);
}

void launch_maxpy_norm(int64_t n, int nv, const double *V, const double *h, double *w, double *part,
                       const int *guard, hipStream_t s) {
    unsigned g = red_grid(n);
    if (nv <= 4) k_maxpy_norm<4><<<g, BT, 0, s>>>(n, nv, V, h, w, part, guard);
    else if (nv <= 8) k_maxpy_norm<8><<<g, BT, 0, s>>>(n, nv, V, h, w, part, guard);
    else if (nv <= 16) k_maxpy_norm<16><<<g, BT, 0, s>>>(n, nv, V, h, w, part, guard);
    else if (nv <= 32) k_maxpy_norm<32><<<g, BT, 0, s>>>(n, nv, V, h, w, part, guard);
    else k_maxpy_norm<kMaxV><<<g, BT, 0, s>>>(n, nv, V, h, w, part, guard);
}

void launch_zaxpy(int64_t n, int nv, const double *Z, const double *y, double *x, hipStream_t s) {
    if (nv <= 0) return;
    unsigned g = red_grid(n);
    if (nv <= 4) k_zaxpy<4><<<g, BT, 0, s>>>(n, nv, Z, y, x);
    else if (nv <= 8) k_zaxpy<8><<<g, BT, 0, s>>>(n, nv, Z, y, x);
    else if (nv <= 16) k_zaxpy<16><<<g, BT, 0, s>>>(n, nv, Z, y, x);
    else if (nv <= 32) k_zaxpy<32><<<g, BT, 0, s>>>(n, nv, Z, y, x);
    else k_zaxpy<kMaxV><<<g, BT, 0, s>>>(n, nv, Z, y, x);
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
    const unsigned g = (stage == 0 || stage == 2) ? (unsigned)(j + 2) : 1u;
    k_arnoldi_fin<<<g, BT, 0, s>>>(stage, j, m, nblk, part, dsc, guard);
}

void launch_givens(int j, int m, double *dsc, hipStream_t s) { k_givens<<<1, 64, 0, s>>>(j, m, dsc); }

void launch_trisolve(int k, int m, double *dsc, hipStream_t s) { k_trisolve<<<1, 64, 0, s>>>(k, m, dsc); }

void launch_norm_fin(int nblk, const double *part, double *out, hipStream_t s) {
    k_norm_fin<<<1, BT, 0, s>>>(nblk, part, out);
}

int red_blocks(int64_t n) { return (int)red_grid(n); }

}  // namespace mgr
