// Kernels of the semi-smooth Newton outer loop (Section 3.1, algorithm
// "Semi-smooth Newton Method") for the complementarity system with unknowns
// (p, rho, S) per cell: residual and active set (steps 1-2), assembly of the
// generalised Jacobian (step 2), and the update u += alpha du (step 4).
//
// Residual: the PDE rows R = L u - f (row sums in ascending column order), the
// constraint row R = min(F, G) with F = S and G = rho - H p.  Active set
// A = {c : F_c >= G_c}; its constraint row is G' = [-H, 1, 0], the inactive one
// F' = [0, 0, 1].  Labels: p -> 3, rho -> 1, S -> 2 on A and 0 off A; the
// evaluation counts the cells whose labels it changed.
#include "mgr_impl.h"

namespace mgr {
namespace {

constexpr int BT = 256;

__device__ inline int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }

__global__ void k_axpy_inplace(int64_t n, double alpha, const double *__restrict__ du, double *__restrict__ u) {
    const int64_t i = gtid();
    if (i < n) u[i] = u[i] + alpha * du[i];
}

// one thread per cell: its two PDE rows, its constraint row, its three labels
__global__ void __launch_bounds__(BT) k_ncp_eval(int64_t ncell, const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ ci, const double *__restrict__ v,
                                                 const double *__restrict__ henry, const double *__restrict__ f,
                                                 const double *__restrict__ u, double *__restrict__ R,
                                                 int32_t *__restrict__ labels, int *nactive, int *nchanged) {
    const int64_t c = gtid();
    int act = 0, chg = 0;
    if (c < ncell) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int64_t row = 3 * c + q;
            double s = 0.0;
            for (int p = rp[row]; p < rp[row + 1]; ++p) s = s + v[p] * u[ci[p]];
            R[row] = s - f[row];
        }
        const double F = u[3 * c + 2];
        const double G = u[3 * c + 1] - henry[c] * u[3 * c];
        act = F >= G;
        R[3 * c + 2] = act ? G : F;
        // the cell's labels before this evaluation (the Jacobian's pattern follows them)
        chg = labels[3 * c] != 3 || labels[3 * c + 1] != 1 || labels[3 * c + 2] != (act ? 2 : 0);
        labels[3 * c] = 3;
        labels[3 * c + 1] = 1;
        labels[3 * c + 2] = act ? 2 : 0;
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        act += __shfl_xor(act, o);
        chg += __shfl_xor(chg, o);
    }
    if ((threadIdx.x & (kWave - 1)) == 0 && act) atomicAdd(nactive, act);
    if ((threadIdx.x & (kWave - 1)) == 0 && chg) atomicAdd(nchanged, chg);
}

__global__ void k_ncp_jac_count(int64_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ labels,
                                int32_t *__restrict__ cnt) {
    const int64_t row = gtid();
    if (row >= n) return;
    cnt[row] = (row % 3 != 2) ? rp[row + 1] - rp[row] : (labels[row] == 2 ? 2 : 1);
}

__global__ void k_ncp_jac_fill(int64_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                               const double *__restrict__ v, const double *__restrict__ henry,
                               const int32_t *__restrict__ labels, const int32_t *__restrict__ Jrp,
                               int32_t *__restrict__ Jci, double *__restrict__ Jv) {
    const int64_t row = gtid();
    if (row >= n) return;
    const int64_t q = Jrp[row];
    if (row % 3 != 2) {
        for (int p = rp[row]; p < rp[row + 1]; ++p) {
            Jci[q + (p - rp[row])] = ci[p];
            Jv[q + (p - rp[row])] = v[p];
        }
        return;
    }
    const int64_t c = row / 3;
    if (labels[row] == 2) {
        Jci[q] = (int32_t)(3 * c);
        Jv[q] = -henry[c];
        Jci[q + 1] = (int32_t)(3 * c + 1);
        Jv[q + 1] = 1.0;
    } else {
        Jci[q] = (int32_t)(3 * c + 2);
        Jv[q] = 1.0;
    }
}

}  // namespace

void launch_axpy_inplace(int64_t n, double alpha, const double *du, double *u, hipStream_t s) {
    if (n > 0) k_axpy_inplace<<<nblocks(n, BT), BT, 0, s>>>(n, alpha, du, u);
}
void launch_ncp_eval(int64_t ncell, const int32_t *rp, const int32_t *ci, const double *v, const double *henry,
                     const double *f, const double *u, double *R, int32_t *labels, int *nactive, int *nchanged,
                     hipStream_t s) {
    if (ncell > 0)
        k_ncp_eval<<<nblocks(ncell, BT), BT, 0, s>>>(ncell, rp, ci, v, henry, f, u, R, labels, nactive, nchanged);
}
void launch_ncp_jac_count(int64_t n, const int32_t *rp, const int32_t *labels, int32_t *cnt, hipStream_t s) {
    if (n > 0) k_ncp_jac_count<<<nblocks(n, BT), BT, 0, s>>>(n, rp, labels, cnt);
}
void launch_ncp_jac_fill(int64_t n, const int32_t *rp, const int32_t *ci, const double *v, const double *henry,
                         const int32_t *labels, const int32_t *Jrp, int32_t *Jci, double *Jv, hipStream_t s) {
    if (n > 0) k_ncp_jac_fill<<<nblocks(n, BT), BT, 0, s>>>(n, rp, ci, v, henry, labels, Jrp, Jci, Jv);
}

}  // namespace mgr
