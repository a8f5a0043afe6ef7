// The fine-level operator of the solve: SpMV / residual on the cell-sliced ELL
// copy of A_0 (the GMRES product and the level-0 residual of the V-cycle).
// Templated on the value type (double; float for the mixed-precision cycle).
#include "mgr_impl.h"

namespace mgr {
namespace {

// Fine-level SpMV on the cell-sliced ELL: one wavefront per 64-cell slice, one
// thread per cell computing all BS rows of its cell (so each cell's outputs are
// written together, without partial-line writes).  Each component's slots are
// read in chunks of kChunk: every column and value load of a chunk (each a contiguous
// wavefront segment) is issued before the dependent gathers of x; the matrix is
// streamed with non-temporal loads so that it does not evict x from the caches.
// Row sums run in ascending column order.  IX = uint16_t: the columns are 16-bit
// offsets from their slot's smallest column (sb, one word per slot, the same for
// the whole wavefront), 0xffff marking padding.
constexpr int kChunk = 16;

template <typename T, typename IX, int MODE, int BS>
__global__ void __launch_bounds__(256) k_csell(int64_t ncell, int64_t nslice, const int32_t *__restrict__ off,
                                                    const int32_t *__restrict__ width,
                                                    const IX *__restrict__ col, const int32_t *__restrict__ sb,
                                                    const T *__restrict__ val, const T *__restrict__ x,
                                                    const T *__restrict__ r, T *__restrict__ y) {
    constexpr bool kOff = sizeof(IX) == 2;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t s = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
    if (s >= nslice) return;
    const int64_t c = s * kWave + lane;
    T out[BS];
#pragma unroll
    for (int comp = 0; comp < BS; ++comp) {
        const int64_t g = s * BS + comp;
        const int64_t o = off[g];
        const int w = width[g];
        const IX *cp = col + o * kWave + lane;
        const T *vp = val + o * kWave + lane;
        T acc = 0;
        for (int t0 = 0; t0 < w; t0 += kChunk) {
            int j[kChunk];
            T a[kChunk], xv[kChunk];
            int base[kOff ? kChunk : 1];
#pragma unroll
            for (int u = 0; u < kChunk; ++u) {
                // every load of the chunk is issued before any of them is used
                if (kOff) {
                    j[u] = t0 + u < w ? (int)__builtin_nontemporal_load(cp + (int64_t)(t0 + u) * kWave) : 0xffff;
                    base[u] = t0 + u < w ? sb[o + t0 + u] : 0;
                } else {
                    j[u] = t0 + u < w ? (int)__builtin_nontemporal_load(cp + (int64_t)(t0 + u) * kWave) : -1;
                }
                a[u] = t0 + u < w ? __builtin_nontemporal_load(vp + (int64_t)(t0 + u) * kWave) : (T)0;
            }
            if (kOff) {
#pragma unroll
                for (int u = 0; u < kChunk; ++u) j[u] = j[u] == 0xffff ? -1 : base[u] + j[u];
            }
#pragma unroll
            for (int u = 0; u < kChunk; ++u) xv[u] = j[u] >= 0 ? x[j[u]] : (T)0;
#pragma unroll
            for (int u = 0; u < kChunk; ++u)
                if (j[u] >= 0) acc = acc + a[u] * xv[u];
        }
        out[comp] = acc;
    }
    if (c < ncell) {
#pragma unroll
        for (int comp = 0; comp < BS; ++comp) {
            const int64_t i = c * BS + comp;
            if (MODE == 0) y[i] = out[comp];
            else if (MODE == 1) y[i] = r[i] - out[comp];
            else y[i] = y[i] + out[comp];
        }
    }
}

}  // namespace

constexpr int BT = 256;

template <typename T>
void launch_csell(int mode, const CSell &A, const T *vals, const T *x, const T *r, T *y, hipStream_t s,
                  KEvents ev) {
    if (A.nslice <= 0) return;
    const unsigned g = nblocks(A.nslice, BT / kWave);
#define MGR_CSELL_M(IX, CI, M, BS)                                                                            \
    do {                                                                                                      \
        if (ev.start)                                                                                         \
            hipExtLaunchKernelGGL(k_csell<T, IX, M, BS>, dim3(g), dim3(BT), 0, s, ev.start, ev.stop, 0, A.ncell, \
                                  A.nslice, A.off, A.width, CI, A.sb, vals, x, r, y);                         \
        else                                                                                                  \
            k_csell<T, IX, M, BS><<<g, BT, 0, s>>>(A.ncell, A.nslice, A.off, A.width, CI, A.sb, vals, x, r, y); \
    } while (0)
#define MGR_CSELL(IX, CI, BS)                            \
    do {                                                 \
        if (mode == 0) MGR_CSELL_M(IX, CI, 0, BS);       \
        else if (mode == 1) MGR_CSELL_M(IX, CI, 1, BS);  \
        else MGR_CSELL_M(IX, CI, 2, BS);                 \
    } while (0)
    if (A.co) {
        if (A.bs == 3) MGR_CSELL(uint16_t, A.co, 3);
        else MGR_CSELL(uint16_t, A.co, 1);
    } else {
        if (A.bs == 3) MGR_CSELL(int32_t, A.col, 3);
        else MGR_CSELL(int32_t, A.col, 1);
    }
#undef MGR_CSELL
#undef MGR_CSELL_M
}

template void launch_csell<double>(int, const CSell &, const double *, const double *, const double *, double *,
                                   hipStream_t, KEvents);
template void launch_csell<float>(int, const CSell &, const float *, const float *, const float *, float *,
                                  hipStream_t, KEvents);

}  // namespace mgr
