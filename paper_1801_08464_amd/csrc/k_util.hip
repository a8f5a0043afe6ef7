// Utility kernels: fills, precision casts and a deterministic exclusive scan.
#include "mgr_impl.h"

namespace mgr {
namespace {

template <typename T>
__global__ void k_fill(T *p, T v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

template <typename A, typename B>
__global__ void k_cast(const A *a, B *b, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (B)a[i];
}

constexpr int kScanBT = 256, kScanIPT = 8, kScanTile = kScanBT * kScanIPT;

// inclusive scan of one value per thread over the block (Hillis-Steele in LDS)
template <int BT>
__device__ int64_t block_inclusive_scan(int64_t v, int64_t *sh) {
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < BT; off <<= 1) {
        int64_t x = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += x;
        __syncthreads();
    }
    int64_t r = sh[t];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(kScanBT) k_scan_tile_sums(const int32_t *in, int64_t n, int64_t *tsum) {
    __shared__ int64_t sh[kScanBT];
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t s = 0;
    for (int i = threadIdx.x; i < kScanTile; i += kScanBT) {
        int64_t idx = base + i;
        if (idx < n) s += in[idx];
    }
    int64_t inc = block_inclusive_scan<kScanBT>(s, sh);
    if (threadIdx.x == kScanBT - 1) tsum[blockIdx.x] = inc;
}

// exclusive scan of the nt tile sums in place (one block of 1024 threads); total -> out[n]
__global__ void __launch_bounds__(1024) k_scan_tiles(int64_t *tsum, int64_t nt, int32_t *out, int64_t n) {
    __shared__ int64_t sh[1024];
    int64_t chunk = (nt + 1023) / 1024;
    int64_t b0 = threadIdx.x * chunk, b1 = b0 + chunk < nt ? b0 + chunk : nt;
    int64_t s = 0;
    for (int64_t b = b0; b < b1; ++b) s += tsum[b];
    int64_t inc = block_inclusive_scan<1024>(s, sh);
    int64_t run = inc - s;
    for (int64_t b = b0; b < b1; ++b) {
        int64_t v = tsum[b];
        tsum[b] = run;
        run += v;
    }
    if (threadIdx.x == 1023) {
        tsum[nt] = inc;
        out[n] = (int32_t)inc;
    }
}

__global__ void __launch_bounds__(kScanBT) k_scan_final(const int32_t *in, int32_t *out, int64_t n,
                                                        const int64_t *tsum) {
    __shared__ int64_t sh[kScanBT];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanIPT;
    int32_t v[kScanIPT];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanIPT; ++k) {
        v[k] = base + k < n ? in[base + k] : 0;
        s += v[k];
    }
    int64_t inc = block_inclusive_scan<kScanBT>(s, sh);
    int64_t run = tsum[blockIdx.x] + inc - s;
#pragma unroll
    for (int k = 0; k < kScanIPT; ++k) {
        if (base + k < n) out[base + k] = (int32_t)run;
        run += v[k];
    }
}

__global__ void k_scan_empty(int32_t *out) { out[0] = 0; }

__global__ void k_iota(int32_t *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (int32_t)i;
}

}  // namespace

void launch_iota(int32_t *p, int64_t n, hipStream_t s) {
    if (n > 0) k_iota<<<nblocks(n, 256), 256, 0, s>>>(p, n);
}
void launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
    if (n > 0) k_fill<int32_t><<<nblocks(n, 256), 256, 0, s>>>(p, v, n);
}
void launch_fill_f64(double *p, double v, int64_t n, hipStream_t s) {
    if (n > 0) k_fill<double><<<nblocks(n, 256), 256, 0, s>>>(p, v, n);
}
void launch_fill_f32(float *p, float v, int64_t n, hipStream_t s) {
    if (n > 0) k_fill<float><<<nblocks(n, 256), 256, 0, s>>>(p, v, n);
}
void launch_cast_f64_f32(const double *a, float *b, int64_t n, hipStream_t s) {
    if (n > 0) k_cast<double, float><<<nblocks(n, 256), 256, 0, s>>>(a, b, n);
}
void launch_cast_f32_f64(const float *a, double *b, int64_t n, hipStream_t s) {
    if (n > 0) k_cast<float, double><<<nblocks(n, 256), 256, 0, s>>>(a, b, n);
}

int64_t scan_tmp_words(int64_t n) { return (n + kScanTile - 1) / kScanTile + 2; }

void launch_scan(const int32_t *in, int32_t *out, int64_t n, int64_t *tmp, hipStream_t s) {
    if (n <= 0) {
        k_scan_empty<<<1, 1, 0, s>>>(out);
        return;
    }
    int64_t nt = (n + kScanTile - 1) / kScanTile;
    k_scan_tile_sums<<<(unsigned)nt, kScanBT, 0, s>>>(in, n, tmp);
    k_scan_tiles<<<1, 1024, 0, s>>>(tmp, nt, out, n);
    k_scan_final<<<(unsigned)nt, kScanBT, 0, s>>>(in, out, n, tmp);
}

}  // namespace mgr
