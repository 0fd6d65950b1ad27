// util.hip -- small device utilities shared by the calls: fill kernels (used
// instead of memset nodes, so that a caller's graph capture records plain
// kernels) and an exclusive prefix sum of int32 counts into int64 offsets.
#include "device.h"
#include "internal.h"

namespace ad {

__global__ __launch_bounds__(kBlock) void fill_f64_kernel(double* __restrict__ p, int64_t m,
                                                          double v) {
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q < m) p[q] = v;
}

__global__ __launch_bounds__(kBlock) void fill_i32_kernel(int32_t* __restrict__ p, int64_t m,
                                                          int32_t v) {
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q < m) p[q] = v;
}

__global__ __launch_bounds__(kBlock) void fill_i64_kernel(int64_t* __restrict__ p, int64_t m,
                                                          int64_t v) {
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q < m) p[q] = v;
}

int launch_fill_f64(double* p, int64_t m, double v, hipStream_t s) {
    if (m <= 0) return AD_OK;
    const int64_t b = (m + kBlock - 1) / kBlock;
    fill_f64_kernel<<<dim3((unsigned)b), dim3(kBlock), 0, s>>>(p, m, v);
    AD_HIP(hipGetLastError());
    return AD_OK;
}

int launch_fill_i32(int32_t* p, int64_t m, int32_t v, hipStream_t s) {
    if (m <= 0) return AD_OK;
    const int64_t b = (m + kBlock - 1) / kBlock;
    fill_i32_kernel<<<dim3((unsigned)b), dim3(kBlock), 0, s>>>(p, m, v);
    AD_HIP(hipGetLastError());
    return AD_OK;
}

// ---------------------------------------------------------------- exclusive scan
// out[0] = 0, out[q + 1] = cnt[0] + ... + cnt[q] for q < m, in three
// launches: per-block totals of kScanTile counts, a single-workgroup scan of
// the totals, and the per-block scan with the block's offset added.
constexpr int kScanThreads = 256;
constexpr int kScanPer = 16;                          // counts per thread
constexpr int kScanTile = kScanThreads * kScanPer;    // counts per block

__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t* sh, int64_t& total) {
    // Hillis-Steele over kScanThreads values in LDS
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int o = 1; o < kScanThreads; o <<= 1) {
        const int64_t a = (t >= o) ? sh[t - o] : 0;
        __syncthreads();
        sh[t] += a;
        __syncthreads();
    }
    total = sh[kScanThreads - 1];
    const int64_t incl = sh[t];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(kScanThreads) void scan_totals_kernel(const int32_t* __restrict__ cnt,
                                                                   int64_t m,
                                                                   int64_t* __restrict__ tot) {
    __shared__ int64_t sh[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    int64_t s = 0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q)
        if (base + q < m) s += cnt[base + q];
    int64_t total;
    block_excl_scan(s, sh, total);
    if (threadIdx.x == 0) tot[blockIdx.x] = total;
}

// One workgroup: exclusive scan of nb block totals in place.
__global__ __launch_bounds__(kScanThreads) void scan_blocks_kernel(int64_t* __restrict__ tot,
                                                                   int64_t nb) {
    __shared__ int64_t sh[kScanThreads];
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kScanThreads) {
        const int64_t q = b0 + threadIdx.x;
        const int64_t v = q < nb ? tot[q] : 0;
        int64_t total;
        const int64_t ex = block_excl_scan(v, sh, total);
        if (q < nb) tot[q] = carry + ex;
        carry += total;
    }
}

__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(const int32_t* __restrict__ cnt,
                                                                  int64_t m,
                                                                  const int64_t* __restrict__ tot,
                                                                  int64_t* __restrict__ out) {
    __shared__ int64_t sh[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    int32_t c[kScanPer];
    int64_t s = 0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        c[q] = (base + q < m) ? cnt[base + q] : 0;
        s += c[q];
    }
    int64_t total;
    int64_t run = block_excl_scan(s, sh, total) + tot[blockIdx.x];
    if (blockIdx.x == 0 && threadIdx.x == 0) out[0] = 0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        run += c[q];
        if (base + q < m) out[base + q + 1] = run;
    }
}

int64_t scan_workspace_bytes(int64_t m) {
    const int64_t nb = (m + kScanTile - 1) / kScanTile;
    return (nb > 0 ? nb : 1) * (int64_t)sizeof(int64_t);
}

__global__ __launch_bounds__(kBlock) void narrow_i64_kernel(const int64_t* __restrict__ a,
                                                            int64_t m, int32_t* __restrict__ b) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < m) b[i] = (int32_t)a[i];
}

// b[0..m) = a[0..m) (values known to fit int32)
int launch_narrow_i64(const int64_t* a, int64_t m, int32_t* b, hipStream_t s) {
    if (m <= 0) return AD_OK;
    narrow_i64_kernel<<<dim3((unsigned)((m + kBlock - 1) / kBlock)), dim3(kBlock), 0, s>>>(a, m, b);
    AD_HIP(hipGetLastError());
    return AD_OK;
}

int launch_excl_scan(const int32_t* cnt, int64_t m, int64_t* out, int64_t* tmp, hipStream_t s) {
    if (m <= 0) {
        fill_i64_kernel<<<dim3(1), dim3(kBlock), 0, s>>>(out, 1, 0);
        AD_HIP(hipGetLastError());
        return AD_OK;
    }
    const int64_t nb = (m + kScanTile - 1) / kScanTile;
    scan_totals_kernel<<<dim3((unsigned)nb), dim3(kScanThreads), 0, s>>>(cnt, m, tmp);
    scan_blocks_kernel<<<dim3(1), dim3(kScanThreads), 0, s>>>(tmp, nb);
    scan_apply_kernel<<<dim3((unsigned)nb), dim3(kScanThreads), 0, s>>>(cnt, m, tmp, out);
    AD_HIP(hipGetLastError());
    return AD_OK;
}

}  // namespace ad
