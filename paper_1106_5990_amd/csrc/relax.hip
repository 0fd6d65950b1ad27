// relax.hip -- test-vector start and relaxation of A x = 0 over a K-wide
// panel (Sec. 3: test vectors are relaxed solutions of the homogeneous
// system from distinct starts; Sec. 5.2 relaxes them by Gauss-Seidel).
//
// Both relaxations are a CSR row-block SpMM: each row group (LPR lanes, one
// 16-byte fragment per lane) walks its row's nonzeros, gathers the
// neighbour's panel row and accumulates a_ij x_j in the panel type.  The
// matrix is streamed once per sweep; neighbour panel rows are re-read
// through L2 (the tile mapping keeps a row range on one XCD).
#include "device.h"
#include "internal.h"
#include "rowops.h"

namespace ad {

// ---------------------------------------------------------------- start
template <typename T>
__global__ __launch_bounds__(kBlock) void tv_init_kernel(int64_t total, int64_t c0, uint64_t seed,
                                                         T* __restrict__ X) {
    constexpr int E = 16 / sizeof(T);
    const int64_t base = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * E;
    if (base >= total) return;
    Frag<T, E> f;
#pragma unroll
    for (int q = 0; q < E; ++q)
        f.v[q] = (T)uniform_pm1(splitmix64_at(seed, (uint64_t)(c0 + base + q)));
    if (base + E <= total) {
        store_frag<T, E>(X + base, f);
    } else {
        for (int q = 0; q < E && base + q < total; ++q) X[base + q] = f.v[q];
    }
}

int launch_tv_init(int dtype, int64_t row0, int64_t nrows, int K, uint64_t seed, void* X,
                   hipStream_t s) {
    const int64_t total = nrows * K;
    if (total == 0) return AD_OK;
    const int E = dtype == AD_F32 ? 4 : 2;
    const int64_t threads = (total + E - 1) / E;
    const int64_t blocks = (threads + kBlock - 1) / kBlock;
    if (dtype == AD_F32)
        tv_init_kernel<float><<<dim3((unsigned)blocks), dim3(kBlock), 0, s>>>(total, row0 * K, seed,
                                                                              (float*)X);
    else
        tv_init_kernel<double><<<dim3((unsigned)blocks), dim3(kBlock), 0, s>>>(total, row0 * K, seed,
                                                                               (double*)X);
    AD_HIP(hipGetLastError());
    return AD_OK;
}

// ---------------------------------------------------------------- Jacobi
// x_new = x - omega * (A x) / a_ii  (row held fixed if a_ii == 0)
template <typename T, int K, int LPR>
__global__ __launch_bounds__(kBlock) void jacobi_kernel(int n, const int* __restrict__ rp,
                                                        const int* __restrict__ ci,
                                                        const T* __restrict__ av,
                                                        const T* __restrict__ Xin,
                                                        T* __restrict__ Xout, T omega, int iter,
                                                        int xcd, unsigned* status) {
    using S = Shape<T, K, LPR>;
    const int lane = threadIdx.x & (kWave - 1);
    const int g = lane / LPR, l = lane % LPR;
    const int wv = threadIdx.x / kWave;
    const int64_t rows_per_tile = (int64_t)S::RPB * iter;
    const int64_t ntiles = (n + rows_per_tile - 1) / rows_per_tile;
    const int64_t tile = xcd ? xcd_tile(ntiles) : (int64_t)blockIdx.x;
    if (tile < 0 || tile >= ntiles) return;
    for (int it = 0; it < iter; ++it) {
        const int64_t i64 = tile * rows_per_tile + (int64_t)it * S::RPB + wv * S::RPW + g;
        if (i64 >= n) break;
        jacobi_row<S, T, K>((int)i64, l, rp, ci, av, Xin, Xout, omega, status);
    }
}

template <typename T, int K, int LPR>
static void jacobi_go(const ad_csr* A, const void* Xin, void* Xout, double omega, unsigned* st,
                      const LaunchCfg& cfg, hipStream_t s) {
    using S = Shape<T, K, LPR>;
    const int64_t rpt = (int64_t)S::RPB * cfg.iter;
    const int64_t ntiles = (A->n + rpt - 1) / rpt;
    const int grid = cfg.xcd_map ? grid_for_tiles(ntiles) : (int)ntiles;
    jacobi_kernel<T, K, LPR><<<dim3(grid), dim3(kBlock), 0, s>>>(
        A->n, A->row_ptr, A->col, (const T*)A->val, (const T*)Xin, (T*)Xout, (T)omega, cfg.iter,
        cfg.xcd_map, st);
}

template <typename T>
static int jacobi_dispatch(int K, const ad_csr* A, const void* Xin, void* Xout, double omega,
                           unsigned* st, const LaunchCfg& cfg, hipStream_t s) {
    return with_k<T>(K, [&](auto kc) {
        constexpr int KK = decltype(kc)::value;
        return with_lpr<T, KK>(cfg.lpr, [&](auto lc) {
            constexpr int L = decltype(lc)::value;
            jacobi_go<T, KK, L>(A, Xin, Xout, omega, st, cfg, s);
        });
    });
}

int launch_jacobi(int dtype, int K, const ad_csr* A, const void* Xin, void* Xout, double omega,
                  unsigned* status, const LaunchCfg& cfg, hipStream_t s) {
    if (A->n == 0) return AD_OK;
    const int rc = (dtype == AD_F32) ? jacobi_dispatch<float>(K, A, Xin, Xout, omega, status, cfg, s)
                                     : jacobi_dispatch<double>(K, A, Xin, Xout, omega, status, cfg, s);
    if (rc) return rc;
    AD_HIP(hipGetLastError());
    return AD_OK;
}

// ---------------------------------------------------------------- colour partition
// Stable partition of the rows by colour: rows of colour 0 first (in index
// order), then colour 1, ..., then rows with an invalid colour.  Three
// launches: per-block class counts, one exclusive scan of the class-major
// count table, per-block scatter with wave ballots for stable ranks.
constexpr int kPartRows = 1024;  // rows per partition block (4 per thread)
constexpr int kMaxColors = 64;

int color_partition_blocks(int n) { return (n + kPartRows - 1) / kPartRows; }

__device__ __forceinline__ int color_class(int c, int nc) {
    return ((unsigned)c < (unsigned)nc) ? c : nc;
}

__global__ __launch_bounds__(kBlock) void color_count_kernel(int n, const int* __restrict__ color,
                                                             int nc, int* __restrict__ counts,
                                                             int nblocks) {
    __shared__ int cnt[kMaxColors + 1];
    for (int q = threadIdx.x; q <= nc; q += kBlock) cnt[q] = 0;
    __syncthreads();
    const int base = blockIdx.x * kPartRows;
    for (int k = 0; k < kPartRows / kBlock; ++k) {
        const int r = base + k * kBlock + threadIdx.x;
        if (r < n) atomicAdd(&cnt[color_class(color[r], nc)], 1);
    }
    __syncthreads();
    for (int q = threadIdx.x; q <= nc; q += kBlock) counts[(size_t)q * nblocks + blockIdx.x] = cnt[q];
}

// Exclusive scan of counts[0 .. m) in place (single workgroup of 1024
// threads), plus seg[q] = scanned value at q * nblocks, seg[nc + 1] = n.
__global__ __launch_bounds__(1024) void scan_counts_kernel(int* __restrict__ counts, int m,
                                                           int nblocks, int nc, int n,
                                                           int* __restrict__ seg) {
    __shared__ int part[1024];
    const int t = threadIdx.x;
    const int chunk = (m + 1023) / 1024;
    const int b = t * chunk, e = min(m, b + chunk);
    int s = 0;
    for (int q = b; q < e; ++q) s += counts[q];
    part[t] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan over the 1024 chunk sums
    for (int o = 1; o < 1024; o <<= 1) {
        int v = (t >= o) ? part[t - o] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = (t > 0) ? part[t - 1] : 0;
    for (int q = b; q < e; ++q) {
        int c = counts[q];
        counts[q] = run;
        run += c;
    }
    __syncthreads();
    for (int q = t; q <= nc; q += 1024) seg[q] = counts[(size_t)q * nblocks];
    if (t == 0) seg[nc + 1] = n;
}

__global__ __launch_bounds__(kBlock) void color_scatter_kernel(int n, const int* __restrict__ color,
                                                               int nc,
                                                               const int* __restrict__ offsets,
                                                               int nblocks,
                                                               int* __restrict__ rowlist,
                                                               unsigned* status) {
    __shared__ int base[kMaxColors + 1];
    __shared__ int wcnt[kWavesPerBlock][kMaxColors + 1];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int q = threadIdx.x; q <= nc; q += kBlock) base[q] = offsets[(size_t)q * nblocks + blockIdx.x];
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    bool bad = false;
    for (int k = 0; k < kPartRows / kBlock; ++k) {
        const int r = blockIdx.x * kPartRows + k * kBlock + threadIdx.x;
        const bool valid = r < n;
        const int c = valid ? color_class(color[r], nc) : -1;
        bad |= (valid && c == nc);
        int rank = 0;
        for (int q = 0; q <= nc; ++q) {
            const uint64_t m = __ballot(c == q);
            if (lane == 0) wcnt[wv][q] = __popcll(m);
            if (c == q) rank = __popcll(m & lt);
        }
        __syncthreads();
        if (valid) {
            int pos = base[c] + rank;
            for (int w = 0; w < wv; ++w) pos += wcnt[w][c];
            rowlist[pos] = r;
        }
        __syncthreads();
        for (int q = threadIdx.x; q <= nc; q += kBlock) {
            int add = 0;
            for (int w = 0; w < kWavesPerBlock; ++w) add += wcnt[w][q];
            base[q] += add;
        }
        __syncthreads();
    }
    if (bad) flag(status, AD_STAT_BAD_COLOR);
}

int launch_color_partition(int n, const int32_t* color, int ncolors, int32_t* rowlist,
                           int32_t* seg, int32_t* counts, int nblocks, unsigned* status,
                           hipStream_t s) {
    if (n == 0) {
        AD_HIP(hipMemsetAsync(seg, 0, sizeof(int32_t) * (ncolors + 2), s));
        return AD_OK;
    }
    color_count_kernel<<<dim3(nblocks), dim3(kBlock), 0, s>>>(n, color, ncolors, counts, nblocks);
    scan_counts_kernel<<<dim3(1), dim3(1024), 0, s>>>(counts, (ncolors + 1) * nblocks, nblocks,
                                                      ncolors, n, seg);
    color_scatter_kernel<<<dim3(nblocks), dim3(kBlock), 0, s>>>(n, color, ncolors, counts,
                                                                nblocks, rowlist, status);
    AD_HIP(hipGetLastError());
    return AD_OK;
}

// ---------------------------------------------------------------- colour-major layout
// The colour phases run on panels stored colour-major: permuted row p holds
// natural row rowlist[p], so the rows of one colour are contiguous and every
// cache line a phase touches holds rows it needs.  A neighbour's permuted
// index jp is read from colp[e] = inv[col[e]]; "smaller colour" is jp <
// seg[c] because the segments are in colour order.

__global__ __launch_bounds__(kBlock) void inverse_perm_kernel(int n, const int* __restrict__ rowlist,
                                                              int* __restrict__ inv) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p < n) inv[rowlist[p]] = (int)p;
}

__global__ __launch_bounds__(kBlock) void permute_cols_kernel(int64_t nnz, const int* __restrict__ ci,
                                                              const int* __restrict__ inv,
                                                              int* __restrict__ colp) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e < nnz) colp[e] = inv[ci[e]];
}

// Xp[p] = hash start of natural row rowlist[p] (or X0[rowlist[p]] if given)
template <typename T>
__global__ __launch_bounds__(kBlock) void start_perm_kernel(int n, int K, const int* __restrict__ rowlist,
                                                            uint64_t seed, const T* __restrict__ X0,
                                                            T* __restrict__ Xp) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= (int64_t)n * K) return;
    const int64_t p = c / K;
    const int k = (int)(c - p * K);
    const int64_t i = rowlist[p];
    Xp[c] = X0 ? X0[i * K + k] : (T)uniform_pm1(splitmix64_at(seed, (uint64_t)(i * K + k)));
}

// X[rowlist[p]] = Xp[p]
template <typename T>
__global__ __launch_bounds__(kBlock) void unpermute_kernel(int n, int K, const int* __restrict__ rowlist,
                                                           const T* __restrict__ Xp, T* __restrict__ X) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= (int64_t)n * K) return;
    const int64_t p = c / K;
    const int k = (int)(c - p * K);
    X[(int64_t)rowlist[p] * K + k] = Xp[c];
}

// One colour phase in the permuted layout.  Rows p in [seg[c], seg[c+1]):
//   x_new = x - (A z) / a_ii,  z_jp = Xnew_p[jp] if jp < seg[c] else Xold_p[jp].
// Xnew_p receives the row when write_perm; Xnat (if not null) receives it at
// its natural position (the last sweep writes the caller's output directly).
// The phase of colour 0 also carries the held rows (invalid colour).
template <typename T, int K, int LPR>
__global__ __launch_bounds__(kBlock) void gs_phase_perm_kernel(
    const int* __restrict__ rp, const int* __restrict__ colp, const T* __restrict__ av, int c,
    int nc, const int* __restrict__ rowlist, const int* __restrict__ seg,
    const T* __restrict__ Xold, T* __restrict__ Xnew, T* __restrict__ Xnat, int write_perm,
    int iter, int xcd, unsigned* status) {
    using S = Shape<T, K, LPR>;
    constexpr int V = S::V, C = S::C;
    const int lane = threadIdx.x & (kWave - 1);
    const int g = lane / LPR, l = lane % LPR;
    const int wv = threadIdx.x / kWave;
    const int b0 = seg[c], b1 = seg[c + 1];
    const int64_t rows_per_tile = (int64_t)S::RPB * iter;
    const int64_t ntiles = (b1 - b0 + rows_per_tile - 1) / rows_per_tile;
    const int64_t tile = xcd ? xcd_tile(ntiles) : (int64_t)blockIdx.x;
    if (tile >= 0 && tile < ntiles) {
        for (int it = 0; it < iter; ++it) {
            const int64_t p = b0 + tile * rows_per_tile + (int64_t)it * S::RPB + wv * S::RPW + g;
            if (p >= b1) break;
            const int i = rowlist[p];
            T y[V], d;
            Frag<T, V> xi;
            row_spmm<S, T, K>((int)p, rp[i], rp[i + 1], colp, av, l,
                              [&](int jp) { return (jp < b0) ? (const T*)Xnew : Xold; }, y, d, xi);
            Frag<T, V> out;
            if (d == T(0)) {
                out = load_lane<T, V, C>(Xold + (size_t)p * K + l * V);
                if (l == 0) flag(status, AD_STAT_ZERO_DIAG);
            } else {
#pragma unroll
                for (int q = 0; q < V; ++q) out.v[q] = xi.v[q] - y[q] / d;
            }
            if (write_perm) store_lane<T, V, C>(Xnew + (size_t)p * K + l * V, out);
            if (Xnat) store_lane<T, V, C>(Xnat + (size_t)i * K + l * V, out);
        }
    }
    if (c == 0) {  // rows with an invalid colour are held fixed
        const int q0 = seg[nc], q1 = seg[nc + 1];
        const int64_t stride = (int64_t)gridDim.x * S::RPB;
        for (int64_t p = q0 + (int64_t)blockIdx.x * S::RPB + wv * S::RPW + g; p < q1; p += stride) {
            const Frag<T, V> v = load_lane<T, V, C>(Xold + (size_t)p * K + l * V);
            store_lane<T, V, C>(Xnew + (size_t)p * K + l * V, v);
            if (Xnat) store_lane<T, V, C>(Xnat + (size_t)rowlist[p] * K + l * V, v);
        }
    }
}

template <typename T, int K, int LPR>
static void gsp_go(const ad_csr* A, const int32_t* colp, int c, int nc, const int32_t* rowlist,
                   const int32_t* seg, const void* Xold, void* Xnew, void* Xnat, int write_perm,
                   unsigned* st, const LaunchCfg& cfg, hipStream_t s) {
    using S = Shape<T, K, LPR>;
    const int64_t rpt = (int64_t)S::RPB * cfg.iter;
    const int64_t ntiles = (A->n + rpt - 1) / rpt;
    const int grid = cfg.xcd_map ? grid_for_tiles(ntiles) : (int)ntiles;
    gs_phase_perm_kernel<T, K, LPR><<<dim3(grid), dim3(kBlock), 0, s>>>(
        A->row_ptr, colp, (const T*)A->val, c, nc, rowlist, seg, (const T*)Xold, (T*)Xnew,
        (T*)Xnat, write_perm, cfg.iter, cfg.xcd_map, st);
}

template <typename T>
static int gsp_dispatch(int K, const ad_csr* A, const int32_t* colp, int c, int nc,
                        const int32_t* rowlist, const int32_t* seg, const void* Xold, void* Xnew,
                        void* Xnat, int write_perm, unsigned* st, const LaunchCfg& cfg,
                        hipStream_t s) {
    return with_k<T>(K, [&](auto kc) {
        constexpr int KK = decltype(kc)::value;
        return with_lpr<T, KK>(cfg.lpr, [&](auto lc) {
            constexpr int L = decltype(lc)::value;
            gsp_go<T, KK, L>(A, colp, c, nc, rowlist, seg, Xold, Xnew, Xnat, write_perm, st, cfg, s);
        });
    });
}

int launch_gs_phase_perm(int dtype, int K, const ad_csr* A, const int32_t* colp, int c,
                         int ncolors, const int32_t* rowlist, const int32_t* seg, const void* Xold,
                         void* Xnew, void* Xnat, int write_perm, unsigned* status,
                         const LaunchCfg& cfg, hipStream_t s) {
    if (A->n == 0) return AD_OK;
    const int rc = (dtype == AD_F32)
                       ? gsp_dispatch<float>(K, A, colp, c, ncolors, rowlist, seg, Xold, Xnew, Xnat,
                                             write_perm, status, cfg, s)
                       : gsp_dispatch<double>(K, A, colp, c, ncolors, rowlist, seg, Xold, Xnew, Xnat,
                                              write_perm, status, cfg, s);
    if (rc) return rc;
    AD_HIP(hipGetLastError());
    return AD_OK;
}

int launch_perm_setup(int n, int64_t nnz, const int32_t* col, const int32_t* rowlist, int32_t* inv,
                      int32_t* colp, hipStream_t s) {
    inverse_perm_kernel<<<dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s>>>(n, rowlist, inv);
    if (nnz > 0)
        permute_cols_kernel<<<dim3((unsigned)((nnz + kBlock - 1) / kBlock)), dim3(kBlock), 0, s>>>(
            nnz, col, inv, colp);
    AD_HIP(hipGetLastError());
    return AD_OK;
}

int launch_start_perm(int dtype, int n, int K, const int32_t* rowlist, uint64_t seed,
                      const void* X0, void* Xp, hipStream_t s) {
    const int64_t m = (int64_t)n * K;
    const unsigned b = (unsigned)((m + kBlock - 1) / kBlock);
    if (dtype == AD_F32)
        start_perm_kernel<float><<<dim3(b), dim3(kBlock), 0, s>>>(n, K, rowlist, seed, (const float*)X0, (float*)Xp);
    else
        start_perm_kernel<double><<<dim3(b), dim3(kBlock), 0, s>>>(n, K, rowlist, seed, (const double*)X0, (double*)Xp);
    AD_HIP(hipGetLastError());
    return AD_OK;
}

int launch_unpermute(int dtype, int n, int K, const int32_t* rowlist, const void* Xp, void* X,
                     hipStream_t s) {
    const int64_t m = (int64_t)n * K;
    const unsigned b = (unsigned)((m + kBlock - 1) / kBlock);
    if (dtype == AD_F32)
        unpermute_kernel<float><<<dim3(b), dim3(kBlock), 0, s>>>(n, K, rowlist, (const float*)Xp, (float*)X);
    else
        unpermute_kernel<double><<<dim3(b), dim3(kBlock), 0, s>>>(n, K, rowlist, (const double*)Xp, (double*)X);
    AD_HIP(hipGetLastError());
    return AD_OK;
}

}  // namespace ad
