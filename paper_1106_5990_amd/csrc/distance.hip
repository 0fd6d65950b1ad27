// distance.hip -- per-edge algebraic distance (Sec. 4.1, eq:measure) and the
// strength graph built from it (Sec. 4.2, eq:strength_graph).
//
// One row group per row i: the target t_i (x_i, or x_i - (A x)_i / a_ii) is
// held in registers; for each stored entry (i, j) the group gathers x_j and
// computes, with two butterfly reductions over K,
//     p = <t, x_j>_w / <x_j, x_j>_w,   mu = sum_k w_k (t_k - p x_jk)^2,
// the residual pass re-using the register-resident x_j.  In FP32 an edge
// whose mu falls below 1e-4 * <t, t>_w (where the FP32 residual loses too
// many digits) is recomputed in FP64 from the same FP32 values.  The strength
// mask needs the row minimum of mu, known only after the row: the lane that
// stored mu_ij re-reads its own store (program order) in a second pass.
//
// For the plain target and panel rows of at most 128 bytes the default
// launch is edge-parallel instead (one lane per stored entry, whole rows of
// x_i and x_j in registers, contiguous mu stores, LDS row minima); a
// positive lanes-per-row choice selects the row-group form above.
#include <math.h>

#include <type_traits>

#include "device.h"
#include "internal.h"
#include "rowops.h"

namespace ad {

template <typename T, int K, int LPR, bool WEIGHTED, int UN>
__global__ __launch_bounds__(kBlock) void algdist_kernel(
    int n, const int* __restrict__ rp, const int* __restrict__ ci, const int* __restrict__ rpt,
    const int* __restrict__ cit, const T* __restrict__ av,
    const T* __restrict__ X, const double* __restrict__ w, int target, T* __restrict__ mu,
    double* __restrict__ pout, double theta, const uint8_t* __restrict__ fmask,
    uint8_t* __restrict__ strong, int* __restrict__ nstrong, int iter, int xcd,
    unsigned* status) {
    using S = Shape<T, K, LPR>;
    constexpr int V = S::V;
    const int lane = threadIdx.x & (kWave - 1);
    const int g = lane / LPR, l = lane % LPR;
    const int wv = threadIdx.x / kWave;
    const int64_t rows_per_tile = (int64_t)S::RPB * iter;
    const int64_t ntiles = (n + rows_per_tile - 1) / rows_per_tile;
    const int64_t tile = map_tile(ntiles, xcd);
    if (tile < 0 || tile >= ntiles) return;

    double wd[V];
    T wt[V];
#pragma unroll
    for (int q = 0; q < V; ++q) {
        wd[q] = w ? w[l * V + q] : 1.0;
        wt[q] = (T)wd[q];
    }
    const bool plain = target == AD_TARGET_PLAIN;

    for (int it = 0; it < iter; ++it) {
        const int64_t iw = tile * rows_per_tile + (int64_t)it * S::RPB + wv * S::RPW;
        if (iw >= n) break;  // whole wavefront
        const int64_t i64 = iw + g;
        const bool ghost = i64 >= n;
        if (ghost && CoopGather<T, V, LPR>::G == 1) break;  // ghosts only serve group loads
        algdist_row<S, T, K, WEIGHTED, UN>(ghost ? n - 1 : (int)i64, ghost, l, rp, ci, rpt, cit, av, X, wd,
                                           wt, plain, mu, pout, theta, fmask, strong, nstrong,
                                           status);
    }
}

template <typename T, int K, int LPR>
static void algdist_go(const ad_csr* A, const ad_csr* At, const void* X, const double* w, int target, void* mu,
                       double* p, double theta, const uint8_t* fmask, uint8_t* strong,
                       int32_t* nstrong, unsigned* st, const LaunchCfg& cfg, hipStream_t s) {
    using S = Shape<T, K, LPR>;
    const int64_t rpt = (int64_t)S::RPB * cfg.iter;
    const int64_t ntiles = (A->n + rpt - 1) / rpt;
    const int grid = grid_for_tiles(ntiles, cfg.xcd_map);
    dist_unroll<T, K, LPR>(nnz_bucket(A->nnz, A->n) >= 2, [&](auto uc) {
        constexpr int UN = decltype(uc)::value;
        if (w)
            algdist_kernel<T, K, LPR, true, UN><<<dim3(grid), dim3(kBlock), 0, s>>>(
                A->n, A->row_ptr, A->col, At->row_ptr, At->col, (const T*)At->val, (const T*)X, w,
                target, (T*)mu, p,
                theta, fmask, strong, nstrong, cfg.iter, cfg.xcd_map, st);
        else
            algdist_kernel<T, K, LPR, false, UN><<<dim3(grid), dim3(kBlock), 0, s>>>(
                A->n, A->row_ptr, A->col, At->row_ptr, At->col, (const T*)At->val, (const T*)X, w,
                target, (T*)mu, p,
                theta, fmask, strong, nstrong, cfg.iter, cfg.xcd_map, st);
    });
}

// Edge-parallel form (plain target): a workgroup takes kEdgeRows rows per
// wavefront; see algdist_edge_rows.
template <typename T, int K, bool WEIGHTED, bool LEAN>
__global__ __launch_bounds__(kBlock) void algdist_edge_kernel(
    int n, const int* __restrict__ rp, const int* __restrict__ ci, const T* __restrict__ X,
    const double* __restrict__ w, T* __restrict__ mu, double* __restrict__ pout, double theta,
    const uint8_t* __restrict__ fmask, uint8_t* __restrict__ strong, int* __restrict__ nstrong,
    int xcd, unsigned* status) {
    __shared__ EdgeLds<T> lds;
    const int64_t rows_per_tile = (int64_t)kEdgeRows * kWavesPerBlock;
    const int64_t ntiles = (n + rows_per_tile - 1) / rows_per_tile;
    const int64_t tile = map_tile(ntiles, xcd);
    if (tile < 0 || tile >= ntiles) return;  // whole workgroup
    const int64_t r0 = tile * rows_per_tile + (int64_t)(threadIdx.x / kWave) * kEdgeRows;
    const int rl = r0 < n ? (int)min<int64_t>(kEdgeRows, n - r0) : 0;
    algdist_edge_rows<T, K, WEIGHTED, LEAN>((int)r0, rl, rp, ci, X, w, mu, pout, theta, fmask,
                                            strong, nstrong, lds, status);
}

template <typename T, int K>
static void algdist_edge_go(const ad_csr* A, const void* X, const double* w, void* mu, double* p,
                            double theta, const uint8_t* fmask, uint8_t* strong, int32_t* nstrong,
                            unsigned* st, const LaunchCfg& cfg, hipStream_t s) {
    const int64_t rpt = (int64_t)kEdgeRows * kWavesPerBlock;
    const int64_t ntiles = (A->n + rpt - 1) / rpt;
    const int grid = grid_for_tiles(ntiles, cfg.xcd_map);
    auto go = [&](auto weighted, auto lean) {
        algdist_edge_kernel<T, K, decltype(weighted)::value, decltype(lean)::value>
            <<<dim3(grid), dim3(kBlock), 0, s>>>(A->n, A->row_ptr, A->col, (const T*)X, w, (T*)mu,
                                                 p, theta, fmask, strong, nstrong, cfg.xcd_map, st);
    };
    using Y = std::true_type;
    using N = std::false_type;
    const bool lean = !fmask && !p;
    if (w)
        lean ? go(Y(), Y()) : go(Y(), N());
    else
        lean ? go(N(), Y()) : go(N(), N());
}

template <typename T>
static int algdist_edge_dispatch(int K, const ad_csr* A, const void* X, const double* w, void* mu,
                                 double* p, double theta, const uint8_t* fmask, uint8_t* strong,
                                 int32_t* nstrong, unsigned* st, const LaunchCfg& cfg,
                                 hipStream_t s) {
    return with_k<T>(K, [&](auto kc) {
        constexpr int KK = decltype(kc)::value;
        if constexpr (KK * (int)sizeof(T) <= kEdgeMaxRowBytes) {
            algdist_edge_go<T, KK>(A, X, w, mu, p, theta, fmask, strong, nstrong, st, cfg, s);
            return AD_OK;
        } else {
            return AD_EINVAL;
        }
    });
}

bool algdist_uses_edge(int dtype, int K, int target, const LaunchCfg& cfg) {
    return cfg.lpr <= 0 && target == AD_TARGET_PLAIN &&
           K * (dtype == AD_F32 ? 4 : 8) <= kEdgeMaxRowBytes;
}

template <typename T>
static int algdist_dispatch(int K, const ad_csr* A, const ad_csr* At, const void* X, const double* w, int target,
                            void* mu, double* p, double theta, const uint8_t* fmask,
                            uint8_t* strong, int32_t* nstrong, unsigned* st, const LaunchCfg& cfg,
                            hipStream_t s) {
    return with_k<T>(K, [&](auto kc) {
        constexpr int KK = decltype(kc)::value;
        return with_lpr<T, KK>(cfg.lpr, [&](auto lc) {
            constexpr int L = decltype(lc)::value;
            algdist_go<T, KK, L>(A, At, X, w, target, mu, p, theta, fmask, strong, nstrong, st, cfg, s);
        });
    });
}

int launch_algdist(int dtype, int K, const ad_csr* A, const void* X, const double* w, int target,
                   void* mu, double* p, double theta, const uint8_t* fmask, uint8_t* strong,
                   int32_t* nstrong, unsigned* status, const LaunchCfg& cfg, hipStream_t s,
                   const ad_csr* At) {
    if (A->n == 0) return AD_OK;
    if (!At) At = A;
    if (algdist_uses_edge(dtype, K, target, cfg)) {
        const int rc = (dtype == AD_F32)
                           ? algdist_edge_dispatch<float>(K, A, X, w, mu, p, theta, fmask, strong,
                                                          nstrong, status, cfg, s)
                           : algdist_edge_dispatch<double>(K, A, X, w, mu, p, theta, fmask, strong,
                                                           nstrong, status, cfg, s);
        if (rc) return rc;
        AD_HIP(hipGetLastError());
        return AD_OK;
    }
    const int rc =
        (dtype == AD_F32)
            ? algdist_dispatch<float>(K, A, At, X, w, target, mu, p, theta, fmask, strong, nstrong,
                                      status, cfg, s)
            : algdist_dispatch<double>(K, A, At, X, w, target, mu, p, theta, fmask, strong, nstrong,
                                       status, cfg, s);
    if (rc) return rc;
    AD_HIP(hipGetLastError());
    return AD_OK;
}

// ---------------------------------------------------------------- strength graph
// One 8-lane group per row: row minimum of mu over F-neighbours j != i, then
// the division-free test m_i > theta mu_ij (zero-distance edges when m_i = 0).
constexpr int kStrLanes = 8;

template <typename T>
__global__ __launch_bounds__(kBlock) void strength_kernel(int n, const int* __restrict__ rp,
                                                          const int* __restrict__ ci,
                                                          const T* __restrict__ mu, double theta,
                                                          const uint8_t* __restrict__ fmask,
                                                          uint8_t* __restrict__ strong,
                                                          int* __restrict__ nstrong) {
    const int l = threadIdx.x % kStrLanes;
    const int64_t i64 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kStrLanes;
    if (i64 >= n) return;  // whole groups exit together
    const int i = (int)i64;
    const int e0 = rp[i], e1 = rp[i + 1];
    const bool in_f = fmask ? (fmask[i] != 0) : true;
    T m = (T)INFINITY;
    for (int e = e0 + l; e < e1; e += kStrLanes) {
        const int j = ci[e];
        if (in_f && j != i && (!fmask || fmask[j])) m = (mu[e] < m) ? mu[e] : m;
    }
    m = group_min<kStrLanes>(m);
    const double md = (double)m;
    int cnt = 0;
    for (int e = e0 + l; e < e1; e += kStrLanes) {
        const int j = ci[e];
        int s = 0;
        if (in_f && j != i && (!fmask || fmask[j])) {
            const double me = (double)mu[e];
            s = (md > 0.0) ? (theta * me < md) : (me == 0.0);
        }
        strong[e] = (uint8_t)s;
        cnt += s;
    }
    cnt = group_sum<kStrLanes>(cnt);
    if (l == 0 && nstrong) nstrong[i] = cnt;
}

int launch_strength(int dtype, const ad_csr* A, const void* mu, double theta,
                    const uint8_t* fmask, uint8_t* strong, int32_t* nstrong, hipStream_t s) {
    if (A->n == 0) return AD_OK;
    const int64_t blocks = ((int64_t)A->n * kStrLanes + kBlock - 1) / kBlock;
    if (dtype == AD_F32)
        strength_kernel<float><<<dim3((unsigned)blocks), dim3(kBlock), 0, s>>>(
            A->n, A->row_ptr, A->col, (const float*)mu, theta, fmask, strong, nstrong);
    else
        strength_kernel<double><<<dim3((unsigned)blocks), dim3(kBlock), 0, s>>>(
            A->n, A->row_ptr, A->col, (const double*)mu, theta, fmask, strong, nstrong);
    AD_HIP(hipGetLastError());
    return AD_OK;
}

// ---------------------------------------------------------------- CSR check
// One thread per row.  Reads only inside row_ptr[0..n] and, for rows whose
// bounds are sane (0 <= rp[i] <= rp[i+1] <= nnz), inside col[].
__global__ __launch_bounds__(kBlock) void csr_validate_kernel(int n, int64_t nnz,
                                                              const int* __restrict__ rp,
                                                              const int* __restrict__ ci,
                                                              unsigned* status) {
    const int64_t i64 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i64 > n) return;
    const int i = (int)i64;
    if (i == n) {
        if (rp[n] != nnz || rp[0] != 0) flag(status, AD_STAT_CSR_ROWPTR);
        return;
    }
    const int b = rp[i], e = rp[i + 1];
    if (b < 0 || e < b || e > nnz) {
        flag(status, AD_STAT_CSR_ROWPTR);
        return;
    }
    bool diag = false, cols_ok = true;
    int prev = -1;
    for (int q = b; q < e; ++q) {
        const int j = ci[q];
        if (j < 0 || j >= n || j <= prev) cols_ok = false;
        diag |= (j == i);
        prev = j;
    }
    if (!cols_ok) flag(status, AD_STAT_CSR_COLS);
    if (!diag) flag(status, AD_STAT_CSR_NODIAG);
}

int launch_csr_validate(const ad_csr* A, unsigned* status, hipStream_t s) {
    const int64_t blocks = ((int64_t)A->n + 1 + kBlock - 1) / kBlock;
    csr_validate_kernel<<<dim3((unsigned)blocks), dim3(kBlock), 0, s>>>(A->n, A->nnz, A->row_ptr,
                                                                        A->col, status);
    AD_HIP(hipGetLastError());
    return AD_OK;
}

}  // namespace ad
