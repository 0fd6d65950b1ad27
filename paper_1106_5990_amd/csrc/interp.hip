// interp.hip -- least-squares interpolation rows (Sec. 3.1, eq:LSfuncrowi /
// eq:modls) on interpolatory sets C_i picked by the one-point distances
// (the systematic scan of the final remark of Sec. 4.3).
//
// Work mapping: a group of LPR adjacent lanes per F row, each lane holding
// V = K / LPR consecutive panel entries, so that one load instruction of the
// group fetches a whole panel row (every fetched cache line fully used).
// Each wavefront owns a window of 128 consecutive rows; it writes the
// (trivial) C rows directly and compacts the window's F rows into an LDS list
// with ballots, so that every lane group then solves a real LS problem
// whatever the C/F pattern.  Per F row the group
//   * scans the row's entries (same addresses in every lane of the group)
//     and keeps the `caliber` C-neighbours of smallest mu (ties: lower
//     column) in a register-resident sorted list;
//   * gathers the target and those panel rows once into registers and forms
//     the FP64 normal equations
//         G_ab = sum_k w_k x_a^k x_b^k,  h_a = sum_k w_k x_a^k t^k
//     (a product of two FP32 values is exact in FP64), reduced over the
//     group with butterflies;
//   * factors G by Cholesky in increasing-mu column order (every lane of the
//     group, redundantly), dropping a column whose pivot is <= 1e-12 of its
//     Gram diagonal, and solves;
//   * evaluates the functional at the minimiser from its definition in FP64
//     on the register-resident values.
#include <math.h>

#include <type_traits>

#include "device.h"
#include "internal.h"
#include "lsops.h"
#include "rowops.h"

namespace ad {

constexpr int kLsRowsPerLane = 2;                   // window rows per lane
constexpr int kLsWindow = kWave * kLsRowsPerLane;   // rows per wavefront window

template <typename T, int K, int LPR, int CALT>
__device__ __forceinline__ double ls_row(int i, int l, const int* __restrict__ rp,
                                         const int* __restrict__ ci, const T* __restrict__ av,
                                         const T* __restrict__ X, const double (&wd)[K / LPR],
                                         const uint8_t* __restrict__ cf, const T* __restrict__ mu,
                                         int cal, int target, int* __restrict__ Pcol,
                                         double* __restrict__ Pval, double* __restrict__ lsv,
                                         int* __restrict__ rstat, unsigned* status) {
    using S = Shape<T, K, LPR>;
    constexpr int V = S::V, C = S::C;
    const int e0 = rp[i], e1 = rp[i + 1];
    int st = 0;

    // C_i: the cal candidates of least (mu, column), sorted; diagonal on the way
    T smu[CALT];
    int scol[CALT];
    int nsel = 0;
    double d = 0.0;
#pragma unroll
    for (int q = 0; q < CALT; ++q) {
        smu[q] = T(0);
        scol[q] = -1;
    }
    // entries are fetched SE at a time so that their loads are in flight
    // together (the scan is otherwise a chain of dependent round trips)
    constexpr int SE = 8;
    for (int eb = e0; eb < e1; eb += SE) {
        int jj[SE];
        T mm[SE];
        bool cand[SE];
#pragma unroll
        for (int u = 0; u < SE; ++u) jj[u] = (eb + u < e1) ? ci[eb + u] : -1;
#pragma unroll
        for (int u = 0; u < SE; ++u) mm[u] = (eb + u < e1) ? mu[eb + u] : T(0);
#pragma unroll
        for (int u = 0; u < SE; ++u) cand[u] = (jj[u] >= 0 && jj[u] != i) ? (cf[jj[u]] != 0) : false;
#pragma unroll
        for (int u = 0; u < SE; ++u)
            if (jj[u] == i) d = (double)av[eb + u];
#pragma unroll
        for (int u = 0; u < SE; ++u)
            if (cand[u]) ls_insert<T, CALT>(smu, scol, nsel, cal, mm[u], jj[u]);
    }

    // target in FP64: x_i, or x_i - (A x)_i / a_ii (residual form, carried
    // as the distance pass carries it, so that both give the same rows)
    double t[V];
    {
        Frag<T, V> f = load_lane<T, V, C>(X + (size_t)i * K + l * V);
#pragma unroll
        for (int q = 0; q < V; ++q) t[q] = (double)f.v[q];
    }
    if (target == AD_TARGET_RESIDUAL) {
        if (d == 0.0) {
            st = 3;
            if (l == 0) flag(status, AD_STAT_ZERO_DIAG);
        } else {
            double y[V];
#pragma unroll
            for (int q = 0; q < V; ++q) y[q] = 0.0;
            for (int e = e0; e < e1; ++e) {
                const int j = ci[e];
                const double a = (double)av[e];
                Frag<T, V> xj = load_lane<T, V, C>(X + (size_t)j * K + l * V);
#pragma unroll
                for (int q = 0; q < V; ++q) y[q] = fma(a, (double)xj.v[q], y[q]);
            }
#pragma unroll
            for (int q = 0; q < V; ++q) t[q] = carried<T>(t[q] - y[q] / d);
        }
    }
    return ls_solve<T, K, LPR, CALT>(i, l, t, wd, GlobalRows<T, K>{X}, scol, nsel, st, cal, Pcol,
                                     Pval, lsv, rstat);
}

template <typename T, int K, int LPR, int CALT>
__global__ __launch_bounds__(kBlock) void ls_interp_kernel(
    int n, const int* __restrict__ rp, const int* __restrict__ ci, const T* __restrict__ av,
    const T* __restrict__ X, const double* __restrict__ w, const uint8_t* __restrict__ cf,
    const T* __restrict__ mu, int cal, int target, int* __restrict__ Pcol,
    double* __restrict__ Pval, double* __restrict__ lsv, int* __restrict__ rstat,
    double* __restrict__ block_sums, int xcd, unsigned* status) {
    using S = Shape<T, K, LPR>;
    constexpr int V = S::V;
    __shared__ int flist[kWavesPerBlock][kLsWindow];
    __shared__ double wsum[kWavesPerBlock];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const int g = lane / LPR, l = lane % LPR;
    const int64_t nwin = (n + kLsWindow - 1) / kLsWindow;
    const int64_t ntiles = (nwin + kWavesPerBlock - 1) / kWavesPerBlock;
    const int64_t tile = map_tile(ntiles, xcd);
    const int64_t win = (tile >= 0 && tile < ntiles) ? tile * kWavesPerBlock + wv : nwin;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    // window scan: C rows written here, F rows listed
    int cnt = 0;
    if (win < nwin) {
        const int64_t w0 = win * kLsWindow;
#pragma unroll
        for (int r = 0; r < kLsRowsPerLane; ++r) {
            const int64_t row = w0 + r * kWave + lane;
            const bool valid = row < n;
            const bool isF = valid && cf[row] == 0;
            if (valid && !isF) ls_c_row(row, cal, Pcol, Pval, lsv, rstat);
            const uint64_t m = __ballot(isF);
            if (isF) flist[wv][cnt + __popcll(m & lt)] = (int)row;
            cnt += __popcll(m);
        }
    }
    __syncthreads();

    double wd[V];
#pragma unroll
    for (int q = 0; q < V; ++q) wd[q] = w ? w[l * V + q] : 1.0;
    double fsum = 0.0;
    for (int base = 0; base < cnt; base += S::RPW) {
        const int idx = base + g;
        if (idx < cnt) {
            const double v = ls_row<T, K, LPR, CALT>(flist[wv][idx], l, rp, ci, av, X, wd, cf, mu,
                                                     cal, target, Pcol, Pval, lsv, rstat, status);
            if (l == 0) fsum += v;
        }
    }
    if (block_sums) {
        // fixed-order reduction: xor butterfly in the wave, then waves in order
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) fsum += __shfl_xor(fsum, o, kWave);
        if (lane == 0) wsum[wv] = fsum;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int q = 0; q < kWavesPerBlock; ++q) s += wsum[q];
            block_sums[blockIdx.x] = s;
        }
    }
}

// Sum of m block partials by one workgroup of 1024 threads in a fixed order:
// thread t adds partials t, t + 1024, ... (coalesced loads, several in
// flight), then an xor butterfly in each wavefront and the wavefront sums
// in order.
__global__ __launch_bounds__(1024) void sum_blocks_kernel(const double* __restrict__ part, int m,
                                                          double* __restrict__ out) {
    __shared__ double wsum[1024 / kWave];
    const int t = threadIdx.x;
    double s = 0.0;
#pragma unroll 8
    for (int q = t; q < m; q += 1024) s += part[q];
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
    if ((t & (kWave - 1)) == 0) wsum[t / kWave] = s;
    __syncthreads();
    if (t == 0) {
        double tot = 0.0;
        for (int w = 0; w < 1024 / kWave; ++w) tot += wsum[w];
        *out = tot;
    }
}

int ls_interp_blocks(int dtype, int K, int n, const LaunchCfg& cfg) {
    (void)dtype;
    (void)K;
    const int64_t nwin = ((int64_t)n + kLsWindow - 1) / kLsWindow;
    const int64_t ntiles = (nwin + kWavesPerBlock - 1) / kWavesPerBlock;
    return grid_for_tiles(ntiles, cfg.xcd_map);
}

template <typename T, int K, int LPR>
static void ls_go(int caliber, const ad_csr* A, const void* X, const double* w, const uint8_t* cf,
                  const void* mu, int target, int32_t* P_col, double* P_val, double* ls_val,
                  int32_t* row_status, double* block_sums, unsigned* st, const LaunchCfg& cfg,
                  hipStream_t s) {
    const int grid = ls_interp_blocks(A->dtype, K, A->n, cfg);
    if (caliber <= 4)
        ls_interp_kernel<T, K, LPR, 4><<<dim3(grid), dim3(kBlock), 0, s>>>(
            A->n, A->row_ptr, A->col, (const T*)A->val, (const T*)X, w, cf, (const T*)mu, caliber,
            target, P_col, P_val, ls_val, row_status, block_sums, cfg.xcd_map, st);
    else
        ls_interp_kernel<T, K, LPR, 8><<<dim3(grid), dim3(kBlock), 0, s>>>(
            A->n, A->row_ptr, A->col, (const T*)A->val, (const T*)X, w, cf, (const T*)mu, caliber,
            target, P_col, P_val, ls_val, row_status, block_sums, cfg.xcd_map, st);
}

// LS rows default to 16 bytes of panel per lane (one chunk), so that all
// gathered rows stay in registers for the second pass.
template <typename T>
constexpr int ls_lpr_default(int K) {
    for (int L = 1; L <= kWave; L *= 2)
        if (lpr_ok<T>(K, L) && (K / L) * (int)sizeof(T) <= 16) return L;
    return lpr_default<T>(K);
}

template <typename T>
static int ls_dispatch(int K, int caliber, const ad_csr* A, const void* X, const double* w,
                       const uint8_t* cf, const void* mu, int target, int32_t* P_col,
                       double* P_val, double* ls_val, int32_t* row_status, double* bs,
                       unsigned* st, const LaunchCfg& cfg, hipStream_t s) {
    return with_k<T>(K, [&](auto kc) {
        constexpr int KK = decltype(kc)::value;
        const int lpr = cfg.lpr > 0 ? cfg.lpr : ls_lpr_default<T>(KK);
        return with_lpr<T, KK>(lpr, [&](auto lc) {
            constexpr int L = decltype(lc)::value;
            ls_go<T, KK, L>(caliber, A, X, w, cf, mu, target, P_col, P_val, ls_val, row_status, bs,
                            st, cfg, s);
        });
    });
}

// ---------------------------------------------------------------- fused distances + LS rows
// One pass per row group: the distances of the row (with the fused strength
// row), the C-neighbour candidates picked from them as they are computed,
// then the LS row on the FP64 target the distance pass formed.  The row's
// CSR entries, distances and panel rows are read once for both results.
template <typename T, int K, int LPR, int CALT, bool WEIGHTED, int UN>
__global__ __launch_bounds__(kBlock) void dist_ls_kernel(
    int n, const int* __restrict__ rp, const int* __restrict__ ci, const T* __restrict__ av,
    const T* __restrict__ X, const double* __restrict__ w, int target, T* __restrict__ mu,
    double theta, const uint8_t* __restrict__ fmask, uint8_t* __restrict__ strong,
    int* __restrict__ nstrong, const uint8_t* __restrict__ cf, int cal, int* __restrict__ Pcol,
    double* __restrict__ Pval, double* __restrict__ lsv, int* __restrict__ rstat,
    double* __restrict__ block_sums, int iter, int xcd, unsigned* status) {
    using S = Shape<T, K, LPR>;
    constexpr int V = S::V;
    __shared__ double wsum[kWavesPerBlock];
    const int lane = threadIdx.x & (kWave - 1);
    const int g = lane / LPR, l = lane % LPR;
    const int wv = threadIdx.x / kWave;
    const int64_t rows_per_tile = (int64_t)S::RPB * iter;
    const int64_t ntiles = (n + rows_per_tile - 1) / rows_per_tile;
    const int64_t tile = map_tile(ntiles, xcd);
    double wd[V];
    T wt[V];
#pragma unroll
    for (int q = 0; q < V; ++q) {
        wd[q] = WEIGHTED ? w[l * V + q] : 1.0;
        wt[q] = (T)wd[q];
    }
    const bool plain = target == AD_TARGET_PLAIN;
    double fsum = 0.0;
    // the tile's rows, reading panel rows from `src`
    auto rows = [&](const auto& src) {
        using Src = typename std::decay<decltype(src)>::type;
        constexpr int G = Src::kCoop ? CoopGather<T, V, LPR>::G : 1;
        for (int it = 0; it < iter; ++it) {
            const int64_t iw = tile * rows_per_tile + (int64_t)it * S::RPB + wv * S::RPW;
            if (iw >= n) break;  // whole wavefront
            const int64_t i64 = iw + g;
            const bool ghost = i64 >= n;
            if (ghost && G == 1) break;  // ghosts only serve group loads
            const int i = ghost ? n - 1 : (int)i64;
            const bool isF = !ghost && cf[i] == 0;
            T smu[CALT];
            int scol[CALT];
            int nsel = 0;
#pragma unroll
            for (int q = 0; q < CALT; ++q) {
                smu[q] = T(0);
                scol[q] = -1;
            }
            double t64[V], d;
            algdist_row_sel<S, T, K, WEIGHTED, UN>(
                i, ghost, l, rp, ci, rp, ci, av, src, wd, wt, plain, mu, nullptr, theta, fmask,
                strong, nstrong, status,
                [&](int j, T m) {
                    if (isF && cf[j] != 0) ls_insert<T, CALT>(smu, scol, nsel, cal, m, j);
                },
                t64, d);
            if (isF) {
                const int st = (!plain && d == 0.0) ? 3 : 0;
                const double v = ls_solve<T, K, LPR, CALT>(i, l, t64, wd, src, scol, nsel, st, cal,
                                                           Pcol, Pval, lsv, rstat);
                if (l == 0) fsum += v;
            } else if (l == 0 && !ghost) {
                ls_c_row(i, cal, Pcol, Pval, lsv, rstat);
            }
        }
    };
    if (tile >= 0 && tile < ntiles) rows(GlobalRows<T, K>{X});
    if (block_sums) {
        // fixed-order reduction: xor butterfly in the wave, then waves in order
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) fsum += __shfl_xor(fsum, o, kWave);
        if (lane == 0) wsum[wv] = fsum;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int q = 0; q < kWavesPerBlock; ++q) s += wsum[q];
            block_sums[blockIdx.x] = s;
        }
    }
}

template <typename T, int K, int LPR>
static int dist_ls_grid(int n, const LaunchCfg& cfg) {
    using S = Shape<T, K, LPR>;
    const int64_t rpt = (int64_t)S::RPB * cfg.iter;
    const int64_t ntiles = (n + rpt - 1) / rpt;
    return grid_for_tiles(ntiles, cfg.xcd_map);
}

int dist_ls_blocks(int dtype, int K, int n, const LaunchCfg& cfg) {
    int grid = 1;
    auto f = [&](auto tag) {
        using T = decltype(tag);
        with_k<T>(K, [&](auto kc) {
            constexpr int KK = decltype(kc)::value;
            return with_lpr<T, KK>(cfg.lpr > 0 ? cfg.lpr : ls_lpr_default<T>(KK), [&](auto lc) {
                constexpr int L = decltype(lc)::value;
                grid = dist_ls_grid<T, KK, L>(n, cfg);
            });
        });
    };
    if (dtype == AD_F32) f(float());
    else f(double());
    return grid;
}

template <typename T>
static int dist_ls_dispatch(int K, int caliber, const ad_csr* A, const void* X, const double* w,
                            int target, void* mu, double theta, const uint8_t* fmask,
                            uint8_t* strong, int32_t* nstrong, const uint8_t* cf, int32_t* P_col,
                            double* P_val, double* ls_val, int32_t* row_status, double* bs,
                            unsigned* st, const LaunchCfg& cfg, hipStream_t s) {
    return with_k<T>(K, [&](auto kc) {
        constexpr int KK = decltype(kc)::value;
        const int lpr = cfg.lpr > 0 ? cfg.lpr : ls_lpr_default<T>(KK);
        return with_lpr<T, KK>(lpr, [&](auto lc) {
            constexpr int L = decltype(lc)::value;
            const int grid = dist_ls_grid<T, KK, L>(A->n, cfg);
            const bool long_rows = nnz_bucket(A->nnz, A->n) >= 2;
            auto go = [&](auto calt, auto weighted) {
                dist_unroll<T, KK, L>(long_rows, [&](auto uc) {
                    dist_ls_kernel<T, KK, L, decltype(calt)::value, decltype(weighted)::value,
                                   decltype(uc)::value><<<dim3(grid), dim3(kBlock), 0, s>>>(
                        A->n, A->row_ptr, A->col, (const T*)A->val, (const T*)X, w, target,
                        (T*)mu, theta, fmask, strong, nstrong, cf, caliber, P_col, P_val, ls_val,
                        row_status, bs, cfg.iter, cfg.xcd_map, st);
                });
            };
            using C4 = std::integral_constant<int, 4>;
            using C8 = std::integral_constant<int, 8>;
            using Y = std::true_type;
            using N = std::false_type;
            if (caliber <= 4) w ? go(C4(), Y()) : go(C4(), N());
            else w ? go(C8(), Y()) : go(C8(), N());
        });
    });
}

int launch_dist_ls(int dtype, int K, int caliber, const ad_csr* A, const void* X, const double* w,
                   int target, void* mu, double theta, const uint8_t* fmask, uint8_t* strong,
                   int32_t* nstrong, const uint8_t* cf, int32_t* P_col, double* P_val,
                   double* ls_val, int32_t* row_status, double* block_sums, double* ls_sum,
                   unsigned* status, const LaunchCfg& cfg, hipStream_t s) {
    if (A->n == 0) {
        return ls_sum ? launch_fill_f64(ls_sum, 1, 0.0, s) : AD_OK;
    }
    double* bs = ls_sum ? block_sums : nullptr;
    const int rc = (dtype == AD_F32)
                       ? dist_ls_dispatch<float>(K, caliber, A, X, w, target, mu, theta, fmask,
                                                 strong, nstrong, cf, P_col, P_val, ls_val,
                                                 row_status, bs, status, cfg, s)
                       : dist_ls_dispatch<double>(K, caliber, A, X, w, target, mu, theta, fmask,
                                                  strong, nstrong, cf, P_col, P_val, ls_val,
                                                  row_status, bs, status, cfg, s);
    if (rc) return rc;
    AD_HIP(hipGetLastError());
    if (ls_sum) {
        const int nb = dist_ls_blocks(dtype, K, A->n, cfg);
        sum_blocks_kernel<<<dim3(1), dim3(1024), 0, s>>>(block_sums, nb, ls_sum);
        AD_HIP(hipGetLastError());
    }
    return AD_OK;
}

int launch_ls_interp(int dtype, int K, int caliber, const ad_csr* A, const void* X,
                     const double* w, const uint8_t* cf, const void* mu, int target,
                     int32_t* P_col, double* P_val, double* ls_val, int32_t* row_status,
                     double* block_sums, double* ls_sum, unsigned* status,
                     const LaunchCfg& cfg, hipStream_t s) {
    if (A->n == 0) {
        return ls_sum ? launch_fill_f64(ls_sum, 1, 0.0, s) : AD_OK;
    }
    double* bs = ls_sum ? block_sums : nullptr;
    const int rc = (dtype == AD_F32)
                       ? ls_dispatch<float>(K, caliber, A, X, w, cf, mu, target, P_col, P_val,
                                            ls_val, row_status, bs, status, cfg, s)
                       : ls_dispatch<double>(K, caliber, A, X, w, cf, mu, target, P_col, P_val,
                                             ls_val, row_status, bs, status, cfg, s);
    if (rc) return rc;
    AD_HIP(hipGetLastError());
    if (ls_sum) {
        const int nb = ls_interp_blocks(dtype, K, A->n, cfg);
        sum_blocks_kernel<<<dim3(1), dim3(1024), 0, s>>>(block_sums, nb, ls_sum);
        AD_HIP(hipGetLastError());
    }
    return AD_OK;
}

}  // namespace ad
