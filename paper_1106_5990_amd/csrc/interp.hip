// interp.hip -- least-squares interpolation rows (Sec. 3.1, eq:LSfuncrowi /
// eq:modls) on interpolatory sets C_i picked by the one-point distances
// (the systematic scan of the final remark of Sec. 4.3).
//
// One row group per row.  Every lane of the group scans the row's entries
// (same addresses, one request per wave) and keeps the `caliber` C-neighbours
// of smallest mu in a register-resident sorted list.  The group then gathers
// those panel rows and the target, forms the FP64 normal equations
//     G_ab = sum_k w_k x_a^k x_b^k,  h_a = sum_k w_k x_a^k t^k
// (FP32 x FP32 products are exact in FP64), reduces them over K with
// butterflies, and every lane solves the tiny system by Cholesky in
// increasing-mu column order, dropping a column whose pivot is <= 1e-12 of
// its Gram diagonal.  The functional at the minimiser is then evaluated
// from its definition in FP64.
#include <math.h>

#include "device.h"
#include "internal.h"

namespace ad {

template <typename T, int K, int CALT>
__global__ __launch_bounds__(kBlock) void ls_interp_kernel(
    int n, const int* __restrict__ rp, const int* __restrict__ ci, const T* __restrict__ av,
    const T* __restrict__ X, const double* __restrict__ w, const uint8_t* __restrict__ cf,
    const T* __restrict__ mu, int cal, int target, int* __restrict__ Pcol,
    double* __restrict__ Pval, double* __restrict__ lsv, int* __restrict__ rstat,
    double* __restrict__ block_sums, int iter, int xcd, unsigned* status) {
    using S = Shape<T, K>;
    constexpr int V = S::V, LPR = S::LPR;
    constexpr int NG = CALT * (CALT + 1) / 2;
    const int lane = threadIdx.x & (kWave - 1);
    const int g = lane / LPR, l = lane % LPR;
    const int wv = threadIdx.x / kWave;
    const int64_t rows_per_tile = (int64_t)S::RPB * iter;
    const int64_t ntiles = (n + rows_per_tile - 1) / rows_per_tile;
    const int64_t tile = xcd ? xcd_tile(ntiles) : (int64_t)blockIdx.x;
    double fsum = 0.0;  // this group's F-row ls values (lane 0 of the group)

    double wd[V];
#pragma unroll
    for (int q = 0; q < V; ++q) wd[q] = w ? w[l * V + q] : 1.0;

    if (tile >= 0 && tile < ntiles) {
        for (int it = 0; it < iter; ++it) {
            const int64_t i64 = tile * rows_per_tile + (int64_t)it * S::RPB + wv * S::RPW + g;
            if (i64 >= n) break;
            const int i = (int)i64;
            int* pc = Pcol + (size_t)i * cal;
            double* pv = Pval + (size_t)i * cal;
            if (cf[i]) {  // a C point interpolates itself
                for (int q = l; q < cal; q += LPR) {
                    pc[q] = (q == 0) ? i : -1;
                    pv[q] = (q == 0) ? 1.0 : 0.0;
                }
                if (l == 0) {
                    lsv[i] = 0.0;
                    rstat[i] = 0;
                }
                continue;
            }
            const int e0 = rp[i], e1 = rp[i + 1];
            int st = 0;

            // target, in FP64 from the panel type
            Frag<T, V> tf = load_frag<T, V>(X + (size_t)i * K + l * V);
            double t[V];
#pragma unroll
            for (int q = 0; q < V; ++q) t[q] = (double)tf.v[q];
            if (target == AD_TARGET_RESIDUAL) {  // formed in FP64
                double y[V];
#pragma unroll
                for (int q = 0; q < V; ++q) y[q] = 0.0;
                double d = 0.0;
                for (int e = e0; e < e1; ++e) {
                    const int j = ci[e];
                    const double a = (double)av[e];
                    Frag<T, V> xj = load_frag<T, V>(X + (size_t)j * K + l * V);
#pragma unroll
                    for (int q = 0; q < V; ++q) y[q] = fma(a, (double)xj.v[q], y[q]);
                    if (j == i) d = a;
                }
                if (d != 0.0) {
#pragma unroll
                    for (int q = 0; q < V; ++q) t[q] = t[q] - y[q] / d;
                } else {
                    st = 3;
                    if (l == 0) flag(status, AD_STAT_ZERO_DIAG);
                }
            }

            // C_i: the cal candidates of least (mu, column), sorted
            T smu[CALT];
            int scol[CALT];
            int nsel = 0;
#pragma unroll
            for (int q = 0; q < CALT; ++q) {
                smu[q] = T(0);
                scol[q] = -1;
            }
            for (int e = e0; e < e1; ++e) {
                const int j = ci[e];
                if (j == i || !cf[j]) continue;
                const T m = mu[e];
                if (m != m) continue;  // NaN distances are never chosen
                int pos = 0;           // insert after the equal ones (lower column)
#pragma unroll
                for (int q = 0; q < CALT; ++q)
                    if (q < nsel && smu[q] <= m) pos = q + 1;
                if (pos >= cal) continue;
#pragma unroll
                for (int q = CALT - 1; q > 0; --q)
                    if (q > pos && q < cal) {
                        smu[q] = smu[q - 1];
                        scol[q] = scol[q - 1];
                    }
#pragma unroll
                for (int q = 0; q < CALT; ++q)
                    if (q == pos) {
                        smu[q] = m;
                        scol[q] = j;
                    }
                nsel = (nsel < cal) ? nsel + 1 : cal;
            }

            double val;
            double coef[CALT];
            bool keep[CALT];
#pragma unroll
            for (int q = 0; q < CALT; ++q) {
                coef[q] = 0.0;
                keep[q] = false;
            }
            if (nsel == 0) {
                double f = 0.0;
#pragma unroll
                for (int q = 0; q < V; ++q) f = fma(wd[q] * t[q], t[q], f);
                val = group_sum<LPR>(f);
                st = st ? st : 1;
            } else {
                // gather the selected panel rows (FP64 copies)
                double xs[CALT][V];
#pragma unroll
                for (int a = 0; a < CALT; ++a) {
                    if (a < nsel) {
                        Frag<T, V> f = load_frag<T, V>(X + (size_t)scol[a] * K + l * V);
#pragma unroll
                        for (int q = 0; q < V; ++q) xs[a][q] = (double)f.v[q];
                    } else {
#pragma unroll
                        for (int q = 0; q < V; ++q) xs[a][q] = 0.0;
                    }
                }
                // normal equations: lower triangle of G (row-major packed) and h
                double G[NG], hv[CALT];
                int gi = 0;
#pragma unroll
                for (int a = 0; a < CALT; ++a) {
                    double ha = 0.0;
#pragma unroll
                    for (int q = 0; q < V; ++q) ha = fma(wd[q] * xs[a][q], t[q], ha);
                    hv[a] = group_sum<LPR>(ha);
#pragma unroll
                    for (int b = 0; b <= a; ++b) {
                        double gab = 0.0;
#pragma unroll
                        for (int q = 0; q < V; ++q) gab = fma(wd[q] * xs[a][q], xs[b][q], gab);
                        G[gi++] = group_sum<LPR>(gab);
                    }
                }
                // Cholesky in increasing-mu order with the drop rule
                double L[NG];
#pragma unroll
                for (int q = 0; q < NG; ++q) L[q] = 0.0;
#pragma unroll
                for (int a = 0; a < CALT; ++a) {
                    if (a >= nsel) continue;
                    const int ra = a * (a + 1) / 2;
#pragma unroll
                    for (int b = 0; b < a; ++b) {
                        const int rb = b * (b + 1) / 2;
                        double s = G[ra + b];
#pragma unroll
                        for (int c = 0; c < b; ++c)
                            if (keep[c]) s -= L[ra + c] * L[rb + c];
                        L[ra + b] = keep[b] ? s / L[rb + b] : 0.0;
                    }
                    double dpiv = G[ra + a];
#pragma unroll
                    for (int b = 0; b < a; ++b)
                        if (keep[b]) dpiv -= L[ra + b] * L[ra + b];
                    keep[a] = dpiv > 1e-12 * G[ra + a];
                    L[ra + a] = keep[a] ? sqrt(dpiv) : 1.0;
                    if (!keep[a]) st = st ? st : 2;
                }
                // L z = h, then L^T coef = z, over the kept columns
                double z[CALT];
#pragma unroll
                for (int a = 0; a < CALT; ++a) {
                    const int ra = a * (a + 1) / 2;
                    double s = hv[a];
#pragma unroll
                    for (int b = 0; b < a; ++b)
                        if (keep[b]) s -= L[ra + b] * z[b];
                    z[a] = keep[a] ? s / L[ra + a] : 0.0;
                }
#pragma unroll
                for (int a = CALT - 1; a >= 0; --a) {
                    double s = z[a];
#pragma unroll
                    for (int b = a + 1; b < CALT; ++b)
                        if (keep[b]) s -= L[b * (b + 1) / 2 + a] * coef[b];
                    coef[a] = keep[a] ? s / L[a * (a + 1) / 2 + a] : 0.0;
                }
                // functional at the minimiser, by its definition
                double f = 0.0;
#pragma unroll
                for (int q = 0; q < V; ++q) {
                    double r = t[q];
#pragma unroll
                    for (int a = 0; a < CALT; ++a)
                        if (keep[a]) r -= coef[a] * xs[a][q];
                    f = fma(wd[q] * r, r, f);
                }
                val = group_sum<LPR>(f);
            }
            if (l == 0) {
                int o = 0;
#pragma unroll
                for (int a = 0; a < CALT; ++a)
                    if (keep[a]) {
                        pc[o] = scol[a];
                        pv[o] = coef[a];
                        ++o;
                    }
                for (; o < cal; ++o) {
                    pc[o] = -1;
                    pv[o] = 0.0;
                }
                lsv[i] = val;
                rstat[i] = st;
                fsum += val;
            }
        }
    }
    if (block_sums) {
        // fixed-order block sum: groups in lane order, waves in order
        __shared__ double part[kBlock];
        part[threadIdx.x] = fsum;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int q = 0; q < kBlock; ++q) s += part[q];
            block_sums[blockIdx.x] = s;
        }
    }
}

__global__ __launch_bounds__(kBlock) void sum_blocks_kernel(const double* __restrict__ part,
                                                            int m, double* __restrict__ out) {
    __shared__ double acc[kBlock];
    double s = 0.0;
    for (int q = threadIdx.x; q < m; q += kBlock) s += part[q];
    acc[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < kBlock; ++q) t += acc[q];
        *out = t;
    }
}

template <typename T, int K>
static int ls_grid(int n, const LaunchCfg& cfg) {
    using S = Shape<T, K>;
    const int64_t rpt = (int64_t)S::RPB * cfg.iter;
    const int64_t ntiles = (n + rpt - 1) / rpt;
    return cfg.xcd_map ? grid_for_tiles(ntiles) : (int)(ntiles > 0 ? ntiles : 1);
}

int ls_interp_blocks(int dtype, int K, int n, const LaunchCfg& cfg) {
#define G_(T)                                        \
    switch (K) {                                     \
        case 2: return ls_grid<T, 2>(n, cfg);        \
        case 4: return ls_grid<T, 4>(n, cfg);        \
        case 8: return ls_grid<T, 8>(n, cfg);        \
        case 16: return ls_grid<T, 16>(n, cfg);      \
        case 32: return ls_grid<T, 32>(n, cfg);      \
        case 64: return ls_grid<T, 64>(n, cfg);      \
        default: return 0;                           \
    }
    if (dtype == AD_F32) {
        G_(float)
    } else {
        G_(double)
    }
#undef G_
}

template <typename T, int K>
static void ls_go(int caliber, const ad_csr* A, const void* X, const double* w, const uint8_t* cf,
                  const void* mu, int target, int32_t* P_col, double* P_val, double* ls_val,
                  int32_t* row_status, double* block_sums, unsigned* st, const LaunchCfg& cfg,
                  hipStream_t s) {
    const int grid = ls_grid<T, K>(A->n, cfg);
    if (caliber <= 4)
        ls_interp_kernel<T, K, 4><<<dim3(grid), dim3(kBlock), 0, s>>>(
            A->n, A->row_ptr, A->col, (const T*)A->val, (const T*)X, w, cf, (const T*)mu, caliber,
            target, P_col, P_val, ls_val, row_status, block_sums, cfg.iter, cfg.xcd_map, st);
    else
        ls_interp_kernel<T, K, 8><<<dim3(grid), dim3(kBlock), 0, s>>>(
            A->n, A->row_ptr, A->col, (const T*)A->val, (const T*)X, w, cf, (const T*)mu, caliber,
            target, P_col, P_val, ls_val, row_status, block_sums, cfg.iter, cfg.xcd_map, st);
}

#define AD_K_SWITCH(T, FN, ...)                         \
    switch (K) {                                        \
        case 2: FN<T, 2>(__VA_ARGS__); break;           \
        case 4: FN<T, 4>(__VA_ARGS__); break;           \
        case 8: FN<T, 8>(__VA_ARGS__); break;           \
        case 16: FN<T, 16>(__VA_ARGS__); break;         \
        case 32: FN<T, 32>(__VA_ARGS__); break;         \
        case 64: FN<T, 64>(__VA_ARGS__); break;         \
        default: return AD_EINVAL;                      \
    }

int launch_ls_interp(int dtype, int K, int caliber, const ad_csr* A, const void* X,
                     const double* w, const uint8_t* cf, const void* mu, int target,
                     int32_t* P_col, double* P_val, double* ls_val, int32_t* row_status,
                     double* block_sums, double* ls_sum, unsigned* status,
                     const LaunchCfg& cfg, hipStream_t s) {
    if (A->n == 0) {
        if (ls_sum) AD_HIP(hipMemsetAsync(ls_sum, 0, sizeof(double), s));
        return AD_OK;
    }
    double* bs = ls_sum ? block_sums : nullptr;
    if (dtype == AD_F32) {
        AD_K_SWITCH(float, ls_go, caliber, A, X, w, cf, mu, target, P_col, P_val, ls_val,
                    row_status, bs, status, cfg, s);
    } else {
        AD_K_SWITCH(double, ls_go, caliber, A, X, w, cf, mu, target, P_col, P_val, ls_val,
                    row_status, bs, status, cfg, s);
    }
    AD_HIP(hipGetLastError());
    if (ls_sum) {
        const int nb = ls_interp_blocks(dtype, K, A->n, cfg);
        sum_blocks_kernel<<<dim3(1), dim3(kBlock), 0, s>>>(block_sums, nb, ls_sum);
        AD_HIP(hipGetLastError());
    }
    return AD_OK;
}

}  // namespace ad
