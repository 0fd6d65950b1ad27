// adjoint.hip -- gradient of the LS interpolation loss with respect to the
// matrix values and the Jacobi damping omega.
//
// Forward (done by the other calls): x^0 from the start, S damped-Jacobi
// sweeps x^{s+1} = x^s - omega D^{-1} A x^s, LS rows p fitted to x^S (plain
// target, Sec. 3.1 eq:LSfuncrowi), loss L = sum_{i in F} ls_val_i.
//
// Backward, all FP64:
//   seed   g_i = dL (2 w (rho_i [i in F] - sum_{q: i in C_q} p_qi rho_q)),
//          rho_q = x_q - sum_j p_qj x_j, p held fixed (it minimises each row's
//          functional, so its own variation does not enter);
//   sweep  s = S-1 .. 0:  y = D^{-1} g;
//          dL/da_ij -= omega <y_i, x_j^s>;  dL/da_ii += omega <y_i, (A x^s)_i> / a_ii;
//          dL/domega -= <y, A x^s>;  g <- g - omega A^T y.
// The transpose products are gathers over a column-major (CSC) index of the
// pattern built here: column j's entries (q, j) sorted by row q, each with
// its position in the CSR, so any pattern works; for a structurally
// symmetric one, column i lists the rows of row i's columns in the same
// order, and the sums are those of a gather through row i.
// Iterates that are not checkpointed are recomputed forward from the last
// checkpoint.  Every reduction has a fixed order (no atomics on values).
#include <math.h>

#include "device.h"
#include "internal.h"
#include "rowops.h"

namespace ad {

// ---------------------------------------------------------------- CSC index
// cnt[j] = entries in column j (cnt zeroed by the caller).
__global__ __launch_bounds__(kBlock) void col_count_kernel(int64_t nnz, const int* __restrict__ ci,
                                                           int* __restrict__ cnt) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e < nnz) atomicAdd(&cnt[ci[e]], 1);
}

// Structurally symmetric patterns: the rows of column j are the columns of
// row j, so entry (i, j) goes to the position of i in row j (binary search)
// and every column comes out in increasing row order with no atomics.  An
// entry whose transpose is missing, repeated or outside column j's segment
// sets *asym; the general path below then redoes the whole index.  Also
// writes the diagonal (when diag is not null).
__global__ __launch_bounds__(kBlock) void col_fill_sym_kernel(
    int n, const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ av,
    const int64_t* __restrict__ cp, int* __restrict__ trow, int* __restrict__ tent,
    double* __restrict__ diag, int* __restrict__ asym, unsigned* status) {
    const int64_t i64 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i64 >= n) return;
    const int i = (int)i64;
    double d = 0.0;
    bool bad = false;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        const int j = ci[e];
        if (diag && j == i) d = av[e];
        const int r0 = rp[j], r1 = rp[j + 1];
        int lo = r0, hi = r1;  // first entry of row j whose column is >= i
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (ci[mid] < i) lo = mid + 1;
            else hi = mid;
        }
        const int64_t pos = lo - r0;
        if (lo < r1 && ci[lo] == i && (lo + 1 == r1 || ci[lo + 1] != i) &&
            pos < cp[j + 1] - cp[j]) {
            trow[cp[j] + pos] = i;
            tent[cp[j] + pos] = e;
        } else {
            bad = true;
        }
    }
    if (bad) atomicOr(asym, 1);
    if (diag) {
        diag[i] = d;
        if (d == 0.0) flag(status, AD_STAT_ZERO_DIAG);
    }
}

// Row i's entries go to their columns' segments in arrival order (cur
// zeroed by the caller); the per-column sort below fixes the order.  Also
// writes the diagonal (when diag is not null).
__global__ __launch_bounds__(kBlock) void col_fill_kernel(int n, const int* __restrict__ rp,
                                                          const int* __restrict__ ci,
                                                          const double* __restrict__ av,
                                                          const int64_t* __restrict__ cp,
                                                          int* __restrict__ cur,
                                                          int* __restrict__ trow,
                                                          int* __restrict__ tent,
                                                          double* __restrict__ diag,
                                                          const int* __restrict__ asym,
                                                          unsigned* status) {
    const int64_t i64 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i64 >= n || *asym == 0) return;
    const int i = (int)i64;
    double d = 0.0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        const int j = ci[e];
        if (diag && j == i) d = av[e];
        const int64_t f = cp[j] + atomicAdd(&cur[j], 1);
        trow[f] = i;
        tent[f] = e;
    }
    if (diag) {
        diag[i] = d;
        if (d == 0.0) flag(status, AD_STAT_ZERO_DIAG);
    }
}

// Sorts each column's (row, entry) pairs by row (insertion sort: columns
// hold a handful of entries), one column per thread.
__global__ __launch_bounds__(kBlock) void col_sort_kernel(int n, const int64_t* __restrict__ cp,
                                                          int* __restrict__ trow,
                                                          int* __restrict__ tent,
                                                          const int* __restrict__ asym) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n || *asym == 0) return;
    const int64_t a = cp[j], b = cp[j + 1];
    for (int64_t f = a + 1; f < b; ++f) {
        const int r = trow[f], t = tent[f];
        int64_t g = f - 1;
        while (g >= a && trow[g] > r) {
            trow[g + 1] = trow[g];
            tent[g + 1] = tent[g];
            --g;
        }
        trow[g + 1] = r;
        tent[g + 1] = t;
    }
}

// R_i = 2 dL w .* rho_i for F rows (rho = x_i - sum_q P_val[i,q] x_{P_col[i,q]}), 0 for C rows.
template <int K, int LPR>
__global__ __launch_bounds__(kBlock) void ls_residual_kernel(int n, const double* __restrict__ X,
                                                             const double* __restrict__ w,
                                                             const uint8_t* __restrict__ cf,
                                                             const int* __restrict__ Pcol,
                                                             const double* __restrict__ Pval,
                                                             int cal, const double* __restrict__ dL,
                                                             double* __restrict__ R) {
    using S = Shape<double, K, LPR>;
    constexpr int V = S::V, C = S::C;
    const int lane = threadIdx.x & (kWave - 1);
    const int g = lane / LPR, l = lane % LPR;
    const int64_t i64 = ((int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave) * S::RPW + g;
    if (i64 >= n) return;
    const int i = (int)i64;
    Frag<double, V> r;
    if (cf[i]) {
#pragma unroll
        for (int q = 0; q < V; ++q) r.v[q] = 0.0;
    } else {
        r = load_lane<double, V, C>(X + (size_t)i * K + l * V);
        for (int q = 0; q < cal; ++q) {
            const int j = Pcol[(size_t)i * cal + q];
            if (j < 0) continue;
            const double p = Pval[(size_t)i * cal + q];
            Frag<double, V> xj = load_lane<double, V, C>(X + (size_t)j * K + l * V);
#pragma unroll
            for (int v = 0; v < V; ++v) r.v[v] -= p * xj.v[v];
        }
        const double s = 2.0 * (*dL);
#pragma unroll
        for (int v = 0; v < V; ++v) r.v[v] *= s * (w ? w[l * V + v] : 1.0);
    }
    store_lane<double, V, C>(R + (size_t)i * K + l * V, r);
}

// g_j = R_j - sum over the rows q that interpolate from j of p_qj R_q (every
// such q stores (q, j), so they are found in column j).
template <int K, int LPR>
__global__ __launch_bounds__(kBlock) void ls_seed_kernel(int n, const int64_t* __restrict__ cp,
                                                         const int* __restrict__ trow,
                                                         const uint8_t* __restrict__ cf,
                                                         const int* __restrict__ Pcol,
                                                         const double* __restrict__ Pval, int cal,
                                                         const double* __restrict__ R,
                                                         double* __restrict__ G) {
    using S = Shape<double, K, LPR>;
    constexpr int V = S::V, C = S::C;
    const int lane = threadIdx.x & (kWave - 1);
    const int g = lane / LPR, l = lane % LPR;
    const int64_t j64 = ((int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave) * S::RPW + g;
    if (j64 >= n) return;
    const int j = (int)j64;
    Frag<double, V> acc = load_lane<double, V, C>(R + (size_t)j * K + l * V);
    for (int64_t f = cp[j]; f < cp[j + 1]; ++f) {
        const int q = trow[f];  // (q, j) is stored
        if (q == j || cf[q]) continue;
        double p = 0.0;
        bool hit = false;
        for (int c = 0; c < cal; ++c)
            if (Pcol[(size_t)q * cal + c] == j) {
                p = Pval[(size_t)q * cal + c];
                hit = true;
            }
        if (!hit) continue;
        Frag<double, V> rq = load_lane<double, V, C>(R + (size_t)q * K + l * V);
#pragma unroll
        for (int v = 0; v < V; ++v) acc.v[v] -= p * rq.v[v];
    }
    store_lane<double, V, C>(G + (size_t)j * K + l * V, acc);
}

// y = D^{-1} g (rows with a zero diagonal get y = 0)
template <int K, int LPR>
__global__ __launch_bounds__(kBlock) void dinv_kernel(int n, const double* __restrict__ diag,
                                                      const double* __restrict__ G,
                                                      double* __restrict__ Y) {
    using S = Shape<double, K, LPR>;
    constexpr int V = S::V, C = S::C;
    const int lane = threadIdx.x & (kWave - 1);
    const int g = lane / LPR, l = lane % LPR;
    const int64_t i64 = ((int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave) * S::RPW + g;
    if (i64 >= n) return;
    const double d = diag[i64];
    Frag<double, V> v = load_lane<double, V, C>(G + (size_t)i64 * K + l * V);
#pragma unroll
    for (int q = 0; q < V; ++q) v.v[q] = (d != 0.0) ? v.v[q] / d : 0.0;
    store_lane<double, V, C>(Y + (size_t)i64 * K + l * V, v);
}

// y = D^{-1} E_c g: rows of colour c with a nonzero diagonal, 0 elsewhere
// (the adjoint of one colour phase).
template <int K, int LPR>
__global__ __launch_bounds__(kBlock) void dinv_colour_kernel(int n, const double* __restrict__ diag,
                                                             const int* __restrict__ color, int c,
                                                             const double* __restrict__ G,
                                                             double* __restrict__ Y) {
    using S = Shape<double, K, LPR>;
    constexpr int V = S::V, C = S::C;
    const int lane = threadIdx.x & (kWave - 1);
    const int g = lane / LPR, l = lane % LPR;
    const int64_t i64 = ((int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave) * S::RPW + g;
    if (i64 >= n) return;
    const double d = diag[i64];
    const bool on = color[i64] == c && d != 0.0;
    Frag<double, V> v = load_lane<double, V, C>(G + (size_t)i64 * K + l * V);
#pragma unroll
    for (int q = 0; q < V; ++q) v.v[q] = on ? v.v[q] / d : 0.0;
    store_lane<double, V, C>(Y + (size_t)i64 * K + l * V, v);
}

// One colour phase in natural row order (the recomputation of the forward
// sweeps): rows of colour c become x_i - (A x)_i / a_ii (held when a_ii = 0),
// every other row is copied.  The row arithmetic is the colour-major phase
// kernel's (same entry order, same operations), so the iterates it
// recomputes are those the forward pass checkpointed.
template <int K, int LPR>
__global__ __launch_bounds__(kBlock) void gs_phase_nat_kernel(int n, const int* __restrict__ rp,
                                                              const int* __restrict__ ci,
                                                              const double* __restrict__ av,
                                                              const int* __restrict__ color, int c,
                                                              const double* __restrict__ Xin,
                                                              double* __restrict__ Xout,
                                                              unsigned* status) {
    using S = Shape<double, K, LPR>;
    constexpr int V = S::V, C = S::C;
    const int lane = threadIdx.x & (kWave - 1);
    const int g = lane / LPR, l = lane % LPR;
    const int64_t i64 = ((int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave) * S::RPW + g;
    if (i64 >= n) return;
    const int i = (int)i64;
    if (color[i] == c) {
        double y[V], d;
        Frag<double, V> xi;
        row_spmm<S, double, K>(i, rp[i], rp[i + 1], ci, av, l, [&](int) { return Xin; }, y, d, xi);
        Frag<double, V> out;
        if (d == 0.0) {
            out = load_lane<double, V, C>(Xin + (size_t)i * K + l * V);
        } else {
#pragma unroll
            for (int q = 0; q < V; ++q) out.v[q] = xi.v[q] - y[q] / d;
        }
        store_lane<double, V, C>(Xout + (size_t)i * K + l * V, out);
    } else {
        store_lane<double, V, C>(Xout + (size_t)i * K + l * V,
                                 load_lane<double, V, C>(Xin + (size_t)i * K + l * V));
    }
}

// dL/dw_k partials: part[b * K + k] = sum over block b's F rows of rho_ik^2,
// rho_i = x_i - sum_q P_val[i,q] x_{P_col[i,q]}.  Fixed order: a lane's
// entries, then the row groups of a wave (xor butterfly over lanes with the
// same entries), then the waves in order.
template <int K, int LPR>
__global__ __launch_bounds__(kBlock) void gradw_partials_kernel(
    int n, const double* __restrict__ X, const uint8_t* __restrict__ cf,
    const int* __restrict__ Pcol, const double* __restrict__ Pval, int cal,
    double* __restrict__ part) {
    using S = Shape<double, K, LPR>;
    constexpr int V = S::V, C = S::C;
    __shared__ double acc[kWavesPerBlock][K];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int g = lane / LPR, l = lane % LPR;
    const int64_t i64 = ((int64_t)blockIdx.x * kWavesPerBlock + wv) * S::RPW + g;
    double sq[V];
#pragma unroll
    for (int q = 0; q < V; ++q) sq[q] = 0.0;
    if (i64 < n && !cf[i64]) {
        const int i = (int)i64;
        Frag<double, V> r = load_lane<double, V, C>(X + (size_t)i * K + l * V);
        for (int q = 0; q < cal; ++q) {
            const int j = Pcol[(size_t)i * cal + q];
            if (j < 0) continue;
            const double p = Pval[(size_t)i * cal + q];
            const Frag<double, V> xj = load_lane<double, V, C>(X + (size_t)j * K + l * V);
#pragma unroll
            for (int v = 0; v < V; ++v) r.v[v] -= p * xj.v[v];
        }
#pragma unroll
        for (int v = 0; v < V; ++v) sq[v] = r.v[v] * r.v[v];
    }
#pragma unroll
    for (int o = kWave / 2; o >= LPR; o >>= 1)
#pragma unroll
        for (int v = 0; v < V; ++v) sq[v] += __shfl_xor(sq[v], o, kWave);
    if (g == 0)
#pragma unroll
        for (int v = 0; v < V; ++v) acc[wv][l * V + v] = sq[v];
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += kBlock) {
        double t = 0.0;
        for (int q = 0; q < kWavesPerBlock; ++q) t += acc[q][k];
        part[(size_t)blockIdx.x * K + k] = t;
    }
}

// out[k] = scale * sum_b part[b * K + k], one workgroup per k, fixed order.
__global__ __launch_bounds__(1024) void sum_columns_kernel(const double* __restrict__ part,
                                                           int64_t m, int K,
                                                           const double* __restrict__ scale,
                                                           double* __restrict__ out) {
    __shared__ double acc[1024];
    const int t = threadIdx.x, k = blockIdx.x;
    const int64_t per = (m + 1023) / 1024;
    double s = 0.0;
    for (int64_t q = t * per; q < m && q < (t + 1) * per; ++q) s += part[q * K + k];
    acc[t] = s;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (t < o) acc[t] += acc[t + o];
        __syncthreads();
    }
    if (t == 0) out[k] = *scale * acc[0];
}

// One backward sweep for row i:
//   z_i = (A x^s)_i, (A^T y)_i = sum over column i's entries (r, i) of a_ri y_r,
//   gval[e] -= omega <y_i, x_col e>,  gval[diag] += omega <y_i, z_i> / a_ii,
//   Gout_i = Gin_i - omega (A^T y)_i,  block partial of -<y_i, z_i>.
// With color (a colour phase's adjoint, y zero off colour c) the row part is
// skipped for rows of another colour (its terms are zero).
template <int K, int LPR>
__global__ __launch_bounds__(kBlock) void adjoint_sweep_kernel(
    int n, const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ av,
    const int64_t* __restrict__ cp, const int* __restrict__ trow, const int* __restrict__ tent,
    const double* __restrict__ diag, const double* __restrict__ Xs,
    const double* __restrict__ Y, const double* __restrict__ Gin, double* __restrict__ Gout,
    double omega, double* __restrict__ gval, double* __restrict__ wpart,
    const int* __restrict__ color, int c) {
    using S = Shape<double, K, LPR>;
    constexpr int V = S::V, C = S::C;
    __shared__ double part[kWavesPerBlock];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const int g = lane / LPR, l = lane % LPR;
    const int64_t i64 = ((int64_t)blockIdx.x * kWavesPerBlock + wv) * S::RPW + g;
    double wsum = 0.0;  // -<y_i, z_i> (lane 0 of the group)
    if (i64 < n) {
        const int i = (int)i64;
        const int e0 = rp[i], e1 = rp[i + 1];
        const Frag<double, V> yi = load_lane<double, V, C>(Y + (size_t)i * K + l * V);
        double z[V], aty[V];
#pragma unroll
        for (int q = 0; q < V; ++q) {
            z[q] = 0.0;
            aty[q] = 0.0;
        }
        int ediag = -1;
        const bool rows_part = !color || color[i] == c;
        for (int e = rows_part ? e0 : e1; e < e1; ++e) {
            const int j = ci[e];
            const double a = av[e];
            const Frag<double, V> xj = load_lane<double, V, C>(Xs + (size_t)j * K + l * V);
            double dot = 0.0;
#pragma unroll
            for (int q = 0; q < V; ++q) {
                z[q] = fma(a, xj.v[q], z[q]);
                dot = fma(yi.v[q], xj.v[q], dot);
            }
            dot = group_sum<LPR>(dot);
            if (j == i) ediag = e;
            if (l == 0) gval[e] -= omega * dot;
        }
        for (int64_t f = cp[i]; f < cp[i + 1]; ++f) {
            const int r = trow[f];
            const double at = av[tent[f]];
            const Frag<double, V> yr = load_lane<double, V, C>(Y + (size_t)r * K + l * V);
#pragma unroll
            for (int q = 0; q < V; ++q) aty[q] = fma(at, yr.v[q], aty[q]);
        }
        double yz = 0.0;
#pragma unroll
        for (int q = 0; q < V; ++q) yz = fma(yi.v[q], z[q], yz);
        yz = group_sum<LPR>(yz);
        const double d = diag[i];
        if (l == 0 && rows_part) {
            if (ediag >= 0 && d != 0.0) gval[ediag] += omega * yz / d;
            wsum = -yz;
        }
        Frag<double, V> gi = load_lane<double, V, C>(Gin + (size_t)i * K + l * V);
#pragma unroll
        for (int q = 0; q < V; ++q) gi.v[q] = fma(-omega, aty[q], gi.v[q]);
        store_lane<double, V, C>(Gout + (size_t)i * K + l * V, gi);
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) wsum += __shfl_xor(wsum, o, kWave);
    if (lane == 0) part[wv] = wsum;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int q = 0; q < kWavesPerBlock; ++q) s += part[q];
        wpart[blockIdx.x] = s;
    }
}

// Fixed-order sum of m partials into *out (one workgroup of 1024 threads).
__global__ __launch_bounds__(1024) void sum_partials_kernel(const double* __restrict__ part,
                                                            int64_t m, double* __restrict__ out) {
    __shared__ double acc[1024];
    const int t = threadIdx.x;
    const int64_t per = (m + 1023) / 1024;
    double s = 0.0;
    for (int64_t q = t * per; q < m && q < (t + 1) * per; ++q) s += part[q];
    acc[t] = s;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (t < o) acc[t] += acc[t + o];
        __syncthreads();
    }
    if (t == 0) *out = acc[0];
}

// The column-major index: cp[n+1] (column starts), trow/tent[nnz] (row and
// CSR position of each entry of a column, by increasing row); diag (if not
// null) the diagonal of the values av.  cnt: n ints, sc: the scan's
// workspace.
int launch_csc_index(int n, int64_t nnz, const int* rp, const int* ci, const double* av, int* cnt,
                     int64_t* cp, int64_t* sc, int* trow, int* tent, double* diag,
                     unsigned* status, hipStream_t s) {
    const int nblk_e = (int)((nnz + kBlock - 1) / kBlock);
    const int nblk_n = (int)(((int64_t)n + kBlock - 1) / kBlock);
    int rc;
    if ((rc = launch_fill_i32(cnt, n, 0, s))) return rc;
    col_count_kernel<<<dim3(nblk_e > 0 ? nblk_e : 1), dim3(kBlock), 0, s>>>(nnz, ci, cnt);
    AD_HIP(hipGetLastError());
    if ((rc = launch_excl_scan(cnt, n, cp, sc, s))) return rc;
    // the scan's workspace, free again, holds the asymmetry flag
    int* asym = (int*)sc;
    if ((rc = launch_fill_i32(asym, 1, 0, s))) return rc;
    col_fill_sym_kernel<<<dim3(nblk_n), dim3(kBlock), 0, s>>>(n, rp, ci, av, cp, trow, tent, diag,
                                                              asym, status);
    AD_HIP(hipGetLastError());
    // the general path (arrival order, then a sort per column) runs only
    // when the flag is set
    if ((rc = launch_fill_i32(cnt, n, 0, s))) return rc;
    col_fill_kernel<<<dim3(nblk_n), dim3(kBlock), 0, s>>>(n, rp, ci, av, cp, cnt, trow, tent, diag,
                                                          asym, status);
    col_sort_kernel<<<dim3(nblk_n), dim3(kBlock), 0, s>>>(n, cp, trow, tent, asym);
    AD_HIP(hipGetLastError());
    return AD_OK;
}

// Backward pass.  relax AD_JACOBI: damped-Jacobi sweeps (grad_omega).
// relax AD_MULTICOLOR_GS: colour-phase sweeps; each sweep's phase states are
// recomputed from its iterate and the phases' adjoints run in reverse colour
// order (omega is 1 and grad_omega, if given, is set to 0).  grad_w (may be
// null) receives dL/dw_k.
template <int K>
static int adjoint_go(ad_handle h, const ad_csr* A, int relax, const int32_t* color, int ncolors,
                      const void* ckpt, int ce, int sweeps, double omega, const double* w,
                      const uint8_t* cf, const int32_t* P_col, const double* P_val, int cal,
                      const void* X_final, const double* dL, double* grad_val,
                      double* grad_omega, double* grad_w, hipStream_t s) {
    constexpr int LPR = lpr_default<double>(K);
    using Sh = Shape<double, K, LPR>;
    const int n = A->n;
    const int64_t nnz = A->nnz;
    const size_t panel = (size_t)n * K * sizeof(double);
    const int rblocks = (int)(((int64_t)n + Sh::RPB - 1) / Sh::RPB);
    const int extra = ce - 1;  // recomputed iterates inside one checkpoint segment
    const bool gs = relax == AD_MULTICOLOR_GS;
    const int nph = gs ? ncolors : 0;  // phase states of one sweep (the first is its iterate)

    WsReq req;
    const size_t o_cnt = req.add(sizeof(int) * (size_t)n);
    const size_t o_cp = req.add(sizeof(int64_t) * ((size_t)n + 1));
    const size_t o_sc = req.add((size_t)scan_workspace_bytes(n));
    const size_t o_tr = req.add(sizeof(int) * (size_t)nnz);
    const size_t o_te = req.add(sizeof(int) * (size_t)nnz);
    const size_t o_dg = req.add(sizeof(double) * (size_t)n);
    const size_t o_g0 = req.add(panel);
    const size_t o_g1 = req.add(panel);
    const size_t o_y = req.add(panel);
    const size_t o_xr = req.add(panel * (size_t)(extra > 0 ? extra : 0));
    const size_t o_wp = req.add(sizeof(double) * (size_t)rblocks * (sweeps > 0 ? sweeps : 1));
    const size_t o_ph = req.add(panel * (size_t)(nph > 1 ? nph : 0));
    const size_t o_gw = req.add(grad_w ? sizeof(double) * (size_t)rblocks * K : 0);
    int rc = ws_reserve(h, req.off, s);
    if (rc) return rc;
    char* ws = (char*)h->ws;
    int* cnt = (int*)(ws + o_cnt);
    int64_t* cp = (int64_t*)(ws + o_cp);
    int64_t* sc = (int64_t*)(ws + o_sc);
    int* trow = (int*)(ws + o_tr);
    int* tent = (int*)(ws + o_te);
    double* diag = (double*)(ws + o_dg);
    double* G[2] = {(double*)(ws + o_g0), (double*)(ws + o_g1)};
    double* Y = (double*)(ws + o_y);
    double* Xr = (double*)(ws + o_xr);
    double* wp = (double*)(ws + o_wp);
    double* Ph = (double*)(ws + o_ph);
    double* gwp = (double*)(ws + o_gw);
    const double* av = (const double*)A->val;
    const size_t pe = (size_t)n * K;  // entries of one panel
    // one full sweep from xin to xout (GS: its phases through the phase
    // state buffers, which are free while iterates are recomputed)
    auto sweep = [&](const double* xin, double* xout) -> int {
        if (!gs) {
            LaunchCfg cfg;
            return launch_jacobi(AD_F64, K, A, xin, xout, omega, h->status, cfg, s);
        }
        const double* src = xin;
        for (int c = 0; c < ncolors; ++c) {
            double* dst = (c == ncolors - 1) ? xout : Ph + (size_t)(c % 2) * pe;
            gs_phase_nat_kernel<K, LPR><<<dim3(rblocks), dim3(kBlock), 0, s>>>(
                n, A->row_ptr, A->col, av, color, c, src, dst, h->status);
            src = dst;
        }
        AD_HIP(hipGetLastError());
        return AD_OK;
    };

    // column-major index of the pattern
    if ((rc = launch_csc_index(n, nnz, A->row_ptr, A->col, av, cnt, cp, sc, trow, tent, diag,
                               h->status, s)))
        return rc;
    if ((rc = launch_fill_f64(grad_val, nnz, 0.0, s))) return rc;
    // seed: R into Y (as scratch), then g into G[0]
    ls_residual_kernel<K, LPR><<<dim3(rblocks), dim3(kBlock), 0, s>>>(
        n, (const double*)X_final, w, cf, P_col, P_val, cal, dL, Y);
    ls_seed_kernel<K, LPR><<<dim3(rblocks), dim3(kBlock), 0, s>>>(n, cp, trow, cf, P_col, P_val,
                                                                   cal, Y, G[0]);
    AD_HIP(hipGetLastError());
    if (grad_w) {
        gradw_partials_kernel<K, LPR><<<dim3(rblocks), dim3(kBlock), 0, s>>>(
            n, (const double*)X_final, cf, P_col, P_val, cal, gwp);
        sum_columns_kernel<<<dim3(K), dim3(1024), 0, s>>>(gwp, rblocks, K, dL, grad_w);
        AD_HIP(hipGetLastError());
    }
    int cur = 0;
    const int nseg = (sweeps + ce - 1) / ce;
    for (int q = nseg - 1; q >= 0; --q) {
        const int s0 = q * ce;
        const int s1 = (s0 + ce < sweeps) ? s0 + ce : sweeps;  // segment sweeps s0 .. s1-1
        const double* xck = (const double*)((const char*)ckpt + (size_t)q * panel);
        // recompute x^{s0+1} .. x^{s1-1}
        for (int r = 1; r < s1 - s0; ++r) {
            const double* src = (r == 1) ? xck : Xr + (size_t)(r - 2) * pe;
            if ((rc = sweep(src, Xr + (size_t)(r - 1) * pe))) return rc;
        }
        for (int st = s1 - 1; st >= s0; --st) {
            const double* xs = (st == s0) ? xck : Xr + (size_t)(st - s0 - 1) * pe;
            if (!gs) {
                dinv_kernel<K, LPR><<<dim3(rblocks), dim3(kBlock), 0, s>>>(n, diag, G[cur], Y);
                adjoint_sweep_kernel<K, LPR><<<dim3(rblocks), dim3(kBlock), 0, s>>>(
                    n, A->row_ptr, A->col, av, cp, trow, tent, diag, xs, Y, G[cur], G[cur ^ 1],
                    omega, grad_val, wp + (size_t)st * rblocks, nullptr, 0);
                AD_HIP(hipGetLastError());
                cur ^= 1;
                continue;
            }
            // phase states: state c is the panel before phase c (state 0 = x^st)
            for (int c = 1; c < ncolors; ++c) {
                const double* src = (c == 1) ? xs : Ph + (size_t)(c - 2) * pe;
                gs_phase_nat_kernel<K, LPR><<<dim3(rblocks), dim3(kBlock), 0, s>>>(
                    n, A->row_ptr, A->col, av, color, c - 1, src, Ph + (size_t)(c - 1) * pe,
                    h->status);
            }
            for (int c = ncolors - 1; c >= 0; --c) {
                const double* v = (c == 0) ? xs : Ph + (size_t)(c - 1) * pe;
                dinv_colour_kernel<K, LPR><<<dim3(rblocks), dim3(kBlock), 0, s>>>(n, diag, color, c,
                                                                                 G[cur], Y);
                adjoint_sweep_kernel<K, LPR><<<dim3(rblocks), dim3(kBlock), 0, s>>>(
                    n, A->row_ptr, A->col, av, cp, trow, tent, diag, v, Y, G[cur], G[cur ^ 1],
                    1.0, grad_val, wp, color, c);
                cur ^= 1;
            }
            AD_HIP(hipGetLastError());
        }
    }
    if (grad_omega) {
        if (gs) {
            if ((rc = launch_fill_f64(grad_omega, 1, 0.0, s))) return rc;
        } else {
            sum_partials_kernel<<<dim3(1), dim3(1024), 0, s>>>(wp, (int64_t)rblocks * sweeps,
                                                               grad_omega);
            AD_HIP(hipGetLastError());
        }
    }
    return AD_OK;
}

int launch_ls_loss_backward(ad_handle h, int K, const ad_csr* A, int relax, const int32_t* color,
                            int ncolors, const void* ckpt, int ce, int sweeps, double omega,
                            const double* w, const uint8_t* cf, const int32_t* P_col,
                            const double* P_val, int cal, const void* X_final, const double* dL,
                            double* grad_val, double* grad_omega, double* grad_w, hipStream_t s) {
    switch (K) {
        case 2: return adjoint_go<2>(h, A, relax, color, ncolors, ckpt, ce, sweeps, omega, w, cf, P_col, P_val, cal, X_final, dL, grad_val, grad_omega, grad_w, s);
        case 4: return adjoint_go<4>(h, A, relax, color, ncolors, ckpt, ce, sweeps, omega, w, cf, P_col, P_val, cal, X_final, dL, grad_val, grad_omega, grad_w, s);
        case 8: return adjoint_go<8>(h, A, relax, color, ncolors, ckpt, ce, sweeps, omega, w, cf, P_col, P_val, cal, X_final, dL, grad_val, grad_omega, grad_w, s);
        case 16: return adjoint_go<16>(h, A, relax, color, ncolors, ckpt, ce, sweeps, omega, w, cf, P_col, P_val, cal, X_final, dL, grad_val, grad_omega, grad_w, s);
        case 32: return adjoint_go<32>(h, A, relax, color, ncolors, ckpt, ce, sweeps, omega, w, cf, P_col, P_val, cal, X_final, dL, grad_val, grad_omega, grad_w, s);
        case 64: return adjoint_go<64>(h, A, relax, color, ncolors, ckpt, ce, sweeps, omega, w, cf, P_col, P_val, cal, X_final, dL, grad_val, grad_omega, grad_w, s);
        default: return AD_EINVAL;
    }
}

}  // namespace ad
