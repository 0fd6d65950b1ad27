// rowops.h -- per-row bodies shared by the single-matrix kernels and the
// batched kernels (so both compute bitwise the same values).
#pragma once

#include <math.h>

#include "device.h"

namespace ad {

// ---------------------------------------------------------------- row SpMM core
// y = sum_e a_e x_{col e} over the row's entries, in CSR order (FMA per term);
// also returns the diagonal value and the row's own fragment.
// pick(j) chooses which panel a neighbour is read from.
template <typename S, typename T, int K, typename Pick>
__device__ __forceinline__ void row_spmm(int i, int e0, int e1, const int* __restrict__ ci,
                                         const T* __restrict__ av, int l, Pick pick,
                                         T (&y)[S::V], T& d, Frag<T, S::V>& xi) {
    constexpr int V = S::V, C = S::C;
    constexpr int U = (V >= 16) ? 2 : 4;  // independent gathers in flight per step
#pragma unroll
    for (int q = 0; q < V; ++q) y[q] = T(0);
    d = T(0);
    int e = e0;
    for (; e + U <= e1; e += U) {
        int j[U];
        T a[U];
        Frag<T, V> x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            j[u] = ci[e + u];
            a[u] = av[e + u];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) x[u] = load_lane<T, V, C>(pick(j[u]) + (size_t)j[u] * K + l * V);
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int q = 0; q < V; ++q) y[q] = fma(a[u], x[u].v[q], y[q]);
            if (j[u] == i) {
                d = a[u];
                xi = x[u];
            }
        }
    }
    for (; e < e1; ++e) {
        const int j = ci[e];
        const T a = av[e];
        Frag<T, V> x = load_lane<T, V, C>(pick(j) + (size_t)j * K + l * V);
#pragma unroll
        for (int q = 0; q < V; ++q) y[q] = fma(a, x.v[q], y[q]);
        if (j == i) {
            d = a;
            xi = x;
        }
    }
}

// x_new_i = x_i - omega (A x)_i / a_ii for one row (held fixed if a_ii == 0).
template <typename S, typename T, int K>
__device__ __forceinline__ void jacobi_row(int i, int l, const int* __restrict__ rp,
                                           const int* __restrict__ ci, const T* __restrict__ av,
                                           const T* __restrict__ Xin, T* __restrict__ Xout,
                                           T omega, unsigned* status) {
    constexpr int V = S::V, C = S::C;
    T y[V], d;
    Frag<T, V> xi;
    row_spmm<S, T, K>(i, rp[i], rp[i + 1], ci, av, l, [&](int) { return Xin; }, y, d, xi);
    Frag<T, V> out;
    if (d == T(0)) {
        out = load_lane<T, V, C>(Xin + (size_t)i * K + l * V);
        if (l == 0) flag(status, AD_STAT_ZERO_DIAG);
    } else {
#pragma unroll
        for (int q = 0; q < V; ++q) out.v[q] = xi.v[q] - omega * y[q] / d;
    }
    store_lane<T, V, C>(Xout + (size_t)i * K + l * V, out);
}

template <typename T> struct Guard { static constexpr bool on = false; };
template <> struct Guard<float> { static constexpr bool on = true; };

// Distances mu_ij of one row (and, when strong != nullptr, its strength
// row): see distance.hip for the method.
// In FP32, p = S_ab / S_bb is formed with the hardware reciprocal: mu is
// stationary in p at the minimiser, so a one-ulp change of p moves mu only at
// second order.  WEIGHTED = false drops the w_k products (w == 1).
template <typename T>
__device__ __forceinline__ T ratio(T a, T b) {
    if constexpr (sizeof(T) == 4) return a * __builtin_amdgcn_rcpf(b);
    else return a / b;
}

template <typename S, typename T, int K, bool WEIGHTED>
__device__ __forceinline__ void algdist_row(int i, int l, const int* __restrict__ rp,
                                            const int* __restrict__ ci, const T* __restrict__ av,
                                            const T* __restrict__ X, const double (&wd)[S::V],
                                            const T (&wt)[S::V], bool plain, T* __restrict__ mu,
                                            double* __restrict__ pout, double theta,
                                            const uint8_t* __restrict__ fmask,
                                            uint8_t* __restrict__ strong, int* __restrict__ nstrong,
                                            unsigned* status) {
    constexpr int V = S::V, C = S::C, LPR = S::LPR;
    const bool fuse = strong != nullptr;
    const int e0 = rp[i], e1 = rp[i + 1];

    // target t_i; the residual form is built in FP64 (products of two
    // panel-type values are exact there), then rounded to the panel type
    // for the main pass; the FP64 copy feeds the guard-band recompute.
    Frag<T, V> t = load_lane<T, V, C>(X + (size_t)i * K + l * V);
    double t64[V];
#pragma unroll
    for (int q = 0; q < V; ++q) t64[q] = (double)t.v[q];
    if (!plain) {
        double y[V];
#pragma unroll
        for (int q = 0; q < V; ++q) y[q] = 0.0;
        double d = 0.0;
        for (int e = e0; e < e1; ++e) {
            const int j = ci[e];
            const double a = (double)av[e];
            Frag<T, V> xj = load_lane<T, V, C>(X + (size_t)j * K + l * V);
#pragma unroll
            for (int q = 0; q < V; ++q) y[q] = fma(a, (double)xj.v[q], y[q]);
            if (j == i) d = a;
        }
        if (d != 0.0) {
#pragma unroll
            for (int q = 0; q < V; ++q) {
                t64[q] = t64[q] - y[q] / d;
                t.v[q] = (T)t64[q];
            }
        } else if (l == 0) {
            flag(status, AD_STAT_ZERO_DIAG);
        }
    }
    T wtt[V];
    T saa = T(0);
#pragma unroll
    for (int q = 0; q < V; ++q) {
        wtt[q] = WEIGHTED ? wt[q] * t.v[q] : t.v[q];
        saa = fma(wtt[q], t.v[q], saa);
    }
    saa = group_sum<LPR>(saa);
    const T guard = (T)1e-4 * saa;

    const bool in_f = fmask ? (fmask[i] != 0) : true;
    T mmin = (T)INFINITY;
    bool bad = false;
    // U edges per step: their column and panel loads are issued together
    constexpr int U = (V >= 16) ? 2 : 4;
    for (int eb = e0; eb < e1; eb += U) {
        int jj[U];
        Frag<T, V> xs[U];
#pragma unroll
        for (int u = 0; u < U; ++u) jj[u] = (eb + u < e1) ? ci[eb + u] : i;
#pragma unroll
        for (int u = 0; u < U; ++u) xs[u] = load_lane<T, V, C>(X + (size_t)jj[u] * K + l * V);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = eb + u;
            if (e >= e1) break;
            const int j = jj[u];
            const Frag<T, V>& xj = xs[u];
            const bool mine = ((e - e0) & (LPR - 1)) == l;
            if (plain && j == i) {
                // x_i against itself: p = 1 and mu = 0 exactly
                if (mine) {
                    mu[e] = T(0);
                    if (pout) pout[e] = 1.0;
                }
                continue;
            }
            T sab = T(0), sbb = T(0);
#pragma unroll
            for (int q = 0; q < V; ++q) {
                sab = fma(wtt[q], xj.v[q], sab);
                sbb = fma(WEIGHTED ? wt[q] * xj.v[q] : xj.v[q], xj.v[q], sbb);
            }
            sab = group_sum<LPR>(sab);
            sbb = group_sum<LPR>(sbb);
            T p = (sbb > T(0)) ? ratio(sab, sbb) : T(0);
            T m = T(0);
#pragma unroll
            for (int q = 0; q < V; ++q) {
                const T r = fma(-p, xj.v[q], t.v[q]);
                m = fma(WEIGHTED ? wt[q] * r : r, r, m);
            }
            m = group_sum<LPR>(m);
            double pd = (double)p;
            if (Guard<T>::on && m < guard) {
                // FP64 recompute from the same FP32 inputs
                double a2 = 0.0, b2 = 0.0;
#pragma unroll
                for (int q = 0; q < V; ++q) {
                    const double xq = (double)xj.v[q], tq = t64[q];
                    a2 = fma(wd[q] * tq, xq, a2);
                    b2 = fma(wd[q] * xq, xq, b2);
                }
                a2 = group_sum<LPR>(a2);
                b2 = group_sum<LPR>(b2);
                pd = (b2 > 0.0) ? a2 / b2 : 0.0;
                double m2 = 0.0;
#pragma unroll
                for (int q = 0; q < V; ++q) {
                    const double r = t64[q] - pd * (double)xj.v[q];
                    m2 = fma(wd[q] * r, r, m2);
                }
                m = (T)group_sum<LPR>(m2);
            }
            bad |= !isfinite(m);
            if (mine) {
                mu[e] = m;
                if (pout) pout[e] = pd;
            }
            if (j != i && (!fmask || fmask[j])) mmin = (m < mmin) ? m : mmin;
        }
    }
    if (bad && l == 0) flag(status, AD_STAT_NONFINITE);

    if (fuse) {
        // second pass: each lane re-reads the mu values it stored
        int cnt = 0;
        const double md = (double)mmin;
        for (int e = e0 + l; e < e1; e += LPR) {
            const int j = ci[e];
            int s = 0;
            if (in_f && j != i && (!fmask || fmask[j])) {
                const double me = (double)mu[e];
                s = (md > 0.0) ? (theta * me < md) : (me == 0.0);
            }
            strong[e] = (uint8_t)s;
            cnt += s;
        }
        cnt = group_sum<LPR>(cnt);
        if (l == 0 && nstrong) nstrong[i] = cnt;
    }
}

}  // namespace ad
