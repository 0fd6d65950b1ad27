// rowops.h -- per-row bodies shared by the single-matrix kernels and the
// batched kernels (so both compute bitwise the same values).
#pragma once

#include <math.h>

#include <type_traits>

#include "device.h"

namespace ad {

// ---------------------------------------------------------------- row SpMM core
// y = sum_e a_e x_{col e} over the row's entries, in CSR order (FMA per term);
// also returns the diagonal value and the row's own fragment.
// ci_of(e) / av_of(e) give entry e's column and value (from global memory or
// from a wavefront's LDS copy); pick(j) chooses which panel a neighbour is
// read from.
template <typename S, typename T, int K, typename CiF, typename AvF, typename Pick>
__device__ __forceinline__ void row_spmm_acc(int i, int e0, int e1, CiF ci_of, AvF av_of, int l,
                                             Pick pick, T (&y)[S::V], T& d, Frag<T, S::V>& xi) {
    constexpr int V = S::V, C = S::C;
    // independent gathers in flight per step (measured: 3 beat 4 by 7% on
    // the colour phases and Jacobi sweeps of stencil rows and matched it on
    // graph rows of about 17 entries; 6 and 8 were slower)
    constexpr int U = (V >= 16) ? 2 : 3;
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
            j[u] = ci_of(e + u);
            a[u] = av_of(e + u);
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
        const int j = ci_of(e);
        const T a = av_of(e);
        Frag<T, V> x = load_lane<T, V, C>(pick(j) + (size_t)j * K + l * V);
#pragma unroll
        for (int q = 0; q < V; ++q) y[q] = fma(a, x.v[q], y[q]);
        if (j == i) {
            d = a;
            xi = x;
        }
    }
}

template <typename S, typename T, int K, typename Pick>
__device__ __forceinline__ void row_spmm(int i, int e0, int e1, const int* __restrict__ ci,
                                         const T* __restrict__ av, int l, Pick pick,
                                         T (&y)[S::V], T& d, Frag<T, S::V>& xi) {
    row_spmm_acc<S, T, K>(
        i, e0, e1, [&](int e) { return ci[e]; }, [&](int e) { return av[e]; }, l, pick, y, d, xi);
}

// ---------------------------------------------------------------- CSR staging
// The rows a wavefront works on are consecutive, so their entries form one
// contiguous range.  The wave copies that range (up to kStageCap entries)
// into its own LDS region with coalesced loads, and its row groups then read
// columns and values from LDS: the per-lane entry loads -- the same entry
// fetched by every lane of a row group -- leave the vector-memory address
// path to the panel gathers.  A row whose entries run past the staged range
// reads them from global memory.
constexpr int kStageCap = 512;  // entries per wavefront

template <typename T>
struct alignas(16) CsrStage {
    int ci[kWavesPerBlock][kStageCap];
    T av[kWavesPerBlock][kStageCap];
};

// orders this wavefront's LDS writes before its later LDS reads
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Copies the wave's entries [s0, s1) of (ci, av) into its region: entries
// [a0, a0 + cnt) with entry g at index g - a0, cnt <= kStageCap.  When both
// arrays are 16-byte aligned, a0 is s0 rounded down to a multiple of 4 and
// whole 4-entry chunks move as 16-byte loads and stores (the tail entry by
// entry); otherwise a0 = s0 and every entry is its own load.
template <typename T>
__device__ __forceinline__ void stage_csr(CsrStage<T>& L, int wv, int lane, int64_t s0,
                                          int64_t s1, const int* __restrict__ ci,
                                          const T* __restrict__ av, int64_t& a0, int& cnt) {
    const bool vec = (((uintptr_t)ci | (uintptr_t)av) & 15) == 0;  // launch-wide
    a0 = vec ? (s0 & ~(int64_t)3) : s0;
    const int64_t sc = s1 - a0;
    cnt = sc < kStageCap ? (int)sc : kStageCap;
    int q0 = 0;
    if (vec) {
        typedef int i4 __attribute__((ext_vector_type(4)));
        constexpr int E = 16 / (int)sizeof(T);
        typedef T tv __attribute__((ext_vector_type(E)));
        const int nch = cnt / 4;
        for (int c = lane; c < nch; c += kWave) {
            *(i4*)&L.ci[wv][4 * c] = *(const i4*)(ci + a0 + 4 * c);
#pragma unroll
            for (int h = 0; h < 4 / E; ++h)
                *(tv*)&L.av[wv][4 * c + h * E] = *(const tv*)(av + a0 + 4 * c + h * E);
        }
        q0 = 4 * nch;
    }
    for (int q = q0 + lane; q < cnt; q += kWave) {
        L.ci[wv][q] = ci[a0 + q];
        L.av[wv][q] = av[a0 + q];
    }
}

// row_spmm with the row's entries from the wave's staged copy when they lie
// inside it (s0: first staged entry, cnt: staged count), else from global.
template <typename S, typename T, int K, typename Pick>
__device__ __forceinline__ void row_spmm_staged(int i, int e0, int e1, const CsrStage<T>& L,
                                                int wv, int64_t s0, int cnt,
                                                const int* __restrict__ ci,
                                                const T* __restrict__ av, int l, Pick pick,
                                                T (&y)[S::V], T& d, Frag<T, S::V>& xi) {
    if ((int64_t)e1 - s0 <= cnt) {
        const int o = -(int)s0;  // LDS index of entry e is e + o
        row_spmm_acc<S, T, K>(
            i, e0, e1, [&](int e) { return L.ci[wv][e + o]; }, [&](int e) { return L.av[wv][e + o]; },
            l, pick, y, d, xi);
    } else {
        row_spmm<S, T, K>(i, e0, e1, ci, av, l, pick, y, d, xi);
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

// jacobi_row with the row's entries from the wave's staged copy
template <typename S, typename T, int K>
__device__ __forceinline__ void jacobi_row_staged(int i, int l, const int* __restrict__ rp,
                                                  const int* __restrict__ ci,
                                                  const T* __restrict__ av, const CsrStage<T>& L,
                                                  int wv, int64_t s0, int cnt,
                                                  const T* __restrict__ Xin, T* __restrict__ Xout,
                                                  T omega, unsigned* status) {
    constexpr int V = S::V, C = S::C;
    T y[V], d;
    Frag<T, V> xi;
    row_spmm_staged<S, T, K>(i, rp[i], rp[i + 1], L, wv, s0, cnt, ci, av, l,
                             [&](int) { return Xin; }, y, d, xi);
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

// The FP64 target entry carried as hi + lo (both panel type; lo is zero for
// FP64 panels, whose hi is the FP64 value itself).
template <typename T>
__device__ __forceinline__ double target64(T hi, T lo) {
    if constexpr (sizeof(T) == 8) return (double)opaque(hi);
    else return (double)opaque(hi) + (double)opaque(lo);
}

// Cooperative panel gather for one lane per row (LPR = 1) when a panel row
// is 32 or 64 bytes: G = 2 or 4 adjacent lanes (rows) load each of their G
// neighbour rows together -- lane s of the group reads the 16-byte piece s
// of every one of them, so each load instruction touches one cache line per
// lane group instead of one per lane -- and the pieces are handed to their
// owners through LDS.  G = 1: every lane loads its own rows.
template <typename T, int V, int LPR>
struct CoopGather {
    static constexpr int B = V * (int)sizeof(T);
    static constexpr int G = (LPR == 1 && (B == 32 || B == 64)) ? B / 16 : 1;
};

template <int G, int U, int k>
__device__ __forceinline__ void coop_bcast_cols(const int (&jj)[U], int (&jk)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) jk[u] = group_bcast<G, k>(jj[u]);
}

// Every lane of the aligned group of G lanes must be active.  LDS slot of
// piece p of the row of lane r: p * 64 + (r ^ p) (16-byte units), which keeps
// both the stores (fixed k) and the loads (fixed p) free of bank conflicts.
template <typename T, int K, int V, int U, int G>
__device__ __forceinline__ void coop_gather(const T* __restrict__ X, const int (&jj)[U],
                                            Frag<T, V> (&xs)[U]) {
    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    constexpr int CP = 16 / (int)sizeof(T);  // panel entries per piece
    static_assert(G * CP == V, "a lane's row is G pieces");
    __shared__ u32x4 buf[kWavesPerBlock][U][G * kWave];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int s = lane & (G - 1), base = lane & ~(G - 1);
    u32x4 pc[U][G];
    int jk[U];
    coop_bcast_cols<G, U, 0>(jj, jk);
#pragma unroll
    for (int u = 0; u < U; ++u) pc[u][0] = *(const u32x4*)(X + (size_t)jk[u] * K + s * CP);
    coop_bcast_cols<G, U, 1>(jj, jk);
#pragma unroll
    for (int u = 0; u < U; ++u) pc[u][1] = *(const u32x4*)(X + (size_t)jk[u] * K + s * CP);
    if constexpr (G == 4) {
        coop_bcast_cols<G, U, 2>(jj, jk);
#pragma unroll
        for (int u = 0; u < U; ++u) pc[u][2] = *(const u32x4*)(X + (size_t)jk[u] * K + s * CP);
        coop_bcast_cols<G, U, 3>(jj, jk);
#pragma unroll
        for (int u = 0; u < U; ++u) pc[u][3] = *(const u32x4*)(X + (size_t)jk[u] * K + s * CP);
    }
    wave_lds_sync();  // the previous step's reads of the slots are done
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int k = 0; k < G; ++k) buf[wv][u][s * kWave + ((base + k) ^ s)] = pc[u][k];
    wave_lds_sync();
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int p = 0; p < G; ++p) {
            const u32x4 w = buf[wv][u][p * kWave + (lane ^ p)];
            typedef T tvec __attribute__((ext_vector_type(CP)));
            const tvec v = __builtin_bit_cast(tvec, w);
#pragma unroll
            for (int q = 0; q < CP; ++q) xs[u].v[p * CP + q] = v[q];
        }
}

// Entries per step of the row-group distance loop when a lane holds under
// 64 bytes of a panel row and loads its rows itself: 3 for matrices of fewer
// than 16 stored entries per row on average, 4 for longer rows (measured: 3
// fills the steps of 9-entry stencil rows exactly, 2 leaves more latency
// exposed and 5 or more cost occupancy; rows of about 17 entries ran best
// with 4).  f(std::integral_constant<int, UN>) is called with the choice;
// shapes where it does not matter get 3 only.
template <typename T, int K, int LPR, typename F>
void dist_unroll(bool long_rows, F&& f) {
    constexpr int V = K / LPR;
    if constexpr (V < 16 && CoopGather<T, V, LPR>::G == 1) {
        if (long_rows) f(std::integral_constant<int, 4>{});
        else f(std::integral_constant<int, 3>{});
    } else {
        f(std::integral_constant<int, 3>{});
    }
}

// ---------------------------------------------------------------- panel row source
// Where the distance and LS row bodies read panel rows from: the panel in
// global memory (gathers through the caches).
template <typename T, int K>
struct GlobalRows {
    const T* __restrict__ X;
    static constexpr bool kCoop = true;  // the cooperative gather may be used
    __device__ __forceinline__ const T* row(int j) const { return X + (size_t)j * K; }
};

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

// sel(j, mu_ij) is called for every off-diagonal entry in CSR order with
// the group-uniform distance (the fused LS kernel picks its C-neighbours
// there); tout receives the FP64 target and dout the diagonal value (0 when
// absent; only looked for with the residual target).  A ghost row (a lane
// past the end of the rows, i clamped to a valid row) has no entries and
// writes nothing, but takes its part in the cooperative panel loads.
// The distances run over the entries of (rp, ci); the residual target is
// formed from the rows of (rpt, cit, av) -- the matrix itself, also when
// (rp, ci) is another pattern such as that of A^d.
template <typename S, typename T, int K, bool WEIGHTED, int UN, typename Src, typename Sel>
__device__ __forceinline__ void algdist_row_sel(int i, bool ghost, int l,
                                                const int* __restrict__ rp,
                                                const int* __restrict__ ci,
                                                const int* __restrict__ rpt,
                                                const int* __restrict__ cit,
                                                const T* __restrict__ av, const Src& src,
                                                const double (&wd)[S::V], const T (&wt)[S::V],
                                                bool plain, T* __restrict__ mu,
                                                double* __restrict__ pout, double theta,
                                                const uint8_t* __restrict__ fmask,
                                                uint8_t* __restrict__ strong,
                                                int* __restrict__ nstrong, unsigned* status,
                                                Sel&& sel, double (&tout)[S::V], double& dout) {
    constexpr int V = S::V, C = S::C, LPR = S::LPR;
    const bool fuse = strong != nullptr;
    const int e0 = rp[i], e1 = ghost ? e0 : rp[i + 1];

    // target t_i; the residual form is built in FP64 (products of two
    // panel-type values are exact there), then rounded to the panel type
    // for the main pass.  The FP64 target that feeds the guard-band
    // recompute and tout is carried as t + tlo, tlo the panel-type rounding
    // of the remainder (zero for the plain target and for FP64 panels):
    // exact where tlo is zero, within 2^-48 relative otherwise.  It is
    // re-formed at each use so that no FP64 copy stays live through the
    // entry loop.
    Frag<T, V> t = load_lane<T, V, C>(src.row(i) + l * V);
    T tlo[V];
#pragma unroll
    for (int q = 0; q < V; ++q) tlo[q] = T(0);
    if (!plain) {
        double y[V];
#pragma unroll
        for (int q = 0; q < V; ++q) y[q] = 0.0;
        double d = 0.0;
        const int f0 = rpt[i], f1 = ghost ? f0 : rpt[i + 1];
        for (int e = f0; e < f1; ++e) {
            const int j = cit[e];
            const double a = (double)av[e];
            Frag<T, V> xj = load_lane<T, V, C>(src.row(j) + l * V);
#pragma unroll
            for (int q = 0; q < V; ++q) y[q] = fma(a, (double)xj.v[q], y[q]);
            if (j == i) d = a;
        }
        if (d != 0.0) {
#pragma unroll
            for (int q = 0; q < V; ++q) {
                const double t64 = (double)t.v[q] - y[q] / d;
                t.v[q] = (T)t64;
                if constexpr (sizeof(T) == 4) tlo[q] = (T)(t64 - (double)t.v[q]);
            }
        } else if (l == 0 && !ghost) {
            flag(status, AD_STAT_ZERO_DIAG);
        }
        dout = d;
    } else {
        dout = 0.0;
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
    // (UN, see dist_unroll, for lanes holding under 64 bytes of a row)
    constexpr int G = Src::kCoop ? CoopGather<T, V, LPR>::G : 1;
    constexpr int U = (G > 1) ? 8 / G : (V >= 16) ? 2 : UN;
    // the next step's column indices are loaded while this step's panel
    // rows are in flight
    int jn[U];
#pragma unroll
    for (int u = 0; u < U; ++u) jn[u] = (e0 + u < e1) ? ci[e0 + u] : i;
    // with the cooperative gather the G rows of a lane group step together
    int nsteps = 0;
    if constexpr (G > 1) nsteps = group_max<G>((e1 - e0 + U - 1) / U);
    for (int eb = e0, st = 0; (G > 1) ? (st < nsteps) : (eb < e1); eb += U, ++st) {
        int jj[U];
        Frag<T, V> xs[U];
#pragma unroll
        for (int u = 0; u < U; ++u) jj[u] = jn[u];
        if constexpr (G > 1) {
            coop_gather<T, K, V, U, G>(src.X, jj, xs);
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) xs[u] = load_lane<T, V, C>(src.row(jj[u]) + l * V);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) jn[u] = (eb + U + u < e1) ? ci[eb + U + u] : i;
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
                    const double xq = (double)xj.v[q], tq = target64(t.v[q], tlo[q]);
                    a2 = fma(wd[q] * tq, xq, a2);
                    b2 = fma(wd[q] * xq, xq, b2);
                }
                a2 = group_sum<LPR>(a2);
                b2 = group_sum<LPR>(b2);
                pd = (b2 > 0.0) ? a2 / b2 : 0.0;
                double m2 = 0.0;
#pragma unroll
                for (int q = 0; q < V; ++q) {
                    const double r = target64(t.v[q], tlo[q]) - pd * (double)xj.v[q];
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
            if (j != i) sel(j, m);
        }
    }
    if (bad && l == 0) flag(status, AD_STAT_NONFINITE);
#pragma unroll
    for (int q = 0; q < V; ++q) tout[q] = (double)t.v[q] + (double)tlo[q];

    if (fuse) {
        // second pass: each lane re-reads the mu values it stored, SB
        // entries' loads in flight together
        int cnt = 0;
        const double md = (double)mmin;
        constexpr int SB = 8;
        for (int eb = e0 + l; eb < e1; eb += SB * LPR) {
            int jj[SB];
            T mm[SB];
            bool fj[SB];
#pragma unroll
            for (int u = 0; u < SB; ++u) {
                const int e = eb + u * LPR;
                jj[u] = (e < e1) ? ci[e] : i;
                mm[u] = (e < e1) ? mu[e] : T(0);
            }
#pragma unroll
            for (int u = 0; u < SB; ++u) fj[u] = !fmask || fmask[jj[u]];
#pragma unroll
            for (int u = 0; u < SB; ++u) {
                const int e = eb + u * LPR;
                if (e >= e1) break;
                int s = 0;
                if (in_f && jj[u] != i && fj[u]) {
                    const double me = (double)mm[u];
                    s = (md > 0.0) ? (theta * me < md) : (me == 0.0);
                }
                strong[e] = (uint8_t)s;
                cnt += s;
            }
        }
        cnt = group_sum<LPR>(cnt);
        if (l == 0 && nstrong && !ghost) nstrong[i] = cnt;
    }
}

template <typename S, typename T, int K, bool WEIGHTED, int UN>
__device__ __forceinline__ void algdist_row(int i, bool ghost, int l, const int* __restrict__ rp,
                                            const int* __restrict__ ci, const int* __restrict__ rpt,
                                            const int* __restrict__ cit, const T* __restrict__ av,
                                            const T* __restrict__ X, const double (&wd)[S::V],
                                            const T (&wt)[S::V], bool plain, T* __restrict__ mu,
                                            double* __restrict__ pout, double theta,
                                            const uint8_t* __restrict__ fmask,
                                            uint8_t* __restrict__ strong, int* __restrict__ nstrong,
                                            unsigned* status) {
    double t64[S::V], d;
    algdist_row_sel<S, T, K, WEIGHTED, UN>(i, ghost, l, rp, ci, rpt, cit, av, GlobalRows<T, K>{X}, wd, wt, plain, mu, pout,
                                           theta, fmask, strong, nstrong, status, [](int, T) {},
                                           t64, d);
}

// ---------------------------------------------------------------- edge-parallel distances
// Plain target only.  One wavefront takes up to kEdgeRows consecutive rows
// [r0, r0 + rl) and walks their stored entries kWave at a time, one entry
// per lane.  The lane gathers x_i and x_j whole (K values each; lanes of one
// row read the same x_i addresses), so S_ab, S_bb, p and mu need no
// cross-lane reduction, and mu is stored contiguously; the next chunk's
// column indices are loaded one chunk ahead.  With the strength row wanted,
// each mu is folded into its row's minimum in LDS (the bit patterns of
// non-negative floats order like unsigned integers) and the first kEdgeKeep
// chunks keep (j, mu) in LDS; a second walk writes the mask and, through LDS
// counters, the counts.
// All threads of the workgroup call it (it holds workgroup barriers); LDS
// regions are per wavefront.
// Per entry the arithmetic is that of algdist_row with one lane per row:
// the sums over k run in index order in the panel type, p in FP32 via the
// hardware reciprocal, the FP64 recompute below 1e-4 S_aa.
constexpr int kEdgeRows = 32;  // measured: 2-3% faster than 64 on graph rows of ~17 entries

// panel rows up to this many bytes use the edge-parallel kernel by default
constexpr int kEdgeMaxRowBytes = 128;

template <typename T>
using OrdBits = typename std::conditional<sizeof(T) == 4, unsigned, unsigned long long>::type;

__device__ __forceinline__ unsigned ord_bits(float m) { return __float_as_uint(m + 0.0f); }
__device__ __forceinline__ unsigned long long ord_bits(double m) {
    return (unsigned long long)__double_as_longlong(m + 0.0);
}
__device__ __forceinline__ float from_ord(unsigned b) { return __uint_as_float(b); }
__device__ __forceinline__ double from_ord(unsigned long long b) {
    return __longlong_as_double((long long)b);
}

// chunks of kWave entries whose (j, mu) stay in LDS for the strength walk
constexpr int kEdgeKeep = 12;

template <typename T>
struct EdgeLds {
    int rp[kWavesPerBlock][kEdgeRows + 1];
    OrdBits<T> mn[kWavesPerBlock][kEdgeRows];
    int cnt[kWavesPerBlock][kEdgeRows];
    T aa[kWavesPerBlock][kEdgeRows];  // S_aa of each row, formed once per row
    T m[kWavesPerBlock][kEdgeKeep][kWave];
    int j[kWavesPerBlock][kEdgeKeep][kWave];
};

// last row of the wave's block whose first entry is <= q, searching [lo, rl)
__device__ __forceinline__ int edge_row(const int* __restrict__ starts, int lo, int rl, int q) {
    int hi = rl - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (starts[mid] <= q) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <typename T, int K, bool WEIGHTED, bool LEAN>
__device__ __forceinline__ void algdist_edge_rows(
    int r0, int rl, const int* __restrict__ rp, const int* __restrict__ ci,
    const T* __restrict__ X, const double* __restrict__ w, T* __restrict__ mu,
    double* __restrict__ pout, double theta, const uint8_t* __restrict__ fmask,
    uint8_t* __restrict__ strong, int* __restrict__ nstrong, EdgeLds<T>& L, unsigned* status) {
    constexpr int C = (K * (int)sizeof(T) <= 16) ? K : 16 / (int)sizeof(T);
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const bool fuse = strong != nullptr;
    int* starts = L.rp[wv];
    if (lane < rl) {
        starts[lane] = rp[r0 + lane];
        L.mn[wv][lane] = ord_bits((T)INFINITY);
        L.cnt[wv][lane] = 0;
        // S_aa of the row, in the order the per-entry loop would form it
        const Frag<T, K> t = load_lane<T, K, C>(X + (size_t)(r0 + lane) * K);
        T saa = T(0);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const T wtk = WEIGHTED ? (T)w[k] * t.v[k] : t.v[k];
            saa = fma(wtk, t.v[k], saa);
        }
        L.aa[wv][lane] = saa;
    }
    if (lane == 0 && rl > 0) starts[rl] = rp[r0 + rl];
    __syncthreads();
    const int b = rl > 0 ? starts[0] : 0, e = rl > 0 ? starts[rl] : 0;
    bool bad = false;
    int row = 0;
    // the next chunk's column index is loaded one chunk ahead
    int jn = (b + lane < e) ? ci[b + lane] : 0;
    for (int q = b + lane, c = 0; q < e; q += kWave, ++c) {
        row = edge_row(starts, row, rl, q);
        const int i = r0 + row;
        const int j = jn;
        jn = (q + kWave < e) ? ci[q + kWave] : 0;
        T m;
        double pd;
        if (j == i) {  // x_i against itself: p = 1 and mu = 0 exactly
            m = T(0);
            pd = 1.0;
        } else {
            const Frag<T, K> t = load_lane<T, K, C>(X + (size_t)i * K);
            const Frag<T, K> x = load_lane<T, K, C>(X + (size_t)j * K);
            T sab = T(0), sbb = T(0);
            const T saa = L.aa[wv][row];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const T wk = WEIGHTED ? (T)w[k] : T(1);
                const T wtk = WEIGHTED ? wk * t.v[k] : t.v[k];
                sab = fma(wtk, x.v[k], sab);
                sbb = fma(WEIGHTED ? wk * x.v[k] : x.v[k], x.v[k], sbb);
            }
            const T p = (sbb > T(0)) ? ratio(sab, sbb) : T(0);
            m = T(0);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const T r = fma(-p, x.v[k], t.v[k]);
                m = fma(WEIGHTED ? (T)w[k] * r : r, r, m);
            }
            pd = (double)p;
            if (Guard<T>::on && m < (T)1e-4 * saa) {
                // FP64 recompute from the same FP32 inputs
                double a2 = 0.0, b2 = 0.0;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const double wk = WEIGHTED ? w[k] : 1.0;
                    const double xq = (double)x.v[k], tq = (double)t.v[k];
                    a2 = fma(wk * tq, xq, a2);
                    b2 = fma(wk * xq, xq, b2);
                }
                pd = (b2 > 0.0) ? a2 / b2 : 0.0;
                double m2 = 0.0;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const double wk = WEIGHTED ? w[k] : 1.0;
                    const double r = (double)t.v[k] - pd * (double)x.v[k];
                    m2 = fma(wk * r, r, m2);
                }
                m = (T)m2;
            }
            bad |= !isfinite(m);
        }
        mu[q] = m;
        if (!LEAN && pout) pout[q] = pd;
        if (fuse) {
            if (c < kEdgeKeep) {
                L.m[wv][c][lane] = m;
                L.j[wv][c][lane] = j;
            }
            if (j != i && (LEAN || !fmask || fmask[j])) atomicMin(&L.mn[wv][row], ord_bits(m));
        }
    }
    if (bad) flag(status, AD_STAT_NONFINITE);
    if (!fuse) return;
    __syncthreads();
    row = 0;
    for (int q = b + lane, c = 0; q < e; q += kWave, ++c) {
        row = edge_row(starts, row, rl, q);
        const int i = r0 + row;
        const bool kept = c < kEdgeKeep;
        const int j = kept ? L.j[wv][c][lane] : ci[q];
        int st = 0;
        if ((LEAN || !fmask || (fmask[i] && fmask[j])) && j != i) {
            const double md = (double)from_ord(L.mn[wv][row]);
            const double me = (double)(kept ? L.m[wv][c][lane] : mu[q]);  // own store
            st = (md > 0.0) ? (theta * me < md) : (me == 0.0);
        }
        strong[q] = (uint8_t)st;
        if (st) atomicAdd(&L.cnt[wv][row], 1);
    }
    __syncthreads();
    if (lane < rl && nstrong) nstrong[r0 + lane] = L.cnt[wv][lane];
}

}  // namespace ad
