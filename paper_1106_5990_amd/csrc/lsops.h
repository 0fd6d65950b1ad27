// lsops.h -- per-row pieces of the least-squares interpolation rows
// (Sec. 3.1, eq:LSfuncrowi / eq:modls), shared by the LS kernel and the
// fused distance + LS kernel so both compute bitwise the same rows.
//
// A row group of LPR lanes works on one F row; every lane of the group holds
// the same candidate list and the same reduced sums.
#pragma once

#include <math.h>

#include "device.h"

namespace ad {

// Insert candidate (m, j) into the sorted list of the `cal` least distances:
// after the equal ones, so that for columns visited in increasing order ties
// go to the lower column.  NaN distances are never chosen.
template <typename T, int CALT>
__device__ __forceinline__ void ls_insert(T (&smu)[CALT], int (&scol)[CALT], int& nsel, int cal,
                                          T m, int j) {
    if (m != m) return;
    int pos = 0;
#pragma unroll
    for (int q = 0; q < CALT; ++q)
        if (q < nsel && smu[q] <= m) pos = q + 1;
    if (pos >= cal) return;
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

// A C point interpolates itself.
__device__ __forceinline__ void ls_c_row(int64_t i, int cal, int* __restrict__ Pcol,
                                         double* __restrict__ Pval, double* __restrict__ lsv,
                                         int* __restrict__ rstat) {
    int* pc = Pcol + (size_t)i * cal;
    double* pv = Pval + (size_t)i * cal;
    pc[0] = (int)i;
    pv[0] = 1.0;
    for (int q = 1; q < cal; ++q) {
        pc[q] = -1;
        pv[q] = 0.0;
    }
    lsv[i] = 0.0;
    rstat[i] = 0;
}

// The LS row of F point i given its target t (FP64, this lane's V entries)
// and its sorted candidates scol[0 .. nsel): gathers the candidates' panel
// rows once, forms the FP64 normal equations
//     G_ab = sum_k w_k x_a^k x_b^k,  h_a = sum_k w_k x_a^k t^k
// reduced over the group, factors G by Cholesky in increasing-mu order
// (dropping a column whose pivot is <= 1e-12 of its Gram diagonal), solves,
// evaluates the functional at the minimiser from its definition, and writes
// the row (lane 0).  st: status so far (3 = zero diagonal on the residual
// target); returns the functional value.
template <typename T, int K, int LPR, int CALT, typename Src>
__device__ __forceinline__ double ls_solve(int i, int l, const double (&t)[K / LPR],
                                           const double (&wd)[K / LPR], const Src& src,
                                           const int (&scol)[CALT], int nsel, int st, int cal,
                                           int* __restrict__ Pcol, double* __restrict__ Pval,
                                           double* __restrict__ lsv, int* __restrict__ rstat) {
    using S = Shape<T, K, LPR>;
    constexpr int V = S::V, C = S::C;
    constexpr int NG = CALT * (CALT + 1) / 2;
    Frag<T, V> xs[CALT];
#pragma unroll
    for (int a = 0; a < CALT; ++a) {
        if (a < nsel) {
            xs[a] = load_lane<T, V, C>(src.row(scol[a]) + l * V);
        } else {
#pragma unroll
            for (int q = 0; q < V; ++q) xs[a].v[q] = T(0);
        }
    }
    double G[NG], hv[CALT], tt = 0.0;
#pragma unroll
    for (int q = 0; q < NG; ++q) G[q] = 0.0;
#pragma unroll
    for (int a = 0; a < CALT; ++a) hv[a] = 0.0;
#pragma unroll
    for (int q = 0; q < V; ++q) {
        const double wt = wd[q] * t[q];
        tt = fma(wt, t[q], tt);
        int gi = 0;
#pragma unroll
        for (int a = 0; a < CALT; ++a) {
            const double wx = wd[q] * (double)xs[a].v[q];
            hv[a] = fma(wx, t[q], hv[a]);
#pragma unroll
            for (int b = 0; b <= a; ++b, ++gi) G[gi] = fma(wx, (double)xs[b].v[q], G[gi]);
        }
    }
    if (nsel == 0) {
        tt = group_sum<LPR>(tt);
    } else {
#pragma unroll
        for (int q = 0; q < NG; ++q) G[q] = group_sum<LPR>(G[q]);
#pragma unroll
        for (int a = 0; a < CALT; ++a) hv[a] = group_sum<LPR>(hv[a]);
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
        val = tt;
        st = st ? st : 1;
    } else {
        // Cholesky (in place, packed lower) in increasing-mu order, drop
        // rule; the reciprocal of each kept pivot (1/sqrt of the pivot) is
        // formed once and the factor and both triangular solves multiply by it
        double rd[CALT];
#pragma unroll
        for (int a = 0; a < CALT; ++a) {
            rd[a] = 0.0;
            if (a >= nsel) continue;
            const int ra = a * (a + 1) / 2;
            const double gaa = G[ra + a];
#pragma unroll
            for (int b = 0; b < a; ++b) {
                const int rb = b * (b + 1) / 2;
                double s = G[ra + b];
#pragma unroll
                for (int c = 0; c < b; ++c)
                    if (keep[c]) s -= G[ra + c] * G[rb + c];
                G[ra + b] = keep[b] ? s * rd[b] : 0.0;
            }
            double piv = gaa;
#pragma unroll
            for (int b = 0; b < a; ++b)
                if (keep[b]) piv -= G[ra + b] * G[ra + b];
            keep[a] = piv > 1e-12 * gaa;
            if (keep[a]) {
                const double r = rsqrt_fp64(piv);
                G[ra + a] = piv * r;
                rd[a] = r;
            } else {
                G[ra + a] = 1.0;
                st = st ? st : 2;
            }
        }
        double z[CALT];
#pragma unroll
        for (int a = 0; a < CALT; ++a) {
            const int ra = a * (a + 1) / 2;
            double s = hv[a];
#pragma unroll
            for (int b = 0; b < a; ++b)
                if (keep[b]) s -= G[ra + b] * z[b];
            z[a] = keep[a] ? s * rd[a] : 0.0;
        }
#pragma unroll
        for (int a = CALT - 1; a >= 0; --a) {
            double s = z[a];
#pragma unroll
            for (int b = a + 1; b < CALT; ++b)
                if (keep[b]) s -= G[b * (b + 1) / 2 + a] * coef[b];
            coef[a] = keep[a] ? s * rd[a] : 0.0;
        }
        // the functional at the minimiser, by its definition
        double f = 0.0;
#pragma unroll
        for (int q = 0; q < V; ++q) {
            double r = t[q];
#pragma unroll
            for (int a = 0; a < CALT; ++a)
                if (keep[a]) r -= coef[a] * (double)opaque(xs[a].v[q]);
            f = fma(wd[q] * r, r, f);
        }
        val = group_sum<LPR>(f);
    }
    if (l == 0) {
        int* pc = Pcol + (size_t)i * cal;
        double* pv = Pval + (size_t)i * cal;
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
    }
    return val;
}

}  // namespace ad
