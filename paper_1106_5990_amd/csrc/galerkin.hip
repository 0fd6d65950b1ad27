// galerkin.hip -- the Galerkin coarse operator A_c = P^T A P and the
// two-grid method used to judge a coarse space (Sec. 5.2).
//
// Interpolation P (n x nc) is given by rows: fine row i holds P_val[i][q] in
// the column of the C point P_col[i][q] (fine index; -1 pads), the C points
// numbered in increasing fine index (cidx, an exclusive scan of cf).
//
// A_c row by row, one wavefront per coarse row I: the fine rows i with
// p_iI != 0 (the transpose of P, sorted by (i, q)), row i's entries of A in
// CSR order, row j's weights in stored order -- every product
// (p_iI * a_ij) * p_jJ gets a sequence number in that nested order and is
// written to LDS with the key (J, sequence).  A bitonic sort by key groups
// the products of each J in generation order, and each group is summed left
// to right.  Products and sums are rounded one by one (no contraction), so
// every coefficient is formed exactly as the plain Gustavson loop forms it.
// A first pass counts the distinct J of each row (the row pointers), a
// second writes them.
//
// Two-grid method (homogeneous system, K error vectors at once): pre
// colour-phase sweeps (the setup's smoother), r = -A e, r_c = P^T r, A_c e_c
// = r_c by dense Cholesky (the factor and its inverse once, row by row with
// wavefront dot products; per cycle two dense triangular products), e +=
// P e_c, post sweeps; ||e||_A per vector after every cycle.
#include <math.h>

#include <climits>
#include <vector>

#include "device.h"
#include "internal.h"
#include "rowops.h"

namespace ad {

constexpr int kGalCap = 2048;  // products of one coarse row (LDS)
constexpr int kGalT = 64;      // P^T entries of one coarse row
constexpr int kGalWave = 64;

__global__ __launch_bounds__(kBlock) void cf_flags_kernel(int n, const uint8_t* __restrict__ cf,
                                                          int* __restrict__ f) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) f[i] = cf[i] != 0;
}

__global__ __launch_bounds__(kBlock) void cidx_kernel(int n, const uint8_t* __restrict__ cf,
                                                      const int64_t* __restrict__ scan,
                                                      int* __restrict__ cidx) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) cidx[i] = cf[i] ? (int)scan[i] : -1;
}

// cnt[I] = entries of column I of P; bad set for a column naming a non-C point
__global__ __launch_bounds__(kBlock) void pt_count_kernel(int n, int cal, const int* __restrict__ Pc,
                                                          const int* __restrict__ cidx,
                                                          int* __restrict__ cnt, unsigned* status) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    for (int q = 0; q < cal; ++q) {
        const int c = Pc[i * cal + q];
        if (c < 0) continue;
        const int I = c < n ? cidx[c] : -1;
        if (I < 0) {
            flag(status, AD_STAT_BAD_INTERP);
            continue;
        }
        atomicAdd(&cnt[I], 1);
    }
}

__global__ __launch_bounds__(kBlock) void pt_fill_kernel(int n, int cal, const int* __restrict__ Pc,
                                                         const int* __restrict__ cidx,
                                                         const int64_t* __restrict__ pt,
                                                         int* __restrict__ cur,
                                                         int64_t* __restrict__ key) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    for (int q = 0; q < cal; ++q) {
        const int c = Pc[i * cal + q];
        if (c < 0 || c >= n) continue;
        const int I = cidx[c];
        if (I < 0) continue;
        key[pt[I] + atomicAdd(&cur[I], 1)] = i * cal + q;
    }
}

// each column's keys (i * cal + q) ascending: by fine row, then stored slot
__global__ __launch_bounds__(kBlock) void pt_sort_kernel(int nc, const int64_t* __restrict__ pt,
                                                         int64_t* __restrict__ key) {
    const int64_t I = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (I >= nc) return;
    const int64_t a = pt[I], b = pt[I + 1];
    for (int64_t f = a + 1; f < b; ++f) {
        const int64_t k = key[f];
        int64_t g = f - 1;
        while (g >= a && key[g] > k) {
            key[g + 1] = key[g];
            --g;
        }
        key[g + 1] = k;
    }
}

// products of row I: P^T entries times the A rows they name, times cal
__global__ __launch_bounds__(kBlock) void gal_slots_kernel(int nc, const int* __restrict__ rp,
                                                           int cal, const int64_t* __restrict__ pt,
                                                           const int64_t* __restrict__ key,
                                                           int* __restrict__ maxslots) {
    const int64_t I = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (I >= nc) return;
    const int64_t a = pt[I], b = pt[I + 1];
    int64_t s = 0;
    for (int64_t f = a; f < b; ++f) {
        const int64_t i = key[f] / cal;
        s += rp[i + 1] - rp[i];
    }
    s *= cal;
    const int64_t nt = b - a;
    const int v = (nt > kGalT || s > kGalCap) ? INT_MAX : (int)s;
    atomicMax(maxslots, v);
}

// Coarse rows by product keys and a sort, one row at a time per workgroup
// of one wavefront: the rows the lane kernel below could not hold.  count
// pass: cnt[I] = distinct columns; fill pass (rpc given): colc / valc.
struct GalRowLds {
    int64_t key[kGalCap];
    double val[kGalCap];
    int s_i[kGalT];
    double s_p[kGalT];
    int s_base[kGalT + 1];
};

template <typename TA>
__device__ void galerkin_row_wave(int I, GalRowLds& L, int n, const int* __restrict__ rp,
                                  const int* __restrict__ ci, const TA* __restrict__ av, int cal,
                                  const int* __restrict__ Pc, const double* __restrict__ Pv,
                                  const int* __restrict__ cidx, const int64_t* __restrict__ pt,
                                  const int64_t* __restrict__ ptkey, const int* __restrict__ rpc,
                                  int* __restrict__ cnt, int* __restrict__ colc,
                                  double* __restrict__ valc) {
    int64_t* key = L.key;
    double* val = L.val;
    int* s_i = L.s_i;
    double* s_p = L.s_p;
    int* s_base = L.s_base;
    const int lane = threadIdx.x;
    const int64_t t0 = pt[I];
    const int nt = (int)(pt[I + 1] - t0);  // <= kGalT (checked on the host)
    int len = 0;
    if (lane < nt) {
        const int64_t k = ptkey[t0 + lane];
        const int i = (int)(k / cal), q = (int)(k % cal);
        s_i[lane] = i;
        s_p[lane] = Pv[k];
        (void)q;
        len = rp[i + 1] - rp[i];
    }
    // exclusive scan of the row lengths over the P^T entries
    int incl = len;
#pragma unroll
    for (int o = 1; o < kGalWave; o <<= 1) {
        const int y = __shfl_up(incl, o, kGalWave);
        if (lane >= o) incl += y;
    }
    if (lane < nt) s_base[lane] = incl - len;
    const int npairs = __shfl(incl, kGalWave - 1, kGalWave);
    if (lane == 0) s_base[nt] = npairs;
    __syncthreads();
    const int nslot = npairs * cal;  // <= kGalCap (checked on the host)
    int m2 = 1;
    while (m2 < nslot) m2 <<= 1;
    for (int s = lane; s < m2; s += kGalWave) key[s] = LLONG_MAX;
    __syncthreads();
    for (int k = lane; k < npairs; k += kGalWave) {
        int lo = 0, hi = nt;  // last t with s_base[t] <= k
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (s_base[mid] <= k) lo = mid;
            else hi = mid;
        }
        const int i = s_i[lo];
        const int e = rp[i] + (k - s_base[lo]);
        const int j = ci[e];
        const double pa = __dmul_rn(s_p[lo], (double)av[e]);
        for (int q = 0; q < cal; ++q) {
            const int c = Pc[(int64_t)j * cal + q];
            const int slot = k * cal + q;
            if (c < 0 || c >= n || cidx[c] < 0) continue;
            key[slot] = ((int64_t)cidx[c] << 32) | (int64_t)slot;
            val[slot] = __dmul_rn(pa, Pv[(int64_t)j * cal + q]);
        }
    }
    __syncthreads();
    // bitonic sort of (key, val) ascending
    for (int size = 2; size <= m2; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int x = lane; x < m2; x += kGalWave) {
                const int y = x ^ stride;
                if (y > x) {
                    const bool up = (x & size) == 0;
                    const int64_t kx = key[x], ky = key[y];
                    if ((kx > ky) == up) {
                        key[x] = ky;
                        key[y] = kx;
                        const double v = val[x];
                        val[x] = val[y];
                        val[y] = v;
                    }
                }
            }
            __syncthreads();
        }
    // run starts: a valid key whose column differs from the previous one's
    const int per = (m2 + kGalWave - 1) / kGalWave;
    const int c0 = lane * per, c1 = (c0 + per < m2) ? c0 + per : m2;
    int starts = 0;
    for (int x = c0; x < c1; ++x) {
        const int64_t k = key[x];
        if (k == LLONG_MAX) break;
        if (x == 0 || (key[x - 1] >> 32) != (k >> 32)) ++starts;
    }
    int sincl = starts;
#pragma unroll
    for (int o = 1; o < kGalWave; o <<= 1) {
        const int y = __shfl_up(sincl, o, kGalWave);
        if (lane >= o) sincl += y;
    }
    if (!rpc) {
        if (lane == kGalWave - 1) cnt[I] = sincl;
        __syncthreads();  // LDS is reused by the workgroup's next row
        return;
    }
    int rank = sincl - starts;
    const int64_t out0 = rpc[I];
    for (int x = c0; x < c1; ++x) {
        const int64_t k = key[x];
        if (k == LLONG_MAX) break;
        const int64_t J = k >> 32;
        if (x > 0 && (key[x - 1] >> 32) == J) continue;
        double acc = val[x];
        for (int y = x + 1; y < m2 && key[y] != LLONG_MAX && (key[y] >> 32) == J; ++y)
            acc = __dadd_rn(acc, val[y]);
        colc[out0 + rank] = (int)J;
        valc[out0 + rank] = acc;
        ++rank;
    }
    __syncthreads();  // LDS is reused by the workgroup's next row
}

template <typename TA>
__global__ __launch_bounds__(kGalWave) void galerkin_row_kernel(
    int n, const int* __restrict__ rp, const int* __restrict__ ci, const TA* __restrict__ av,
    int cal, const int* __restrict__ Pc, const double* __restrict__ Pv,
    const int* __restrict__ cidx, const int64_t* __restrict__ pt,
    const int64_t* __restrict__ ptkey, const int* __restrict__ rpc, int* __restrict__ cnt,
    int* __restrict__ colc, double* __restrict__ valc, const int* __restrict__ rows,
    const int* __restrict__ nrows) {
    __shared__ GalRowLds L;
    const int m = *nrows;
    for (int x = blockIdx.x; x < m; x += gridDim.x)
        galerkin_row_wave<TA>(rows[x], L, n, rp, ci, av, cal, Pc, Pv, cidx, pt, ptkey, rpc, cnt,
                              colc, valc);
}

// One coarse row per lane: the row's products in the order the expansion
// generates them (P^T entries by (i, slot), then row i of A, then row j's
// slots), each added into the lane's LDS map of distinct coarse columns,
// kept sorted by column (binary search, insertion by shifting).  Products
// and sums are explicitly rounded, so each coefficient is the same sum as
// the sort kernel's.  A row with more than kGalMap distinct columns is
// appended to the spill list (in no particular order) and left to the sort
// kernel.  count pass (FILL false): cnt[I]; fill pass: colc / valc.
constexpr int kGalMap = 32;

template <typename TA, bool FILL>
__global__ __launch_bounds__(kWave) void galerkin_lane_kernel(
    int n, int nc, const int* __restrict__ rp, const int* __restrict__ ci,
    const TA* __restrict__ av, int cal, const int* __restrict__ Pc, const double* __restrict__ Pv,
    const int* __restrict__ cidx, const int64_t* __restrict__ pt,
    const int64_t* __restrict__ ptkey, const int* __restrict__ rpc, int* __restrict__ cnt,
    int* __restrict__ colc, double* __restrict__ valc, int* __restrict__ spill,
    int* __restrict__ nspill) {
    __shared__ int mcol[kGalMap][kWave];
    __shared__ double mval[FILL ? kGalMap : 1][kWave];
    const int lane = threadIdx.x;
    const int64_t I64 = (int64_t)blockIdx.x * kWave + lane;
    if (I64 >= nc) return;  // no workgroup barriers below
    const int I = (int)I64;
    int m = 0;
    bool over = false;
    const int64_t t1 = pt[I + 1];
    for (int64_t t = pt[I]; t < t1 && !over; ++t) {
        const int64_t k = ptkey[t];
        const int i = (int)(k / cal);
        const double piI = Pv[k];
        const int e1 = rp[i + 1];
        for (int e = rp[i]; e < e1 && !over; ++e) {
            const int j = ci[e];
            const double pa = __dmul_rn(piI, (double)av[e]);
            for (int q = 0; q < cal; ++q) {
                const int c = Pc[(int64_t)j * cal + q];
                if (c < 0 || c >= n) continue;
                const int J = cidx[c];
                if (J < 0) continue;
                const double prod = __dmul_rn(pa, Pv[(int64_t)j * cal + q]);
                int lo = 0, hi = m;  // first map position whose column is >= J
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (mcol[mid][lane] < J) lo = mid + 1;
                    else hi = mid;
                }
                if (lo < m && mcol[lo][lane] == J) {
                    if (FILL) mval[lo][lane] = __dadd_rn(mval[lo][lane], prod);
                    continue;
                }
                if (m == kGalMap) {
                    over = true;
                    break;
                }
                for (int x = m; x > lo; --x) {
                    mcol[x][lane] = mcol[x - 1][lane];
                    if (FILL) mval[x][lane] = mval[x - 1][lane];
                }
                mcol[lo][lane] = J;
                if (FILL) mval[lo][lane] = prod;
                ++m;
            }
        }
    }
    if (over) {
        spill[atomicAdd(nspill, 1)] = I;
        return;
    }
    if (!FILL) {
        cnt[I] = m;
        return;
    }
    const int64_t o = rpc[I];
    for (int x = 0; x < m; ++x) {
        colc[o + x] = mcol[x][lane];
        valc[o + x] = mval[x][lane];
    }
}

// ---------------------------------------------------------------- two-grid pieces
// Dense coarse matrices are row-major: L[i * nc + p] = L_ip.
// L = A_c (every stored entry; the factorisation reads the lower triangle)
__global__ __launch_bounds__(kBlock) void dense_scatter_kernel(int nc, const int* __restrict__ rpc,
                                                               const int* __restrict__ colc,
                                                               const double* __restrict__ valc,
                                                               double* __restrict__ L) {
    const int64_t I = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (I >= nc) return;
    for (int e = rpc[I]; e < rpc[I + 1]; ++e) L[I * nc + colc[e]] = valc[e];
}

// sum_{p < m} x[p] y[p] over one wavefront (lanes stride p), fixed order
__device__ __forceinline__ double wave_dot(const double* __restrict__ x,
                                           const double* __restrict__ y, int m, int lane) {
    double s = 0.0;
    for (int p = lane; p < m; p += kWave) s += x[p] * y[p];
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
    return s;
}

// Cholesky, column k (left-looking): L_kk = sqrt(a_kk - sum_{p<k} L_kp^2);
// bad on a non-positive pivot.  One wavefront.
__global__ __launch_bounds__(kWave) void chol_diag_kernel(int nc, int k, double* __restrict__ L,
                                                          int* bad) {
    const int lane = threadIdx.x;
    const double* row = L + (int64_t)k * nc;
    const double s = wave_dot(row, row, k, lane);
    if (lane == 0) {
        const double d = L[(int64_t)k * nc + k] - s;
        if (!(d > 0.0)) *bad = 1;
        L[(int64_t)k * nc + k] = d > 0.0 ? sqrt(d) : 1.0;
    }
}

// L_ik = (a_ik - sum_{p<k} L_ip L_kp) / L_kk for i > k, one wavefront per row
__global__ __launch_bounds__(kBlock) void chol_col_kernel(int nc, int k, double* __restrict__ L) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t i = k + 1 + (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    if (i >= nc) return;
    const double s = wave_dot(L + i * nc, L + (int64_t)k * nc, k, lane);
    if (lane == 0) L[i * nc + k] = (L[i * nc + k] - s) / L[(int64_t)k * nc + k];
}

// L^{-1} by forward substitution of all unit vectors at once, step k:
// rows i > k of B (initially I) lose L_ik x_k, where x_k = B[k,:] / L_kk is
// final once the steps before k are done (only columns j <= k are nonzero).
// One wavefront per row i.
__global__ __launch_bounds__(kBlock) void inv_update_kernel(int nc, int k,
                                                            const double* __restrict__ L,
                                                            double* __restrict__ B) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t i = k + 1 + (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    if (i >= nc) return;
    const double f = L[i * nc + k] / L[(int64_t)k * nc + k];
    if (f == 0.0) return;
    for (int64_t j = lane; j <= k; j += kWave) B[i * nc + j] -= f * B[(int64_t)k * nc + j];
}

// Li[i][j] = B[i][j] / L_ii (j <= i), and its transpose LiT[j][i]
__global__ __launch_bounds__(kBlock) void inv_scale_kernel(int nc, const double* __restrict__ L,
                                                           double* __restrict__ B,
                                                           double* __restrict__ BT) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t i = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    if (i >= nc) return;
    const double d = L[i * nc + i];
    for (int64_t j = lane; j <= i; j += kWave) {
        const double v = B[i * nc + j] / d;
        B[i * nc + j] = v;
        BT[j * nc + i] = v;
    }
}

// Y[i][k] = sum_{j <= i} Li[i][j] B[j][k]   (Y = L^{-1} B), one wavefront per row
__global__ __launch_bounds__(kBlock) void lower_apply_kernel(int nc, int K,
                                                             const double* __restrict__ Li,
                                                             const double* __restrict__ B,
                                                             double* __restrict__ Y) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t i = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    if (i >= nc) return;
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int64_t j = lane; j <= i; j += kWave) s += Li[i * nc + j] * B[j * K + k];
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
        if (lane == 0) Y[i * K + k] = s;
    }
}

// X[j][k] = sum_{i >= j} LiT[j][i] Y[i][k]   (X = L^{-T} Y), one wavefront per row
__global__ __launch_bounds__(kBlock) void upper_apply_kernel(int nc, int K,
                                                             const double* __restrict__ LiT,
                                                             const double* __restrict__ Y,
                                                             double* __restrict__ X) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t j = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    if (j >= nc) return;
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int64_t i = j + lane; i < nc; i += kWave) s += LiT[j * nc + i] * Y[i * K + k];
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
        if (lane == 0) X[j * K + k] = s;
    }
}

// R = -A E (n x K panels)
template <int K, int LPR>
__global__ __launch_bounds__(kBlock) void neg_apply_kernel(int n, const int* __restrict__ rp,
                                                           const int* __restrict__ ci,
                                                           const double* __restrict__ av,
                                                           const double* __restrict__ E,
                                                           double* __restrict__ R) {
    using S = Shape<double, K, LPR>;
    constexpr int V = S::V, C = S::C;
    const int lane = threadIdx.x & (kWave - 1);
    const int g = lane / LPR, l = lane % LPR;
    const int64_t i64 = ((int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave) * S::RPW + g;
    if (i64 >= n) return;
    double y[V], d;
    Frag<double, V> xi;
    row_spmm<S, double, K>((int)i64, rp[i64], rp[i64 + 1], ci, av, l, [&](int) { return E; }, y, d,
                           xi);
    Frag<double, V> out;
#pragma unroll
    for (int q = 0; q < V; ++q) out.v[q] = -y[q];
    store_lane<double, V, C>(R + (size_t)i64 * K + l * V, out);
}

// Rc[I][k] = sum over P^T entries t of row I (by (i, q)) of p_t R[i_t][k]
__global__ __launch_bounds__(kBlock) void restrict_kernel(int nc, int K, int cal,
                                                          const int64_t* __restrict__ pt,
                                                          const int64_t* __restrict__ key,
                                                          const double* __restrict__ Pv,
                                                          const double* __restrict__ R,
                                                          double* __restrict__ Rc) {
    const int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (x >= (int64_t)nc * K) return;
    const int64_t I = x / K, k = x % K;
    double s = 0.0;
    for (int64_t f = pt[I]; f < pt[I + 1]; ++f) {
        const int64_t kk = key[f];
        s += Pv[kk] * R[(kk / cal) * K + k];
    }
    Rc[x] = s;
}

// E[i][k] += sum_q Pv[i][q] Ec[cidx(Pc[i][q])][k]
__global__ __launch_bounds__(kBlock) void prolong_kernel(int n, int K, int cal,
                                                         const int* __restrict__ Pc,
                                                         const double* __restrict__ Pv,
                                                         const int* __restrict__ cidx,
                                                         const double* __restrict__ Ec,
                                                         double* __restrict__ E) {
    const int64_t x = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (x >= (int64_t)n * K) return;
    const int64_t i = x / K, k = x % K;
    double s = 0.0;
    for (int q = 0; q < cal; ++q) {
        const int c = Pc[i * cal + q];
        if (c >= 0 && c < n && cidx[c] >= 0) s += Pv[i * cal + q] * Ec[(int64_t)cidx[c] * K + k];
    }
    E[x] += s;
}

// part[b * K + k] = sum over block b's rows of e_ik (A e)_ik
template <int K, int LPR>
__global__ __launch_bounds__(kBlock) void anorm_partials_kernel(int n, const int* __restrict__ rp,
                                                                const int* __restrict__ ci,
                                                                const double* __restrict__ av,
                                                                const double* __restrict__ E,
                                                                double* __restrict__ part) {
    using S = Shape<double, K, LPR>;
    constexpr int V = S::V;
    __shared__ double acc[kWavesPerBlock][K];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int g = lane / LPR, l = lane % LPR;
    const int64_t i64 = ((int64_t)blockIdx.x * kWavesPerBlock + wv) * S::RPW + g;
    double sq[V];
#pragma unroll
    for (int q = 0; q < V; ++q) sq[q] = 0.0;
    if (i64 < n) {
        double y[V], d;
        Frag<double, V> xi;
        row_spmm<S, double, K>((int)i64, rp[i64], rp[i64 + 1], ci, av, l, [&](int) { return E; }, y,
                               d, xi);
        const Frag<double, V> ei = load_lane<double, V, S::C>(E + (size_t)i64 * K + l * V);
#pragma unroll
        for (int q = 0; q < V; ++q) sq[q] = ei.v[q] * y[q];
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

// out[k] = sum_b part[b * K + k], one workgroup per k, fixed order
__global__ __launch_bounds__(1024) void columns_sum_kernel(const double* __restrict__ part,
                                                           int64_t m, int K,
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
    if (t == 0) out[k] = acc[0];
}

static unsigned nblocks(int64_t m, int64_t per) {
    const int64_t b = (m + per - 1) / per;
    return (unsigned)(b > 0 ? b : 1);
}

// ---------------------------------------------------------------- host side
int galerkin_prepare(const GalerkinIn& g, GalerkinWork& w, int* nc_out, hipStream_t s) {
    const int n = g.n;
    int rc;
    cf_flags_kernel<<<dim3(nblocks(n, kBlock)), dim3(kBlock), 0, s>>>(n, g.cf, w.flags);
    AD_HIP(hipGetLastError());
    if ((rc = launch_excl_scan(w.flags, n, w.scan, w.scan_tmp, s))) return rc;
    cidx_kernel<<<dim3(nblocks(n, kBlock)), dim3(kBlock), 0, s>>>(n, g.cf, w.scan, w.cidx);
    int64_t ncl = 0;
    AD_HIP(hipMemcpyAsync(&ncl, w.scan + n, sizeof ncl, hipMemcpyDeviceToHost, s));
    AD_HIP(hipStreamSynchronize(s));
    *nc_out = (int)ncl;
    return AD_OK;
}

int galerkin_transpose(const GalerkinIn& g, GalerkinWork& w, int nc, unsigned* status,
                       hipStream_t s) {
    const int n = g.n;
    int rc;
    if ((rc = launch_fill_i32(w.cnt, nc > 0 ? nc : 1, 0, s))) return rc;
    pt_count_kernel<<<dim3(nblocks(n, kBlock)), dim3(kBlock), 0, s>>>(n, g.cal, g.Pc, w.cidx, w.cnt,
                                                                     status);
    AD_HIP(hipGetLastError());
    if ((rc = launch_excl_scan(w.cnt, nc, w.pt, w.scan_tmp, s))) return rc;
    if ((rc = launch_fill_i32(w.cnt, nc > 0 ? nc : 1, 0, s))) return rc;
    pt_fill_kernel<<<dim3(nblocks(n, kBlock)), dim3(kBlock), 0, s>>>(n, g.cal, g.Pc, w.cidx, w.pt,
                                                                    w.cnt, w.ptkey);
    pt_sort_kernel<<<dim3(nblocks(nc, kBlock)), dim3(kBlock), 0, s>>>(nc, w.pt, w.ptkey);
    AD_HIP(hipGetLastError());
    return AD_OK;
}

// The products of every coarse row: the lane kernel, then the sort kernel
// on the rows it spilled (count pass: rpc == nullptr, counts into cnt).
template <typename TA>
static int galerkin_products_t(const GalerkinIn& g, GalerkinWork& w, int nc, const int* rpc,
                               int* cnt, int* colc, double* valc, hipStream_t s) {
    int rc;
    if ((rc = launch_fill_i32(w.nspill, 1, 0, s))) return rc;
    const unsigned nb = nblocks(nc, kWave);
    if (rpc)
        galerkin_lane_kernel<TA, true><<<dim3(nb), dim3(kWave), 0, s>>>(
            g.n, nc, g.rp, g.ci, (const TA*)g.av, g.cal, g.Pc, g.Pv, w.cidx, w.pt, w.ptkey, rpc,
            cnt, colc, valc, w.spill, w.nspill);
    else
        galerkin_lane_kernel<TA, false><<<dim3(nb), dim3(kWave), 0, s>>>(
            g.n, nc, g.rp, g.ci, (const TA*)g.av, g.cal, g.Pc, g.Pv, w.cidx, w.pt, w.ptkey, rpc,
            cnt, colc, valc, w.spill, w.nspill);
    AD_HIP(hipGetLastError());
    // a fixed grid walks the spill list (its length stays on the device)
    const unsigned grid = (unsigned)(nc < 1024 ? nc : 1024);
    galerkin_row_kernel<TA><<<dim3(grid), dim3(kGalWave), 0, s>>>(
        g.n, g.rp, g.ci, (const TA*)g.av, g.cal, g.Pc, g.Pv, w.cidx, w.pt, w.ptkey, rpc, cnt, colc,
        valc, w.spill, w.nspill);
    AD_HIP(hipGetLastError());
    return AD_OK;
}

static int galerkin_products(const GalerkinIn& g, GalerkinWork& w, int nc, const int* rpc,
                             int* cnt, int* colc, double* valc, hipStream_t s) {
    if (nc == 0) return AD_OK;
    return g.dtype == AD_F32
               ? galerkin_products_t<float>(g, w, nc, rpc, cnt, colc, valc, s)
               : galerkin_products_t<double>(g, w, nc, rpc, cnt, colc, valc, s);
}

int galerkin_rows_run(const GalerkinIn& g, GalerkinWork& w, int nc, int* rpc, int64_t* nnz_c,
                      hipStream_t s) {
    int rc;
    if ((rc = launch_fill_i32(w.maxslots, 1, 0, s))) return rc;
    gal_slots_kernel<<<dim3(nblocks(nc, kBlock)), dim3(kBlock), 0, s>>>(nc, g.rp, g.cal, w.pt,
                                                                       w.ptkey, w.maxslots);
    AD_HIP(hipGetLastError());
    int mx = 0;
    AD_HIP(hipMemcpyAsync(&mx, w.maxslots, sizeof mx, hipMemcpyDeviceToHost, s));
    AD_HIP(hipStreamSynchronize(s));
    if (mx > kGalCap) return AD_EUNSUPPORTED;
    if ((rc = galerkin_products(g, w, nc, nullptr, w.cnt, nullptr, nullptr, s))) return rc;
    // row pointers: exclusive scan of the counts (int64), narrowed to int32
    if ((rc = launch_excl_scan(w.cnt, nc, w.scan, w.scan_tmp, s))) return rc;
    int64_t tot = 0;
    AD_HIP(hipMemcpyAsync(&tot, w.scan + nc, sizeof tot, hipMemcpyDeviceToHost, s));
    AD_HIP(hipStreamSynchronize(s));
    if (tot > INT32_MAX) return AD_EUNSUPPORTED;
    if ((rc = launch_narrow_i64(w.scan, (int64_t)nc + 1, rpc, s))) return rc;
    *nnz_c = tot;
    return AD_OK;
}

int galerkin_cols_run(const GalerkinIn& g, GalerkinWork& w, int nc, const int* rpc, int* colc,
                      double* valc, hipStream_t s) {
    return galerkin_products(g, w, nc, rpc, nullptr, colc, valc, s);
}

// diagonal entries of the row-major nc x nc matrix M set to 1 (M zeroed)
__global__ __launch_bounds__(kBlock) void identity_kernel(int nc, double* __restrict__ M) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < nc) M[i * nc + i] = 1.0;
}

int coarse_factor(int nc, const int* rpc, const int* colc, const double* valc, double* L,
                  double* Li, double* LiT, int* bad, hipStream_t s) {
    if (nc > kCoarseSolveMax) return AD_EUNSUPPORTED;
    int rc;
    if ((rc = launch_fill_f64(L, (int64_t)nc * nc, 0.0, s))) return rc;
    if ((rc = launch_fill_f64(Li, (int64_t)nc * nc, 0.0, s))) return rc;
    if ((rc = launch_fill_f64(LiT, (int64_t)nc * nc, 0.0, s))) return rc;
    if ((rc = launch_fill_i32(bad, 1, 0, s))) return rc;
    dense_scatter_kernel<<<dim3(nblocks(nc, kBlock)), dim3(kBlock), 0, s>>>(nc, rpc, colc, valc, L);
    for (int k = 0; k < nc; ++k) {
        chol_diag_kernel<<<dim3(1), dim3(kWave), 0, s>>>(nc, k, L, bad);
        if (k + 1 < nc)
            chol_col_kernel<<<dim3(nblocks(nc - k - 1, kWavesPerBlock)), dim3(kBlock), 0, s>>>(nc, k,
                                                                                             L);
    }
    // L^{-1} (in Li) and its transpose (in LiT)
    identity_kernel<<<dim3(nblocks(nc, kBlock)), dim3(kBlock), 0, s>>>(nc, Li);
    for (int k = 0; k + 1 < nc; ++k)
        inv_update_kernel<<<dim3(nblocks(nc - k - 1, kWavesPerBlock)), dim3(kBlock), 0, s>>>(nc, k, L,
                                                                                           Li);
    inv_scale_kernel<<<dim3(nblocks(nc, kWavesPerBlock)), dim3(kBlock), 0, s>>>(nc, L, Li, LiT);
    AD_HIP(hipGetLastError());
    return AD_OK;
}

template <int K>
static int tg_cycle_go(const GalerkinIn& g, const GalerkinWork& w, int nc, const double* Li,
                       const double* LiT, double* E, double* R, double* Rc, hipStream_t s) {
    constexpr int LPR = lpr_default<double>(K);
    using Sh = Shape<double, K, LPR>;
    const int n = g.n;
    const unsigned rb = nblocks(n, Sh::RPB);
    neg_apply_kernel<K, LPR><<<dim3(rb), dim3(kBlock), 0, s>>>(n, g.rp, g.ci, (const double*)g.av, E,
                                                                R);
    restrict_kernel<<<dim3(nblocks((int64_t)nc * K, kBlock)), dim3(kBlock), 0, s>>>(
        nc, K, g.cal, w.pt, w.ptkey, g.Pv, R, Rc);
    // Rc <- A_c^{-1} Rc through R's storage (n >= nc rows of K)
    lower_apply_kernel<<<dim3(nblocks(nc, kWavesPerBlock)), dim3(kBlock), 0, s>>>(nc, K, Li, Rc, R);
    upper_apply_kernel<<<dim3(nblocks(nc, kWavesPerBlock)), dim3(kBlock), 0, s>>>(nc, K, LiT, R,
                                                                                Rc);
    prolong_kernel<<<dim3(nblocks((int64_t)n * K, kBlock)), dim3(kBlock), 0, s>>>(
        n, K, g.cal, g.Pc, g.Pv, w.cidx, Rc, E);
    AD_HIP(hipGetLastError());
    return AD_OK;
}

template <int K>
static int anorm_go(const GalerkinIn& g, const double* E, double* part, double* out,
                    hipStream_t s) {
    constexpr int LPR = lpr_default<double>(K);
    using Sh = Shape<double, K, LPR>;
    const unsigned rb = nblocks(g.n, Sh::RPB);
    anorm_partials_kernel<K, LPR><<<dim3(rb), dim3(kBlock), 0, s>>>(g.n, g.rp, g.ci,
                                                                     (const double*)g.av, E, part);
    columns_sum_kernel<<<dim3(K), dim3(1024), 0, s>>>(part, rb, K, out);
    AD_HIP(hipGetLastError());
    return AD_OK;
}

int two_grid_blocks(int n, int K) {
    return (int)nblocks(n, (int64_t)kWavesPerBlock * (kWave / lpr_default<double>(K)));
}

int coarse_correction(const GalerkinIn& g, const GalerkinWork& w, int nc, int K, const double* Li,
                      const double* LiT, double* E, double* R, double* Rc, hipStream_t s) {
    switch (K) {
        case 2: return tg_cycle_go<2>(g, w, nc, Li, LiT, E, R, Rc, s);
        case 4: return tg_cycle_go<4>(g, w, nc, Li, LiT, E, R, Rc, s);
        case 8: return tg_cycle_go<8>(g, w, nc, Li, LiT, E, R, Rc, s);
        case 16: return tg_cycle_go<16>(g, w, nc, Li, LiT, E, R, Rc, s);
        case 32: return tg_cycle_go<32>(g, w, nc, Li, LiT, E, R, Rc, s);
        case 64: return tg_cycle_go<64>(g, w, nc, Li, LiT, E, R, Rc, s);
        default: return AD_EINVAL;
    }
}

int a_norms_sq(const GalerkinIn& g, int K, const double* E, double* part, double* out,
               hipStream_t s) {
    switch (K) {
        case 2: return anorm_go<2>(g, E, part, out, s);
        case 4: return anorm_go<4>(g, E, part, out, s);
        case 8: return anorm_go<8>(g, E, part, out, s);
        case 16: return anorm_go<16>(g, E, part, out, s);
        case 32: return anorm_go<32>(g, E, part, out, s);
        case 64: return anorm_go<64>(g, E, part, out, s);
        default: return AD_EINVAL;
    }
}

}  // namespace ad
