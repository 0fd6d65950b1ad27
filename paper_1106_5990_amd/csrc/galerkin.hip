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

// Blocked Cholesky and inverse of the dense coarse matrix, in 64-wide
// blocks: the diagonal block is factored in LDS by one workgroup, which also
// forms its inverse W; the block column below is L_panel = A_panel W^T and
// the trailing matrix loses L_panel L_panel^T (64 x 64 output tiles, FP64
// MFMA, operands staged in LDS 16 columns of the inner dimension at a time).
// The inverse X = L^{-1} follows by blocked forward substitution of the
// identity: block row k becomes W_k times itself, then the rows below lose
// L_{., k} times it.
constexpr int kDb = 64;   // block width
constexpr int kDk = 16;   // inner-dimension chunk staged in LDS

// Factor the diagonal block at (kb, kb) of width b in place (lower part) and
// write W = L_kk^{-1} (64 x 64 row-major, zero outside its lower b x b
// part) to Wk.  A non-positive pivot sets *bad and is replaced by 1.
__global__ __launch_bounds__(kBlock) void chol_block_kernel(int nc, int kb, int b,
                                                            double* __restrict__ L,
                                                            double* __restrict__ Wk, int* bad) {
    __shared__ double T[kDb][kDb + 1];
    __shared__ double Wl[kDb][kDb + 1];
    const int t = threadIdx.x;
    for (int q = t; q < kDb * kDb; q += kBlock) {
        const int r = q / kDb, c = q % kDb;
        T[r][c] = (r < b && c < b) ? L[(int64_t)(kb + r) * nc + kb + c] : 0.0;
    }
    __syncthreads();
    for (int j = 0; j < b; ++j) {
        if (t == 0) {
            const double d = T[j][j];
            if (!(d > 0.0)) *bad = 1;
            T[j][j] = d > 0.0 ? sqrt(d) : 1.0;
        }
        __syncthreads();
        for (int r = j + 1 + t; r < b; r += kBlock) T[r][j] /= T[j][j];
        __syncthreads();
        const int w = b - j - 1;
        for (int q = t; q < w * w; q += kBlock) {
            const int r = j + 1 + q / w, c = j + 1 + q % w;
            if (c <= r) T[r][c] -= T[r][j] * T[c][j];
        }
        __syncthreads();
    }
    // column c of W by forward substitution of the unit vector e_c
    if (t < b) {
        const int c = t;
        for (int r = 0; r < c; ++r) Wl[r][c] = 0.0;
        for (int r = c; r < b; ++r) {
            double v = (r == c) ? 1.0 : 0.0;
            for (int p = c; p < r; ++p) v -= T[r][p] * Wl[p][c];
            Wl[r][c] = v / T[r][r];
        }
    }
    __syncthreads();
    for (int q = t; q < kDb * kDb; q += kBlock) {
        const int r = q / kDb, c = q % kDb;
        if (r < b && c < b && c <= r) L[(int64_t)(kb + r) * nc + kb + c] = T[r][c];
        Wk[q] = (r < b && c < b && c <= r) ? Wl[r][c] : 0.0;
    }
}

enum DenseTile { kTilePanel, kTileSyrk, kTileInvDiag, kTileInvUpdate };

// One 64 x 64 output tile: acc[r][c] = sum_{p < b} Aop(r, p) Bop(p, c), then
// stored (panel, inverse diagonal) or subtracted (updates); 256 threads, the
// products on the FP64 matrix cores.  Operands by mode, with base = kb + b:
//   panel:       rows base.. of L, cols kb..;  A = L[r][kb + p], B = W[c][p]
//   syrk:        tile (tr >= tc) of L at (base + 64 tr, base + 64 tc);
//                A = L[r][kb + p], B = L[c][kb + p]
//   inv diag:    rows kb.. of X, cols 64 x;  A = W[r][p], B = X[kb + p][c]
//   inv update:  rows base.. of X, cols 64 x;  A = L[r][kb + p], B = X[kb + p][c]
// In the in-place modes the tile's operand loads all precede its stores.
template <int MODE>
__global__ __launch_bounds__(kBlock) void dense_tile_kernel(int nc, int kb, int b,
                                                            double* __restrict__ L,
                                                            const double* __restrict__ Wk,
                                                            double* __restrict__ X) {
    __shared__ double As[kDb][kDk + 1];
    __shared__ double Bs[kDk][kDb + 1];
    const int t = threadIdx.x;
    const int base = kb + b;
    int R0, C0, rmax, cmax;
    if (MODE == kTilePanel) {
        R0 = base + blockIdx.x * kDb; C0 = kb; rmax = nc; cmax = base;
    } else if (MODE == kTileSyrk) {
        if (blockIdx.x > blockIdx.y) return;
        R0 = base + blockIdx.y * kDb; C0 = base + blockIdx.x * kDb; rmax = nc; cmax = nc;
    } else if (MODE == kTileInvDiag) {
        R0 = kb; C0 = blockIdx.x * kDb; rmax = base; cmax = base;
    } else {
        R0 = base + blockIdx.y * kDb; C0 = blockIdx.x * kDb; rmax = nc; cmax = base;
    }
    // matrix cores: wavefront w owns rows 16 w .. 16 w + 15 of the tile as
    // four 16 x 16 blocks, each accumulated by FP64 MFMA 16 x 16 x 4 steps
    // (lane l feeds A[16 w + l % 16][k + l / 16] and B[k + l / 16][16 jb + l % 16]
    // and holds D[l / 16 + 4 v][l % 16], v = 0..3)
    const int lane = t & (kWave - 1), w = t / kWave;
    const int l16 = lane & 15, lq = lane >> 4;
    typedef double double4_t __attribute__((ext_vector_type(4)));
    double4_t acc[4];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) acc[jb] = double4_t{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < b; k0 += kDk) {
        // A chunk: 64 rows x 16; each thread 4 consecutive p of one row
        for (int q = t; q < kDb * kDk / 4; q += kBlock) {
            const int r = q / (kDk / 4), p0 = (q % (kDk / 4)) * 4;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int p = k0 + p0 + u;
                double v = 0.0;
                if (R0 + r < rmax && p < b) {
                    if (MODE == kTileInvDiag) v = Wk[r * kDb + p];
                    else v = L[(int64_t)(R0 + r) * nc + kb + p];
                }
                As[r][p0 + u] = v;
            }
        }
        // B chunk: 16 x 64
        for (int q = t; q < kDb * kDk / 4; q += kBlock) {
            if (MODE == kTilePanel || MODE == kTileSyrk) {
                const int c = q / (kDk / 4), p0 = (q % (kDk / 4)) * 4;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int p = k0 + p0 + u;
                    double v = 0.0;
                    if (C0 + c < cmax && p < b)
                        v = (MODE == kTilePanel) ? Wk[c * kDb + p]
                                                 : L[(int64_t)(C0 + c) * nc + kb + p];
                    Bs[p0 + u][c] = v;
                }
            } else {
                const int pp = q / (kDb / 4), c0 = (q % (kDb / 4)) * 4;
                const int p = k0 + pp;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int c = c0 + u;
                    Bs[pp][c] = (p < b && C0 + c < cmax) ? X[(int64_t)(kb + p) * nc + C0 + c] : 0.0;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int st = 0; st < kDk / 4; ++st) {
            const double a = As[w * 16 + l16][st * 4 + lq];
#pragma unroll
            for (int jb = 0; jb < 4; ++jb) {
                const double bv = Bs[st * 4 + lq][jb * 16 + l16];
                acc[jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[jb], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    double* C = (MODE == kTilePanel || MODE == kTileSyrk) ? L : X;
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
        const int c = C0 + jb * 16 + l16;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = R0 + w * 16 + lq + 4 * v;
            if (r >= rmax || c >= cmax) continue;
            double* dst = C + (int64_t)r * nc + c;
            if (MODE == kTilePanel || MODE == kTileInvDiag) *dst = acc[jb][v];
            else *dst -= acc[jb][v];
        }
    }
}

// LiT = Li^T through 32 x 32 LDS tiles (Li's upper part is zero)
__global__ __launch_bounds__(kBlock) void dense_transpose_kernel(int nc, const double* __restrict__ Li,
                                                                 double* __restrict__ LiT) {
    __shared__ double tl[32][33];
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;  // 32 x 8
    const int bx = blockIdx.x, by = blockIdx.y;
    for (int r = ty; r < 32; r += 8) {
        const int i = by * 32 + r, j = bx * 32 + tx;
        tl[r][tx] = (i < nc && j < nc) ? Li[(int64_t)i * nc + j] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int j = bx * 32 + r, i = by * 32 + tx;
        if (i < nc && j < nc) LiT[(int64_t)j * nc + i] = tl[tx][r];
    }
}

// Y[i][k] = sum_{j <= i} Li[i][j] B[j][k]   (Y = L^{-1} B), one wavefront per
// row: each Li entry is read once per kApplyK columns
constexpr int kApplyK = 8;
__global__ __launch_bounds__(kBlock) void lower_apply_kernel(int nc, int K,
                                                             const double* __restrict__ Li,
                                                             const double* __restrict__ B,
                                                             double* __restrict__ Y) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t i = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    if (i >= nc) return;
    for (int k0 = 0; k0 < K; k0 += kApplyK) {
        double s[kApplyK];
#pragma unroll
        for (int k = 0; k < kApplyK; ++k) s[k] = 0.0;
        for (int64_t j = lane; j <= i; j += kWave) {
            const double l = Li[i * nc + j];
#pragma unroll
            for (int k = 0; k < kApplyK; ++k)
                if (k0 + k < K) s[k] += l * B[j * K + k0 + k];
        }
#pragma unroll
        for (int k = 0; k < kApplyK; ++k) {
            double v = s[k];
#pragma unroll
            for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
            if (lane == 0 && k0 + k < K) Y[i * K + k0 + k] = v;
        }
    }
}

// X[j][k] = sum_{i >= j} LiT[j][i] Y[i][k]   (X = L^{-T} Y), one wavefront per
// row, each LiT entry read once per kApplyK columns
__global__ __launch_bounds__(kBlock) void upper_apply_kernel(int nc, int K,
                                                             const double* __restrict__ LiT,
                                                             const double* __restrict__ Y,
                                                             double* __restrict__ X) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t j = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    if (j >= nc) return;
    for (int k0 = 0; k0 < K; k0 += kApplyK) {
        double s[kApplyK];
#pragma unroll
        for (int k = 0; k < kApplyK; ++k) s[k] = 0.0;
        for (int64_t i = j + lane; i < nc; i += kWave) {
            const double l = LiT[j * nc + i];
#pragma unroll
            for (int k = 0; k < kApplyK; ++k)
                if (k0 + k < K) s[k] += l * Y[i * K + k0 + k];
        }
#pragma unroll
        for (int k = 0; k < kApplyK; ++k) {
            double v = s[k];
#pragma unroll
            for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
            if (lane == 0 && k0 + k < K) X[j * K + k0 + k] = v;
        }
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

size_t coarse_factor_workspace(int nc) {
    return sizeof(double) * (size_t)((nc + kDb - 1) / kDb) * kDb * kDb;
}

int coarse_factor(int nc, const int* rpc, const int* colc, const double* valc, double* L,
                  double* Li, double* LiT, double* Wblk, int* bad, hipStream_t s) {
    if (nc > kCoarseSolveMax) return AD_EUNSUPPORTED;
    if (nc == 0) return launch_fill_i32(bad, 1, 0, s);
    int rc;
    if ((rc = launch_fill_f64(L, (int64_t)nc * nc, 0.0, s))) return rc;
    if ((rc = launch_fill_f64(Li, (int64_t)nc * nc, 0.0, s))) return rc;
    if ((rc = launch_fill_i32(bad, 1, 0, s))) return rc;
    dense_scatter_kernel<<<dim3(nblocks(nc, kBlock)), dim3(kBlock), 0, s>>>(nc, rpc, colc, valc, L);
    for (int kb = 0; kb < nc; kb += kDb) {
        const int b = (nc - kb < kDb) ? nc - kb : kDb;
        double* Wk = Wblk + (size_t)(kb / kDb) * kDb * kDb;
        chol_block_kernel<<<dim3(1), dim3(kBlock), 0, s>>>(nc, kb, b, L, Wk, bad);
        const int m = nc - kb - b;
        if (m > 0) {
            const unsigned T = (unsigned)((m + kDb - 1) / kDb);
            dense_tile_kernel<kTilePanel><<<dim3(T), dim3(kBlock), 0, s>>>(nc, kb, b, L, Wk, Li);
            dense_tile_kernel<kTileSyrk><<<dim3(T, T), dim3(kBlock), 0, s>>>(nc, kb, b, L, Wk, Li);
        }
    }
    AD_HIP(hipGetLastError());
    // L^{-1} (in Li, from the identity) and its transpose (in LiT)
    identity_kernel<<<dim3(nblocks(nc, kBlock)), dim3(kBlock), 0, s>>>(nc, Li);
    for (int kb = 0; kb < nc; kb += kDb) {
        const int b = (nc - kb < kDb) ? nc - kb : kDb;
        const double* Wk = Wblk + (size_t)(kb / kDb) * kDb * kDb;
        const unsigned Tc = (unsigned)((kb + b + kDb - 1) / kDb);
        dense_tile_kernel<kTileInvDiag><<<dim3(Tc), dim3(kBlock), 0, s>>>(nc, kb, b, L, Wk, Li);
        const int m = nc - kb - b;
        if (m > 0) {
            const unsigned Tr = (unsigned)((m + kDb - 1) / kDb);
            dense_tile_kernel<kTileInvUpdate><<<dim3(Tc, Tr), dim3(kBlock), 0, s>>>(nc, kb, b, L, Wk,
                                                                                    Li);
        }
    }
    const unsigned T32 = (unsigned)((nc + 31) / 32);
    dense_transpose_kernel<<<dim3(T32, T32), dim3(kBlock), 0, s>>>(nc, Li, LiT);
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
