// longrange.hip -- long-range connectivity and the search over interpolatory
// sets (Sec. 4.1 eq. graph, the closing remark of Sec. 4.2, Sec. 4.3).
//
// Pattern of A^d.  Row i of A^d holds (structurally) every j within graph
// distance d of i; A^d itself is never formed.  One wavefront per row runs
// a breadth-first search of depth d over the graph of A, a level at a
// time: the frontier's rows of A are walked with every lane taking its own
// entries, inserted into an LDS hash set (open addressing,
// compare-and-swap), new vertices appended to a list that holds the levels
// in order.  A wavefront handles several rows, clearing only the slots a
// row took.  The count pass writes |row|; the fill pass repeats the search
// and writes the list sorted (bitonic sort in LDS).
//
// Interpolatory-set search.  One wavefront per F row: the row's candidates
// (the C-points of its row of the pattern, i excluded, in column order) and
// their panel rows are staged in LDS, with the FP64 target and the FP64
// Gram matrix G_ab = <x_a, x_b>_w and h_a = <x_a, t>_w of all candidates.
// Every set W of each size m <= caliber is then a small Cholesky on
// entries of G (a set with a pivot <= kSearchDep = 1e-8 of its Gram
// diagonal is numerically dependent and skipped: the Gram entries carry
// rounding of order eps |x_a| |x_b|, which earlier small pivots amplify, so
// a smaller pivot can be rounding alone), whose back substitution gives the
// minimiser; LS_W is then evaluated by its definition from the rows in LDS.
// Lanes take consecutive blocks of the sets in lexicographic order (the
// first unranked, the rest by successor); the least (value, rank) over the
// wave is that size's best.  The size is chosen by the penalty rule in
// increasing size against the incumbent, on values relative to
// S = <t, t>_w; the chosen set's weights come from its Cholesky solve and
// its functional is evaluated by definition once more, lanes over k.

#include <math.h>

#include "device.h"
#include "internal.h"

namespace ad {

// ---------------------------------------------------------------- pattern of A^d
constexpr int kPowCap = 1024;   // entries per row of A^d
constexpr int kPowHash = 2048;  // LDS hash slots per wavefront (load factor <= 1/2 + 1/32)
constexpr int kPowWaves = 4;    // wavefronts per workgroup
constexpr int kPowRows = 8;     // rows per wavefront (the hash is cleared once per wavefront)

struct PowLds {
    int hash[kPowWaves][kPowHash];
    int list[kPowWaves][kPowCap];  // the vertices in the order found
    short slot[kPowWaves][kPowCap];  // the hash slot each one took
    int off[kPowWaves][kPowCap];   // expansion offsets of the frontier
    int n[kPowWaves];
};

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// exclusive wave prefix of v over the lanes; *total receives the sum
__device__ __forceinline__ int wave_excl(int v, int lane, int* total) {
    int x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    *total = __shfl(x, kWave - 1, kWave);
    return x - v;
}

// Inserts j; appends it to the list when new.  false when the list is full.
__device__ __forceinline__ bool pow_insert(int j, PowLds& L, int wv) {
    int* hash = L.hash[wv];
    unsigned slot = ((unsigned)j * 2654435761u) & (kPowHash - 1);
    for (int probe = 0; probe < kPowHash; ++probe) {
        const int prev = atomicCAS(&hash[slot], -1, j);
        if (prev == j) return true;  // already in the set
        if (prev == -1) {            // new
            const int pos = atomicAdd(&L.n[wv], 1);
            if (pos >= kPowCap) return false;
            L.list[wv][pos] = j;
            L.slot[wv][pos] = (short)slot;
            return true;
        }
        slot = (slot + 1) & (kPowHash - 1);
    }
    return false;
}

// Breadth-first search of depth d from row i, a level at a time: the
// frontier's rows of A are walked with every lane taking its own entries
// (all of a level's loads in flight together) and inserting them into the
// wavefront's LDS hash set, new vertices appended to the list, so the list
// holds the levels one after the other.  Returns |row of A^d| (the list),
// or -1 past kPowCap.  The caller clears the used slots afterwards.
__device__ int pow_row(int i, int d, const int* __restrict__ rp, const int* __restrict__ ci,
                       PowLds& L, int wv, int lane) {
    int* list = L.list[wv];
    int* off = L.off[wv];
    if (lane == 0) {
        L.n[wv] = 0;
    }
    wave_sync_lds();
    if (lane == 0) pow_insert(i, L, wv);
    wave_sync_lds();
    int lo = 0, hi = 1;
    bool over = false;
    for (int lev = 0; lev < d && lo < hi && !over; ++lev) {
        const int nf = hi - lo;
        int total = 0;
        for (int c0 = 0; c0 < nf; c0 += kWave) {
            const int q = c0 + lane;
            const int deg = q < nf ? rp[list[lo + q] + 1] - rp[list[lo + q]] : 0;
            int sum;
            const int ex = wave_excl(deg, lane, &sum);
            if (q < nf) off[q] = total + ex;
            total += sum;
        }
        wave_sync_lds();
        for (int k = lane; k < total; k += kWave) {
            int a = 0, b = nf;  // last frontier entry with off <= k
            while (b - a > 1) {
                const int mid = (a + b) >> 1;
                if (off[mid] <= k) a = mid;
                else b = mid;
            }
            const int u = list[lo + a];
            if (!pow_insert(ci[rp[u] + (k - off[a])], L, wv) ||
                __atomic_load_n(&L.n[wv], __ATOMIC_RELAXED) > kPowCap) {
                over = true;
                break;
            }
        }
        wave_sync_lds();
        lo = hi;
        hi = L.n[wv];
        over = __any(over) || hi > kPowCap;
    }
    return over ? -1 : hi;
}

// back to an empty hash: the slots the row's vertices took, or every slot
// after an overflow (whose last inserts are not in the list)
__device__ __forceinline__ void pow_clear(PowLds& L, int wv, int lane) {
    const int m = L.n[wv];
    if (m > kPowCap) {
        for (int q = lane; q < kPowHash; q += kWave) L.hash[wv][q] = -1;
    } else {
        for (int q = lane; q < m; q += kWave) L.hash[wv][L.slot[wv][q]] = -1;
    }
    wave_sync_lds();
}

__device__ __forceinline__ void pow_init(PowLds& L, int wv, int lane) {
    for (int q = lane; q < kPowHash; q += kWave) L.hash[wv][q] = -1;
    wave_sync_lds();
}

// ---------------------------------------------------------------- lane rows
// For d <= 2 a row of A^d is {i} with N(i) and, for d = 2, N(j) of every j in
// N(i): one lane per row merges these into its own LDS list, kept sorted
// (binary search, insertion by shifting), of at most kPowLane entries.  The
// count pass marks a row that outgrows the list (kPowMarked) for the
// hash-set kernels; the fill pass takes the rows whose length (from the row
// pointers) is at most kPowLane, keeping the kPowLane smallest columns.
constexpr int kPowLane = 64;
constexpr int kPowMarked = -2;

template <bool FILL>
__global__ __launch_bounds__(kWave) void pow_lane_kernel(int n, int d, const int* __restrict__ rp,
                                                         const int* __restrict__ ci,
                                                         int* __restrict__ cnt,
                                                         const int* __restrict__ rpd,
                                                         int* __restrict__ cid, unsigned* status) {
    __shared__ int lst[kPowLane][kWave];
    const int lane = threadIdx.x;
    const int64_t i64 = (int64_t)blockIdx.x * kWave + lane;
    if (i64 >= n) return;  // no workgroup barriers below
    const int i = (int)i64;
    int room = 0;
    if (FILL) {
        room = rpd[i + 1] - rpd[i];
        if (room > kPowLane) return;  // a row for the hash-set kernel
    }
    int m = 0;
    bool over = false;
    auto insert = [&](int v) {
        int lo = 0, hi = m;  // first position whose entry is >= v
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (lst[mid][lane] < v) lo = mid + 1;
            else hi = mid;
        }
        if (lo < m && lst[lo][lane] == v) return;
        if (m == kPowLane) {  // full: keep the kPowLane smallest
            over = true;
            if (lo == m) return;
            --m;
        }
        for (int x = m; x > lo; --x) lst[x][lane] = lst[x - 1][lane];
        lst[lo][lane] = v;
        ++m;
    };
    insert(i);
    const int e0 = rp[i], e1 = rp[i + 1];
    for (int e = e0; e < e1; ++e) insert(ci[e]);
    if (d == 2) {
        for (int e = e0; e < e1 && (FILL || !over); ++e) {
            const int j = ci[e];
            const int f1 = rp[j + 1];
            for (int f = rp[j]; f < f1 && (FILL || !over); ++f) insert(ci[f]);
        }
    }
    if (!FILL) {
        cnt[i] = over ? kPowMarked : m;
        return;
    }
    // row pointers that do not match this row's length are flagged, and no
    // entry is written outside the row
    if (over || m != room) flag(status, AD_STAT_PATTERN);
    const int cw = room < m ? room : m;
    int* out = cid + rpd[i];
    for (int x = 0; x < cw; ++x) out[x] = lst[x][lane];
}

// The hash-set kernels: every row (d > 2), or only the rows the lane
// kernel left (count pass: marked; fill pass: longer than kPowLane).
__global__ __launch_bounds__(kWave* kPowWaves) void pow_count_kernel(int n, int d,
                                                                     const int* __restrict__ rp,
                                                                     const int* __restrict__ ci,
                                                                     int* __restrict__ cnt,
                                                                     bool marked) {
    __shared__ PowLds L;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int64_t i0 = ((int64_t)blockIdx.x * kPowWaves + wv) * kPowRows;
    if (i0 >= n) return;  // whole wavefront
    pow_init(L, wv, lane);
    for (int64_t i = i0; i < i0 + kPowRows && i < n; ++i) {
        if (marked && cnt[i] != kPowMarked) continue;
        const int c = pow_row((int)i, d, rp, ci, L, wv, lane);
        if (lane == 0) cnt[i] = c;
        pow_clear(L, wv, lane);
    }
}

__global__ __launch_bounds__(kWave* kPowWaves) void pow_fill_kernel(
    int n, int d, const int* __restrict__ rp, const int* __restrict__ ci,
    const int* __restrict__ rpd, int* __restrict__ cid, int lane_rows, unsigned* status) {
    __shared__ PowLds L;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int64_t i0 = ((int64_t)blockIdx.x * kPowWaves + wv) * kPowRows;
    if (i0 >= n) return;  // whole wavefront
    pow_init(L, wv, lane);
    for (int64_t i = i0; i < i0 + kPowRows && i < n; ++i) {
        if (rpd[i + 1] - rpd[i] <= lane_rows) continue;  // done by the lane kernel
        const int c = pow_row((int)i, d, rp, ci, L, wv, lane);
        pow_clear(L, wv, lane);
        if (c < 0) continue;  // the count pass refused such a matrix
        int* a = L.list[wv];
        int m = 1;
        while (m < c) m <<= 1;
        for (int q = c + lane; q < m; q += kWave) a[q] = 0x7fffffff;
        wave_sync_lds();
        // bitonic sort of a[0 .. m), m a power of two <= kPowCap
        for (int k = 2; k <= m; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int q = lane; q < m; q += kWave) {
                    const int p = q ^ j;
                    if (p > q) {
                        const int x = a[q], y = a[p];
                        const bool up = (q & k) == 0;
                        if ((x > y) == up) {
                            a[q] = y;
                            a[p] = x;
                        }
                    }
                }
                wave_sync_lds();
            }
        }
        // row pointers that do not match this row's length (not those of the
        // same A and d) are flagged, and no entry is written outside the row
        const int room = rpd[i + 1] - rpd[i];
        if (room != c && lane == 0) flag(status, AD_STAT_PATTERN);
        const int cw = room < c ? room : c;
        int* out = cid + rpd[i];
        for (int q = lane; q < cw; q += kWave) out[q] = a[q];
        wave_sync_lds();
    }
}

// rpd[0] = 0, rpd[i + 1] = rpd[i] + cnt[i] (int32), total into *tot; a
// negative count (a row over the cap) or a total past int32 sets *bad.
__global__ __launch_bounds__(kBlock) void pow_rows_kernel(int n, const int* __restrict__ cnt,
                                                          const int64_t* __restrict__ pre,
                                                          int* __restrict__ rpd,
                                                          int64_t* __restrict__ tot,
                                                          int* __restrict__ bad) {
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q > n) return;
    const int64_t v = pre[q];
    if (q < n && cnt[q] < 0) atomicOr(bad, 1);
    if (v > 0x7fffffffLL) atomicOr(bad, 2);
    rpd[q] = (int)v;
    if (q == n) *tot = v;
}

size_t pow_rows_workspace(int n) {
    return sizeof(int) * ((size_t)n + 1) + sizeof(int64_t) * ((size_t)n + 2) +
           (size_t)scan_workspace_bytes(n) + 1024;
}

int launch_pow_rows(int n, int d, const int* rp, const int* ci, int* rpd, void* ws,
                    int64_t* host_tot, int* host_bad, hipStream_t s) {
    WsReq req;
    const size_t o_cnt = req.add(sizeof(int) * ((size_t)n + 1));
    const size_t o_pre = req.add(sizeof(int64_t) * ((size_t)n + 1));
    const size_t o_sc = req.add((size_t)scan_workspace_bytes(n));
    const size_t o_tot = req.add(sizeof(int64_t) + sizeof(int));
    char* w = (char*)ws;
    int* cnt = (int*)(w + o_cnt);
    int64_t* pre = (int64_t*)(w + o_pre);
    int64_t* tot = (int64_t*)(w + o_tot);
    int* bad = (int*)(w + o_tot + sizeof(int64_t));
    int rc;
    if ((rc = launch_fill_i32(bad, 1, 0, s))) return rc;
    if (n > 0) {
        const bool lanes = d <= 2;
        if (lanes) {
            const unsigned nl = (unsigned)(((int64_t)n + kWave - 1) / kWave);
            pow_lane_kernel<false><<<dim3(nl), dim3(kWave), 0, s>>>(n, d, rp, ci, cnt, nullptr,
                                                                   nullptr, nullptr);
            AD_HIP(hipGetLastError());
        }
        const int64_t per = (int64_t)kPowWaves * kPowRows;
        const unsigned nb = (unsigned)(((int64_t)n + per - 1) / per);
        pow_count_kernel<<<dim3(nb), dim3(kWave * kPowWaves), 0, s>>>(n, d, rp, ci, cnt, lanes);
        AD_HIP(hipGetLastError());
    }
    if ((rc = launch_excl_scan(cnt, n, pre, (int64_t*)(w + o_sc), s))) return rc;
    const unsigned nb = (unsigned)(((int64_t)n + 1 + kBlock - 1) / kBlock);
    pow_rows_kernel<<<dim3(nb), dim3(kBlock), 0, s>>>(n, cnt, pre, rpd, tot, bad);
    AD_HIP(hipGetLastError());
    AD_HIP(hipMemcpyAsync(host_tot, tot, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    AD_HIP(hipMemcpyAsync(host_bad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    AD_HIP(hipStreamSynchronize(s));
    return AD_OK;
}

int launch_pow_cols(int n, int d, const int* rp, const int* ci, const int* rpd, int* cid,
                    unsigned* status, hipStream_t s) {
    if (n == 0) return AD_OK;
    const bool lanes = d <= 2;
    if (lanes) {
        const unsigned nl = (unsigned)(((int64_t)n + kWave - 1) / kWave);
        pow_lane_kernel<true><<<dim3(nl), dim3(kWave), 0, s>>>(n, d, rp, ci, nullptr, rpd, cid,
                                                              status);
        AD_HIP(hipGetLastError());
    }
    const int64_t per = (int64_t)kPowWaves * kPowRows;
    const unsigned nb = (unsigned)(((int64_t)n + per - 1) / per);
    pow_fill_kernel<<<dim3(nb), dim3(kWave * kPowWaves), 0, s>>>(n, d, rp, ci, rpd, cid,
                                                                   lanes ? kPowLane : -1, status);
    AD_HIP(hipGetLastError());
    return AD_OK;
}

// ---------------------------------------------------------------- set search
// A wavefront searches one F row at a time: the target and the candidates'
// panel rows go to the wavefront's LDS slice, the lanes form h and the
// packed Gram matrix, then every lane fits a contiguous block of subsets of
// each size in lexicographic order.  Consecutive subsets of a block share
// their leading positions, so the Cholesky rows of those positions are kept
// and only the rows from the first changed position on are refactored (the
// same operations in the same order as a full factorization of each set).
// A first pass with room for kSearchFast candidates handles every row and
// marks the F rows with more (row status -1); a second pass with room for
// kSearchCand takes only the marked rows.
constexpr int kSearchCand = 64;  // candidates per row (the cap of the search)
constexpr int kSearchFast = 32;  // candidates per row in the first pass
constexpr int kSearchCal = 4;    // largest set size
constexpr int kSearchMarked = -1;  // row status between the two passes

template <typename T, int K, int NCAP>
struct SearchLds {
    double g[NCAP * (NCAP + 1) / 2];  // packed lower triangle, (a, b) at a (a + 1) / 2 + b, b <= a
    double h[NCAP];
    double t[K];
    double w[K];
    T x[NCAP][K + 1];  // candidate panel rows (padded against bank conflicts)
    int cand[NCAP];
};

// C(a, b) for b <= 4 and a <= kSearchCand (at most C(64, 4) = 635376)
__device__ __forceinline__ int binom_small(int a, int b) {
    if (b < 0 || a < b) return 0;
    switch (b) {
        case 0: return 1;
        case 1: return a;
        case 2: return a * (a - 1) / 2;
        case 3: return a * (a - 1) * (a - 2) / 6;
        default: return a * (a - 1) / 2 * ((a - 2) * (a - 3) / 2) / 6;
    }
}

// The combination of rank r (lexicographic order) of m out of nc.
__device__ __forceinline__ void unrank(int r, int nc, int m, int (&idx)[kSearchCal]) {
    int c = 0;
#pragma unroll
    for (int q = 0; q < kSearchCal; ++q) {
        if (q >= m) break;
        for (;;) {
            const int cnt = binom_small(nc - c - 1, m - q - 1);
            if (r < cnt) break;
            r -= cnt;
            ++c;
        }
        idx[q] = c++;
    }
}

// The successor of idx in lexicographic order; returns the first position
// that changed (-1 after the last combination).
__device__ __forceinline__ int next_comb(int nc, int m, int (&idx)[kSearchCal]) {
    // the last position below its largest value (constant register indices)
    int q = -1;
#pragma unroll
    for (int p = 0; p < kSearchCal; ++p)
        if (p < m && idx[p] != nc - m + p) q = p;
    if (q < 0) return -1;
#pragma unroll
    for (int p = 0; p < kSearchCal; ++p) {
        if (p == q) ++idx[p];
        else if (p > q && p < m) idx[p] = idx[p > 0 ? p - 1 : 0] + 1;
    }
    return q;
}

// G_W entry of positions (a, b), a >= b: the positions of a set are in
// increasing candidate order, so idx[a] >= idx[b] and the entry sits in row
// idx[a] of the packed triangle.
__device__ __forceinline__ double gram_ab(const double* g, int ia, int ib) {
    return g[(((unsigned)ia * (unsigned)(ia + 1)) >> 1) + (unsigned)ib];
}

// A pivot at or below this fraction of its Gram diagonal marks a dependent set.
constexpr double kSearchDep = 1e-8;
// Bound on the short form's rounding, in units of S + M sum_a c_a^2 G_aa.
constexpr double kSearchRound = 1e-12;

// Cholesky factor of G_W for the leading positions of W: the off-diagonal
// rows of L, the reciprocals of its diagonal and z = L^{-1} h_W.
struct SetFit {
    double L[kSearchCal][kSearchCal];
    double inv[kSearchCal];
    double z[kSearchCal];
};

// Rows [from, upto) of the factor of G_W (W = candidates idx[...]), rows
// below `from` already in F.  Returns the first position whose pivot fails
// the dependence rule (<= kSearchDep of its Gram diagonal), or upto.
__device__ __forceinline__ int fit_rows(const double* g, const double* h, int from, int upto,
                                        const int (&idx)[kSearchCal], SetFit& F) {
#pragma unroll
    for (int a = 0; a < kSearchCal; ++a) {
        if (a < from) continue;
        if (a >= upto) break;
        const double gaa = gram_ab(g, idx[a], idx[a]);
#pragma unroll
        for (int b = 0; b < kSearchCal; ++b) {
            if (b >= a) break;
            double s = gram_ab(g, idx[a], idx[b]);
#pragma unroll
            for (int c = 0; c < kSearchCal; ++c) {
                if (c >= b) break;
                s -= F.L[a][c] * F.L[b][c];
            }
            F.L[a][b] = s * F.inv[b];
        }
        double piv = gaa;
#pragma unroll
        for (int b = 0; b < kSearchCal; ++b) {
            if (b >= a) break;
            piv -= F.L[a][b] * F.L[a][b];
        }
        if (!(piv > kSearchDep * gaa)) return a;
        F.inv[a] = 1.0 / sqrt(piv);
        double s = h[idx[a]];
#pragma unroll
        for (int b = 0; b < kSearchCal; ++b) {
            if (b >= a) break;
            s -= F.L[a][b] * F.z[b];
        }
        F.z[a] = s * F.inv[a];
    }
    return upto;
}

// The functional of the set whose leading M - 1 positions are factored in
// F, against the lane's best value `cut`.  The last row l = L_{M-1, <M-1}
// and pivot p complete the factor; back substitution L^T c = z gives the
// minimiser (its last entry (h - l . z) / p, no square root).  The short
// form S - |z|^2 cancels: it cannot resolve a value much below eps S, nor
// one of a set whose weights cancel, and a value it rounds to zero or below
// would pass the penalty rule as an exact fit.  Its error is within
// kSearchRound (S + M sum_a c_a^2 G_aa) (rounding of the Gram entries
// carried through the minimiser; 1.7 eps times that bound at most over
// 27 000 sets of near-exact and nearly dependent fits), so a set whose
// short form minus that bound is not below `cut` cannot beat the lane's
// best and is dropped; every other set is evaluated by its definition,
// sum_k w_k (t_k - sum_a c_a x_{a,k})^2 over the candidate rows in LDS,
// off only by |X_W dc|^2.  false when the last pivot fails the dependence
// rule or the set is dropped.
template <int M, typename T, int K, int NCAP>
__device__ __forceinline__ bool last_value(const SearchLds<T, K, NCAP>& Ls, double S, double cut,
                                           const int (&idx)[kSearchCal], const SetFit& F,
                                           double* val) {
    constexpr int A = M - 1;
    const double gaa = gram_ab(Ls.g, idx[A], idx[A]);
    double l[kSearchCal];
#pragma unroll
    for (int b = 0; b < A; ++b) {
        double s = gram_ab(Ls.g, idx[A], idx[b]);
#pragma unroll
        for (int c = 0; c < b; ++c) s -= l[c] * F.L[b][c];
        l[b] = s * F.inv[b];
    }
    double piv = gaa;
#pragma unroll
    for (int b = 0; b < A; ++b) piv -= l[b] * l[b];
    if (!(piv > kSearchDep * gaa)) return false;
    double t = Ls.h[idx[A]];
#pragma unroll
    for (int b = 0; b < A; ++b) t -= l[b] * F.z[b];
    double c[kSearchCal];
    c[A] = t / piv;
    double zz = t * c[A];  // z_{M-1}^2
    double cg = c[A] * c[A] * gaa;
#pragma unroll
    for (int b = A - 1; b >= 0; --b) {
        double s = F.z[b] - l[b] * c[A];
#pragma unroll
        for (int a = b + 1; a < A; ++a) s -= F.L[a][b] * c[a];
        c[b] = s * F.inv[b];
        zz = fma(F.z[b], F.z[b], zz);
        cg = fma(c[b] * c[b], gram_ab(Ls.g, idx[b], idx[b]), cg);
    }
    if (S - zz - kSearchRound * (S + (double)M * cg) >= cut) return false;
    double v = 0.0;
#pragma unroll 1
    for (int k = 0; k < K; ++k) {
        double r = Ls.t[k];
#pragma unroll
        for (int a = 0; a < M; ++a) r -= c[a] * (double)Ls.x[idx[a]][k];
        v = fma(Ls.w[k] * r, r, v);
    }
    *val = v;
    return true;
}

// The minimiser of a fitted set of size m: back substitution L^T c = z.
__device__ __forceinline__ void fit_coef(const SetFit& F, int m, double (&coef)[kSearchCal]) {
#pragma unroll
    for (int a = kSearchCal - 1; a >= 0; --a) {
        if (a >= m) continue;
        double s = F.z[a];
#pragma unroll
        for (int b = 0; b < kSearchCal; ++b)
            if (b > a && b < m) s -= F.L[b][a] * coef[b];
        coef[a] = s * F.inv[a];
    }
}

// A value equal in every lane of the wavefront, moved to scalar registers.
__device__ __forceinline__ double wave_uniform(double x) {
    return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(x)),
                            __builtin_amdgcn_readfirstlane(__double2loint(x)));
}

// x^e for x >= 0, e >= 0 from exp(e log x), both by series: log by
// reduction to m 2^k with m in [sqrt(1/2), sqrt(2)) and log m =
// 2 atanh((m - 1) / (m + 1)) (odd-power series, 12 terms), exp by
// reduction to r + j ln 2 with |r| <= ln 2 / 2 and the Taylor series of e^r
// (18 terms), ln 2 split in a high and a low part.  The relative error
// grows with |e log x| (about 1e-13 at e log x = -660, a few 1e-16 for
// |e log x| below 1); only the penalty rule's thresholds use it, where a
// library pow would set the register count of the whole kernel.  Out of
// line: called a few times per row, inlined it raised the search kernel
// from 157 to 179 VGPRs (3 to 2 wavefronts per SIMD).
__device__ __noinline__ double pow_series(double x, double e) {
    if (e == 0.0) return 1.0;
    if (!(x > 0.0)) return 0.0;
    if (isinf(x)) return x;
    constexpr double kLn2Hi = 6.93147180369123816490e-01;  // leading bits of ln 2
    constexpr double kLn2Lo = 1.90821492927058770002e-10;  // ln 2 - kLn2Hi
    int k = 0;
    double m = frexp(x, &k);  // x = m 2^k, m in [1/2, 1)
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        --k;
    }
    const double sr = (m - 1.0) / (m + 1.0);
    const double s2 = sr * sr;
    double poly = 1.0 / 23.0;
#pragma unroll
    for (int j = 21; j >= 1; j -= 2) poly = fma(poly, s2, 1.0 / (double)j);
    const double logx_lo = 2.0 * sr * poly + (double)k * kLn2Lo;
    const double y_hi = e * (double)k * kLn2Hi, y_lo = e * logx_lo;
    const double y = y_hi + y_lo;
    if (y < -745.2) return 0.0;
    if (y > 709.7) return INFINITY;
    const double jn = rint(y * 1.44269504088896340736);
    const double r = (y_hi - jn * kLn2Hi) + (y_lo - jn * kLn2Lo);
    double t = 1.0;
#pragma unroll
    for (int j = 18; j >= 1; --j) t = fma(t, r * (1.0 / (double)j), 1.0);
    return ldexp(t, (int)jn);
}

// The lane's block of size-M sets (consecutive ranks in lexicographic
// order): the least functional and its rank into (bv, br).  The Cholesky
// rows of the leading positions are refactored only from the first
// position that changed, and not at all while an unchanged leading
// position stays dependent.
template <int M, typename T, int K, int NCAP>
__device__ __forceinline__ void best_of_size(const SearchLds<T, K, NCAP>& Ls, double S, int nc,
                                             int lane, double& bv, int& br) {
    const double* g = Ls.g;
    const double* h = Ls.h;
    const int total = binom_small(nc, M);
    const int per = (total + kWave - 1) / kWave;
    const int r0 = lane * per, r1 = (r0 + per < total) ? r0 + per : total;
    if (r0 >= r1) return;
    int idx[kSearchCal];
    unrank(r0, nc, M, idx);
    SetFit F;
    int lead = fit_rows(g, h, 0, M - 1, idx, F);  // first dependent leading position, or M - 1
    for (int r = r0;;) {
        double v;
        if (lead == M - 1 && last_value<M>(Ls, S, bv, idx, F, &v) && v < bv) {
            bv = v;
            br = r;
        }
        if (++r >= r1) break;
        const int q = next_comb(nc, M, idx);
        if (q < M - 1 && q <= lead) lead = fit_rows(g, h, q, M - 1, idx, F);
    }
}

// One row of the search.  FIRST: an F row with more than NCAP candidates is
// marked for the second pass; otherwise (NCAP = kSearchCand) such a row is
// left empty with status 4.
template <typename T, int K, int NCAP, bool FIRST>
__device__ void search_row(int i, int lane, SearchLds<T, K, NCAP>& L, const int* __restrict__ rp,
                           const int* __restrict__ ci, const T* __restrict__ av,
                           const int* __restrict__ rpg, const int* __restrict__ cig,
                           const T* __restrict__ X, const double* __restrict__ w,
                           const uint8_t* __restrict__ cf, int cal, double gamma, int target,
                           int* __restrict__ Pcol, double* __restrict__ Pval,
                           double* __restrict__ lsv, int* __restrict__ rstat, unsigned* status) {
    int* pc = Pcol + (size_t)i * cal;
    double* pv = Pval + (size_t)i * cal;
    if (cf[i]) {  // a C point interpolates itself
        if (lane < cal) {
            pc[lane] = lane == 0 ? i : -1;
            pv[lane] = lane == 0 ? 1.0 : 0.0;
        }
        if (lane == 0) {
            lsv[i] = 0.0;
            rstat[i] = 0;
        }
        return;
    }
    // candidates: C points of row i of the pattern, i excluded, in column order
    const int g0 = rpg[i], g1 = rpg[i + 1];
    int nc = 0;
    for (int e0 = g0; e0 < g1; e0 += kWave) {
        const int e = e0 + lane;
        const int j = e < g1 ? cig[e] : -1;
        const bool isc = j >= 0 && j != i && cf[j] != 0;
        const uint64_t bal = __ballot(isc);
        const int pos = nc + __popcll(bal & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
        if (isc && pos < NCAP) L.cand[pos] = j;
        nc += __popcll(bal);
    }
    if (FIRST && nc > NCAP) {
        if (lane == 0) rstat[i] = kSearchMarked;
        return;
    }
    bool over = false;
    if (nc > NCAP) {
        over = true;
        nc = NCAP;
    }
    int st = 0;
    // target (FP64): lane k holds t_k
    if (lane < K) {
        const double wk = w ? w[lane] : 1.0;
        double t = (double)X[(size_t)i * K + lane];
        if (target == AD_TARGET_RESIDUAL) {
            double y = 0.0, d = 0.0;
            for (int e = rp[i]; e < rp[i + 1]; ++e) {
                const int j = ci[e];
                const double a = (double)av[e];
                y = fma(a, (double)X[(size_t)j * K + lane], y);
                if (j == i) d = a;
            }
            if (d != 0.0) t = t - y / d;
            else st = 3;
        }
        L.t[lane] = t;
        L.w[lane] = wk;
    }
    st = __shfl(st, 0, kWave);
    if (st == 3 && lane == 0) flag(status, AD_STAT_ZERO_DIAG);
    wave_sync_lds();
    // candidate rows and the target's functional S = <t, t>_w
    for (int q = lane; q < nc * K; q += kWave) {
        const int a = q / K, k = q % K;
        L.x[a][k] = X[(size_t)L.cand[a] * K + k];
    }
    wave_sync_lds();
    double S = 0.0;
#pragma unroll 4
    for (int k = 0; k < K; ++k) S = fma(L.w[k] * L.t[k], L.t[k], S);
    S = wave_uniform(S);
    // h_a and the Gram matrix of the candidates
    if (lane < nc) {
        double s = 0.0;
#pragma unroll 4
        for (int k = 0; k < K; ++k) s = fma(L.w[k] * (double)L.x[lane][k], L.t[k], s);
        L.h[lane] = s;
    }
    const int npair = nc * (nc + 1) / 2;
    for (int p = lane; p < npair; p += kWave) {
        int a = (int)((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
        while (a * (a + 1) / 2 > p) --a;
        while ((a + 1) * (a + 2) / 2 <= p) ++a;
        const int b = p - a * (a + 1) / 2;
        double s = 0.0;
#pragma unroll 4
        for (int k = 0; k < K; ++k) s = fma(L.w[k] * (double)L.x[a][k], (double)L.x[b][k], s);
        L.g[p] = s;
    }
    wave_sync_lds();

    // best set of each size (its value and rank; rank = total: none fitted)
    // a row past the candidate cap is left empty (status 4)
    const int mmax = over ? 0 : (cal < nc ? cal : nc);
    double bvs[kSearchCal];
    int brs[kSearchCal];
#pragma unroll
    for (int q = 0; q < kSearchCal; ++q) {
        bvs[q] = INFINITY;
        brs[q] = 0x7fffffff;
    }
    // The penalty rule takes size m only below thr_m = (incumbent / S)^(gamma
    // (m - size)) S, where the incumbent is what the scan after this loop
    // holds once it has passed the smaller sizes (run_m, run_v follow it size
    // by size with the same rule); and a set of size m below that can also
    // only lie below prev, the best of the largest smaller size that has one
    // (a superset never fits worse).  So min(prev, thr_m), with a relative
    // slack of 1e-12 against rounding, starts each lane's screen: a set at or
    // above it cannot be taken, and a size none of whose sets gets below it
    // is treated as having none, which changes no choice.
    double prev = INFINITY, run_v = 0.0;
    int run_m = 0;
    for (int m = 1; m <= mmax; ++m) {
        const int total = binom_small(nc, m);
        double cut = prev, thr_rel = 0.0;
        if (run_m > 0) {
            thr_rel = wave_uniform(
                pow_series(S > 0.0 ? run_v / S : 0.0, gamma * (double)(m - run_m)));
            cut = fmin(cut, S * thr_rel * (1.0 + 1e-12));
        }
        double bv = cut;
        int br = total;
        switch (m) {
            case 1: best_of_size<1>(L, S, nc, lane, bv, br); break;
            case 2: best_of_size<2>(L, S, nc, lane, bv, br); break;
            case 3: best_of_size<3>(L, S, nc, lane, bv, br); break;
            default: best_of_size<4>(L, S, nc, lane, bv, br); break;
        }
        // least (value, rank) over the wave: lanes hold increasing rank blocks
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) {
            const double ov = __shfl_xor(bv, o, kWave);
            const int orr = __shfl_xor(br, o, kWave);
            if (ov < bv || (ov == bv && orr < br)) {
                bv = ov;
                br = orr;
            }
        }
        if (br >= total) {
            br = 0x7fffffff;  // every set dependent, or none below the cut: not taken
        } else {
            prev = wave_uniform(bv);
            // the scan's rule (below) for this size: any set found is below thr_m
            if (run_m == 0 || (S > 0.0 ? bv / S : 0.0) < thr_rel) {
                run_m = m;
                run_v = prev;
            }
        }
#pragma unroll
        for (int q = 0; q < kSearchCal; ++q)
            if (q == m - 1) {
                bvs[q] = bv;
                brs[q] = br;
            }
    }
    // the penalty rule: a scan in increasing size against the incumbent
    int inc_m = 0, inc_r = 0;
    double inc_v = 0.0;
#pragma unroll
    for (int q = 0; q < kSearchCal; ++q) {
        const int m = q + 1;
        if (m > mmax || brs[q] == 0x7fffffff) continue;
        bool take = inc_m == 0;
        if (!take) {
            const double rel = S > 0.0 ? bvs[q] / S : 0.0;
            const double inc_rel = S > 0.0 ? inc_v / S : 0.0;
            take = rel < pow_series(inc_rel, gamma * (double)(m - inc_m));
        }
        if (take) {
            inc_m = m;
            inc_v = bvs[q];
            inc_r = brs[q];
        }
    }
    int inc_idx[kSearchCal] = {0, 0, 0, 0};
    if (inc_m > 0) unrank(inc_r, nc, inc_m, inc_idx);

    // the chosen set: weights by its Cholesky solve, functional by definition
    double coef[kSearchCal] = {0.0, 0.0, 0.0, 0.0};
    double val;
    if (inc_m > 0) {
        SetFit F;
        fit_rows(L.g, L.h, 0, inc_m, inc_idx, F);
        fit_coef(F, inc_m, coef);
        double r = 0.0;
        if (lane < K) {
            r = L.t[lane];
#pragma unroll
            for (int a = 0; a < kSearchCal; ++a)
                if (a < inc_m) r -= coef[a] * (double)L.x[inc_idx[a]][lane];
            r = L.w[lane] * r * r;
        }
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) r += __shfl_xor(r, o, kWave);
        val = r;
    } else {
        val = S;
    }
    int mycol = -1;
    double mycoef = 0.0;
#pragma unroll
    for (int a = 0; a < kSearchCal; ++a)
        if (lane == a && a < inc_m) {
            mycol = L.cand[inc_idx[a]];
            mycoef = coef[a];
        }
    if (lane < cal) {
        pc[lane] = mycol;
        pv[lane] = mycoef;
    }
    if (lane == 0) {
        lsv[i] = val;
        rstat[i] = over ? 4 : (inc_m == 0 ? (st ? st : 1) : st);
        if (over) flag(status, AD_STAT_SEARCH_CAP);
    }
    wave_sync_lds();  // the slice is reused by the wavefront's next row
}

// Each wavefront takes a chunk of 64 consecutive rows.  FIRST: every row of
// the chunk; second pass: the chunk's rows marked by the first.
template <typename T, int K, int NCAP, int WAVES, bool FIRST>
__global__ __launch_bounds__(kWave* WAVES) void ls_search_kernel(
    int n, const int* __restrict__ rp, const int* __restrict__ ci, const T* __restrict__ av,
    const int* __restrict__ rpg, const int* __restrict__ cig, const T* __restrict__ X,
    const double* __restrict__ w, const uint8_t* __restrict__ cf, int cal, double gamma,
    int target, int* __restrict__ Pcol, double* __restrict__ Pval, double* __restrict__ lsv,
    int* __restrict__ rstat, unsigned* status) {
    __shared__ SearchLds<T, K, NCAP> L[WAVES];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int64_t i0 = ((int64_t)blockIdx.x * WAVES + wv) * kWave;
    if (i0 >= n) return;  // whole wavefront
    const int i1 = (int)(i0 + kWave < n ? i0 + kWave : n);
    if (FIRST) {
        for (int i = (int)i0; i < i1; ++i)
            search_row<T, K, NCAP, true>(i, lane, L[wv], rp, ci, av, rpg, cig, X, w, cf, cal,
                                         gamma, target, Pcol, Pval, lsv, rstat, status);
    } else {
        const int me = (int)i0 + lane;
        uint64_t marked = __ballot(me < i1 && rstat[me] == kSearchMarked);
        while (marked) {
            const int q = __builtin_ctzll(marked);
            marked &= marked - 1;
            search_row<T, K, NCAP, false>((int)i0 + q, lane, L[wv], rp, ci, av, rpg, cig, X, w,
                                          cf, cal, gamma, target, Pcol, Pval, lsv, rstat, status);
        }
    }
}

template <typename T>
static int ls_search_dispatch(int K, const ad_csr* A, const int* rpg, const int* cig,
                              const void* X, const double* w, const uint8_t* cf, int cal,
                              double gamma, int target, int* Pcol, double* Pval, double* lsv,
                              int* rstat, unsigned* status, hipStream_t s) {
    return with_k<T>(K, [&](auto kc) {
        constexpr int KK = decltype(kc)::value;
        constexpr int W1 = 4, W2 = 1;
        const int64_t chunks = ((int64_t)A->n + kWave - 1) / kWave;
        const unsigned g1 = (unsigned)((chunks + W1 - 1) / W1);
        const unsigned g2 = (unsigned)((chunks + W2 - 1) / W2);
        ls_search_kernel<T, KK, kSearchFast, W1, true><<<dim3(g1), dim3(kWave * W1), 0, s>>>(
            A->n, A->row_ptr, A->col, (const T*)A->val, rpg, cig, (const T*)X, w, cf, cal, gamma,
            target, Pcol, Pval, lsv, rstat, status);
        ls_search_kernel<T, KK, kSearchCand, W2, false><<<dim3(g2), dim3(kWave * W2), 0, s>>>(
            A->n, A->row_ptr, A->col, (const T*)A->val, rpg, cig, (const T*)X, w, cf, cal, gamma,
            target, Pcol, Pval, lsv, rstat, status);
        return (int)AD_OK;
    });
}

int launch_ls_search(int dtype, int K, const ad_csr* A, const int* rpg, const int* cig,
                     const void* X, const double* w, const uint8_t* cf, int caliber, double gamma,
                     int target, int32_t* P_col, double* P_val, double* ls_val,
                     int32_t* row_status, unsigned* status, hipStream_t s) {
    if (A->n == 0) return AD_OK;
    const int rc = (dtype == AD_F32)
                       ? ls_search_dispatch<float>(K, A, rpg, cig, X, w, cf, caliber, gamma,
                                                   target, P_col, P_val, ls_val, row_status,
                                                   status, s)
                       : ls_search_dispatch<double>(K, A, rpg, cig, X, w, cf, caliber, gamma,
                                                    target, P_col, P_val, ls_val, row_status,
                                                    status, s);
    if (rc) return rc;
    AD_HIP(hipGetLastError());
    return AD_OK;
}

}  // namespace ad
