// relax.hip -- test-vector start and relaxation of A x = 0 over a K-wide
// panel (Sec. 3: test vectors are relaxed solutions of the homogeneous
// system from distinct starts; Sec. 5.2 relaxes them by Gauss-Seidel).
//
// Both relaxations are a CSR row-block SpMM: each row group (LPR lanes, one
// 16-byte fragment per lane) walks its row's nonzeros, gathers the
// neighbour's panel row and accumulates a_ij x_j in the panel type.  The
// matrix is streamed once per sweep; neighbour panel rows are re-read
// through L2 (the tile mapping keeps a row range on one XCD).
#include "device.h"
#include "internal.h"
#include "rowops.h"

namespace ad {

// ---------------------------------------------------------------- start
template <typename T>
__global__ __launch_bounds__(kBlock) void tv_init_kernel(int64_t total, int64_t c0, uint64_t seed,
                                                         T* __restrict__ X) {
    constexpr int E = 16 / sizeof(T);
    const int64_t base = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * E;
    if (base >= total) return;
    Frag<T, E> f;
    uint64_t z = splitmix64_state(seed, (uint64_t)(c0 + base));
#pragma unroll
    for (int q = 0; q < E; ++q, z += kSplitmixGamma) f.v[q] = (T)uniform_pm1(splitmix64_mix(z));
    if (base + E <= total) {
        store_frag<T, E>(X + base, f);
    } else {
        for (int q = 0; q < E && base + q < total; ++q) X[base + q] = f.v[q];
    }
}

int launch_tv_init(int dtype, int64_t row0, int64_t nrows, int K, uint64_t seed, void* X,
                   hipStream_t s) {
    const int64_t total = nrows * K;
    if (total == 0) return AD_OK;
    const int E = dtype == AD_F32 ? 4 : 2;
    const int64_t threads = (total + E - 1) / E;
    const int64_t blocks = (threads + kBlock - 1) / kBlock;
    if (dtype == AD_F32)
        tv_init_kernel<float><<<dim3((unsigned)blocks), dim3(kBlock), 0, s>>>(total, row0 * K, seed,
                                                                              (float*)X);
    else
        tv_init_kernel<double><<<dim3((unsigned)blocks), dim3(kBlock), 0, s>>>(total, row0 * K, seed,
                                                                               (double*)X);
    AD_HIP(hipGetLastError());
    return AD_OK;
}

// ---------------------------------------------------------------- Jacobi
// x_new = x - omega * (A x) / a_ii  (row held fixed if a_ii == 0)
template <typename T, int K, int LPR>
__global__ __launch_bounds__(kBlock) void jacobi_kernel(int n, const int* __restrict__ rp,
                                                        const int* __restrict__ ci,
                                                        const T* __restrict__ av,
                                                        const T* __restrict__ Xin,
                                                        T* __restrict__ Xout, T omega, int iter,
                                                        int xcd, unsigned* status) {
    using S = Shape<T, K, LPR>;
    const int lane = threadIdx.x & (kWave - 1);
    const int g = lane / LPR, l = lane % LPR;
    const int wv = threadIdx.x / kWave;
    const int64_t rows_per_tile = (int64_t)S::RPB * iter;
    const int64_t ntiles = (n + rows_per_tile - 1) / rows_per_tile;
    const int64_t tile = map_tile(ntiles, xcd);
    if (tile < 0 || tile >= ntiles) return;
    __shared__ CsrStage<T> stg;
    for (int it = 0; it < iter; ++it) {
        const int64_t iw = tile * rows_per_tile + (int64_t)it * S::RPB + wv * S::RPW;
        if (iw >= n) break;  // whole wavefront
        const int64_t ie = (iw + S::RPW < n) ? iw + S::RPW : (int64_t)n;
        int64_t a0;
        int cnt;
        wave_lds_sync();
        stage_csr(stg, wv, lane, (int64_t)rp[iw], (int64_t)rp[ie], ci, av, a0, cnt);
        wave_lds_sync();
        const int64_t i64 = iw + g;
        if (i64 >= n) continue;
        jacobi_row_staged<S, T, K>((int)i64, l, rp, ci, av, stg, wv, a0, cnt, Xin, Xout, omega,
                                   status);
    }
}

template <typename T, int K, int LPR>
static void jacobi_go(const ad_csr* A, const void* Xin, void* Xout, double omega, unsigned* st,
                      const LaunchCfg& cfg, hipStream_t s) {
    using S = Shape<T, K, LPR>;
    const int64_t rpt = (int64_t)S::RPB * cfg.iter;
    const int64_t ntiles = (A->n + rpt - 1) / rpt;
    const int grid = grid_for_tiles(ntiles, cfg.xcd_map);
    jacobi_kernel<T, K, LPR><<<dim3(grid), dim3(kBlock), 0, s>>>(
        A->n, A->row_ptr, A->col, (const T*)A->val, (const T*)Xin, (T*)Xout, (T)omega, cfg.iter,
        cfg.xcd_map, st);
}

template <typename T>
static int jacobi_dispatch(int K, const ad_csr* A, const void* Xin, void* Xout, double omega,
                           unsigned* st, const LaunchCfg& cfg, hipStream_t s) {
    return with_k<T>(K, [&](auto kc) {
        constexpr int KK = decltype(kc)::value;
        return with_lpr<T, KK>(cfg.lpr, [&](auto lc) {
            constexpr int L = decltype(lc)::value;
            jacobi_go<T, KK, L>(A, Xin, Xout, omega, st, cfg, s);
        });
    });
}

int launch_jacobi(int dtype, int K, const ad_csr* A, const void* Xin, void* Xout, double omega,
                  unsigned* status, const LaunchCfg& cfg, hipStream_t s) {
    if (A->n == 0) return AD_OK;
    const int rc = (dtype == AD_F32) ? jacobi_dispatch<float>(K, A, Xin, Xout, omega, status, cfg, s)
                                     : jacobi_dispatch<double>(K, A, Xin, Xout, omega, status, cfg, s);
    if (rc) return rc;
    AD_HIP(hipGetLastError());
    return AD_OK;
}

// ---------------------------------------------------------------- colour partition
// Stable partition of the rows by colour: rows of colour 0 first (in index
// order), then colour 1, ..., then rows with an invalid colour.  Three
// launches: per-block class counts (and class sums of the row lengths), one
// exclusive scan of the class-major tables, per-block scatter.  With the
// row lengths the scatter also writes the colour-major row pointers: the
// entries before a permuted row are those of the lower classes plus those
// of the same class's earlier rows, which is the same class-major scan over
// the lengths.  A thread holds kPartR consecutive rows of its block; the
// block works class by class over the classes present in it.
constexpr int kPartR = 4;                       // consecutive rows per thread
constexpr int kPartRows = kPartR * kBlock;      // rows per partition block
constexpr int kMaxColors = 64;

int color_partition_blocks(int n) { return (n + kPartRows - 1) / kPartRows; }

__device__ __forceinline__ int color_class(int c, int nc) {
    return ((unsigned)c < (unsigned)nc) ? c : nc;
}

template <typename U>
__device__ __forceinline__ U wave_incl_scan(U v) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const U t = __shfl_up(v, o, kWave);
        if (lane >= o) v += t;
    }
    return v;
}

// The thread's rows: class (-1 past the end) and, with rp, length.
__device__ __forceinline__ void part_rows(int n, const int* __restrict__ color, int nc,
                                          const int* __restrict__ rp, int (&c)[kPartR],
                                          int (&len)[kPartR]) {
    const int r0 = blockIdx.x * kPartRows + threadIdx.x * kPartR;
    int b[kPartR + 1];
#pragma unroll
    for (int k = 0; k < kPartR; ++k) c[k] = (r0 + k < n) ? color_class(color[r0 + k], nc) : -1;
#pragma unroll
    for (int k = 0; k <= kPartR; ++k) b[k] = (rp && r0 + k <= n) ? rp[r0 + k] : 0;
#pragma unroll
    for (int k = 0; k < kPartR; ++k) len[k] = (c[k] >= 0) ? b[k + 1] - b[k] : 0;
}

// Marks the classes present in the block (present[0 .. nc] zeroed by the
// caller and synchronised).
__device__ __forceinline__ void part_mark(const int (&c)[kPartR], int* present) {
#pragma unroll
    for (int k = 0; k < kPartR; ++k)
        if (c[k] >= 0) present[c[k]] = 1;
}

// Exclusive scan over the workgroup of a packed (count | length << 32)
// value; returns the thread's exclusive prefix and sets tot to the total.
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t v, uint64_t* wtot, uint64_t& tot) {
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const uint64_t incl = wave_incl_scan(v);
    if (lane == kWave - 1) wtot[wv] = incl;
    __syncthreads();
    uint64_t off = incl - v;
    tot = 0;
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) {
        const uint64_t x = wtot[w];
        off += (w < wv) ? x : 0;
        tot += x;
    }
    __syncthreads();
    return off;
}

__device__ __forceinline__ uint64_t pack_cl(int cnt, int len) {
    return (uint64_t)(uint32_t)cnt | ((uint64_t)(uint32_t)len << 32);
}

// counts[q * nblocks + b]: rows of class q in block b; with rp, lens at
// counts + (nc + 1) * nblocks: their total row length.
__global__ __launch_bounds__(kBlock) void color_count_kernel(int n, const int* __restrict__ color,
                                                             int nc, const int* __restrict__ rp,
                                                             int* __restrict__ counts,
                                                             int nblocks) {
    __shared__ int present[kMaxColors + 1];
    __shared__ uint64_t wtot[kWavesPerBlock];
    for (int q = threadIdx.x; q <= nc; q += kBlock) present[q] = 0;
    int c[kPartR], len[kPartR];
    part_rows(n, color, nc, rp, c, len);
    __syncthreads();
    part_mark(c, present);
    __syncthreads();
    int* lens = counts + (size_t)(nc + 1) * nblocks;
    for (int q = 0; q <= nc; ++q) {
        if (!present[q]) {  // block-uniform
            if (threadIdx.x == 0) {
                counts[(size_t)q * nblocks + blockIdx.x] = 0;
                if (rp) lens[(size_t)q * nblocks + blockIdx.x] = 0;
            }
            continue;
        }
        int tc = 0, tl = 0;
#pragma unroll
        for (int k = 0; k < kPartR; ++k)
            if (c[k] == q) {
                ++tc;
                tl += len[k];
            }
        uint64_t tot;
        (void)block_excl_scan(pack_cl(tc, tl), wtot, tot);
        if (threadIdx.x == 0) {
            counts[(size_t)q * nblocks + blockIdx.x] = (int)(uint32_t)tot;
            if (rp) lens[(size_t)q * nblocks + blockIdx.x] = (int)(tot >> 32);
        }
    }
}

// Exclusive scans of the class-major tables counts[0 .. m) and (with lens)
// counts[m .. 2m) by one workgroup of 1024 threads, both in one pass: a
// thread's contiguous run (loads of kScanRun values in flight together, as
// 16-byte loads when both tables are 16-byte aligned and the run is whole;
// kept in registers) is summed, the run sums (count in the low, length in
// the high 32 bits of one 64-bit value: neither field can carry, both
// totals being below 2^31) are scanned across the workgroup, and the run is
// rewritten.  seg[q] = scanned count at q * nblocks, seg[nc + 1] = n, and
// with the lengths rpp[n] = their total.
constexpr int kScanRun = 8;

__global__ __launch_bounds__(1024) void scan_counts_kernel(int* __restrict__ counts, int m,
                                                           int nblocks, int nc, int n,
                                                           int* __restrict__ seg, int with_lens,
                                                           int* __restrict__ rpp) {
    __shared__ uint64_t wtot[1024 / kWave];
    const int t = threadIdx.x, lane = t & (kWave - 1), wv = t / kWave;
    int* lens = counts + m;
    const bool vec_ok = (((uintptr_t)counts | (uintptr_t)lens) & 15) == 0;
    uint64_t carry = 0;
    // rounds of 1024 * kScanRun entries; thread t takes a contiguous run
    for (int r0 = 0; r0 < m; r0 += 1024 * kScanRun) {
        const int b = r0 + t * kScanRun;
        int vc[kScanRun], vl[kScanRun];
        if (vec_ok && b + kScanRun <= m) {
            typedef int int4v __attribute__((ext_vector_type(4)));
#pragma unroll
            for (int k = 0; k < kScanRun; k += 4) {
                const int4v c4 = *reinterpret_cast<const int4v*>(counts + b + k);
                const int4v l4 = with_lens ? *reinterpret_cast<const int4v*>(lens + b + k)
                                           : int4v{0, 0, 0, 0};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    vc[k + q] = c4[q];
                    vl[k + q] = l4[q];
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < kScanRun; ++k) {
                vc[k] = (b + k < m) ? counts[b + k] : 0;
                vl[k] = (with_lens && b + k < m) ? lens[b + k] : 0;
            }
        }
        uint64_t run = 0;
#pragma unroll
        for (int k = 0; k < kScanRun; ++k) run += pack_cl(vc[k], vl[k]);
        const uint64_t incl = wave_incl_scan(run);
        if (lane == kWave - 1) wtot[wv] = incl;
        __syncthreads();
        uint64_t off = carry + incl - run, tot = 0;
        for (int w = 0; w < 1024 / kWave; ++w) {
            const uint64_t x = wtot[w];
            off += (w < wv) ? x : 0;
            tot += x;
        }
        int oc = (int)(uint32_t)off, ol = (int)(off >> 32);
#pragma unroll
        for (int k = 0; k < kScanRun; ++k)
            if (b + k < m) {
                counts[b + k] = oc;
                oc += vc[k];
                if (with_lens) {
                    lens[b + k] = ol;
                    ol += vl[k];
                }
            }
        carry += tot;
        __syncthreads();
    }
    if (with_lens && t == 0) rpp[n] = (int)(carry >> 32);
    for (int q = t; q <= nc; q += 1024) seg[q] = counts[(size_t)q * nblocks];
    if (t == 0) seg[nc + 1] = n;
}

// Stable positions and (with rp) entry offsets: per class present in the
// block, one workgroup scan of the threads' (count, length) gives each
// thread's start, and its rows of that class follow in order.  A position
// outside [0, n) is dropped and flagged instead of written.
__global__ __launch_bounds__(kBlock) void color_scatter_kernel(
    int n, const int* __restrict__ color, int nc, const int* __restrict__ rp,
    const int* __restrict__ offsets, int nblocks, int* __restrict__ rowlist,
    int* __restrict__ inv, int* __restrict__ rpp, unsigned* status) {
    __shared__ int present[kMaxColors + 1];
    __shared__ uint64_t wtot[kWavesPerBlock];
    const bool with_rp = rpp != nullptr;
    for (int q = threadIdx.x; q <= nc; q += kBlock) present[q] = 0;
    int c[kPartR], len[kPartR];
    part_rows(n, color, nc, with_rp ? rp : nullptr, c, len);
    __syncthreads();
    part_mark(c, present);
    __syncthreads();
    const int* loff = offsets + (size_t)(nc + 1) * nblocks;
    const int r0 = blockIdx.x * kPartRows + threadIdx.x * kPartR;
    bool bad = false, oob = false;
#pragma unroll
    for (int k = 0; k < kPartR; ++k) bad |= (c[k] == nc);
    for (int q = 0; q <= nc; ++q) {
        if (!present[q]) continue;  // block-uniform
        int tc = 0, tl = 0;
#pragma unroll
        for (int k = 0; k < kPartR; ++k)
            if (c[k] == q) {
                ++tc;
                tl += len[k];
            }
        uint64_t tot;
        const uint64_t ex = block_excl_scan(pack_cl(tc, tl), wtot, tot);
        int pos = offsets[(size_t)q * nblocks + blockIdx.x] + (int)(uint32_t)ex;
        int off = with_rp ? loff[(size_t)q * nblocks + blockIdx.x] + (int)(ex >> 32) : 0;
#pragma unroll
        for (int k = 0; k < kPartR; ++k)
            if (c[k] == q) {
                if (pos >= 0 && pos < n) {
                    rowlist[pos] = r0 + k;
                    if (inv) inv[r0 + k] = pos;
                    if (with_rp) rpp[pos] = off;
                } else {
                    oob = true;
                }
                ++pos;
                off += len[k];
            }
    }
    // an out-of-range position can only come from colours that changed
    // between the count and scatter launches
    if (bad || oob) flag(status, AD_STAT_BAD_COLOR);
}

int launch_color_partition(int n, const int32_t* color, int ncolors, const int32_t* rp,
                           int32_t* rowlist, int32_t* inv, int32_t* seg, int32_t* counts,
                           int nblocks, int32_t* rpp, unsigned* status, hipStream_t s) {
    if (n == 0) {
        int rc = launch_fill_i32(seg, ncolors + 2, 0, s);
        if (!rc && rpp) rc = launch_fill_i32(rpp, 1, 0, s);
        return rc;
    }
    const int* rpu = rpp ? rp : nullptr;
    color_count_kernel<<<dim3(nblocks), dim3(kBlock), 0, s>>>(n, color, ncolors, rpu, counts,
                                                              nblocks);
    scan_counts_kernel<<<dim3(1), dim3(1024), 0, s>>>(counts, (ncolors + 1) * nblocks, nblocks,
                                                      ncolors, n, seg, rpp ? 1 : 0, rpp);
    color_scatter_kernel<<<dim3(nblocks), dim3(kBlock), 0, s>>>(
        n, color, ncolors, rpu, counts, nblocks, rowlist, inv, rpp, status);
    AD_HIP(hipGetLastError());
    return AD_OK;
}

// ---------------------------------------------------------------- colour-major layout
// The colour phases run on panels stored colour-major: permuted row p holds
// natural row rowlist[p], so the rows of one colour are contiguous and every
// cache line a phase touches holds rows it needs.  A neighbour's permuted
// index jp is read from colp[e] = inv[col[e]]; "smaller colour" is jp <
// seg[c] because the segments are in colour order.  Permuted row p holds the
// entries of natural row rowlist[p] in their CSR order (row pointers from
// the partition), columns mapped to permuted indices.

// Entry copy in natural order, one wavefront per kCopyRows natural rows:
// the rows' natural and permuted entry starts go to LDS, then the wave
// walks the rows' natural entry range kWave entries at a time (contiguous
// loads; each row's entries land as one contiguous run, and rows that are
// neighbours in a colour are neighbours in the copy); a lane finds the row
// of its entry by binary search over the starts.  colpp = inv[col],
// valpp = val.  With Xp (K * sizeof(T) >= 16), the wavefront also writes the
// hash start rows of its natural rows at their permuted positions, the same
// values start_perm_kernel forms, so that the start's integer work overlaps
// the copy's memory traffic instead of running as a launch of its own.
constexpr int kCopyRows = 64;
constexpr int kPermUnroll = 4;

template <typename T>
__global__ __launch_bounds__(kBlock) void permute_entries_kernel(
    int n, const int* __restrict__ rp, const int* __restrict__ ci, const T* __restrict__ av,
    const int* __restrict__ inv, const int* __restrict__ rpp, int* __restrict__ colpp,
    T* __restrict__ valpp, int K, uint64_t seed, T* __restrict__ Xp) {
    __shared__ int s_rp[kWavesPerBlock][kCopyRows + 1];  // natural starts, then the end
    __shared__ int s_dst[kWavesPerBlock][kCopyRows];     // permuted starts
    __shared__ int s_inv[kWavesPerBlock][kCopyRows];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int64_t r0 = ((int64_t)blockIdx.x * kWavesPerBlock + wv) * kCopyRows;
    const int rl = r0 < n ? (int)min<int64_t>(kCopyRows, n - r0) : 0;
    if (lane < rl) {
        s_rp[wv][lane] = rp[r0 + lane];
        s_inv[wv][lane] = inv[r0 + lane];
        s_dst[wv][lane] = rpp[s_inv[wv][lane]];
    }
    if (lane == 0 && rl > 0) s_rp[wv][rl] = rp[r0 + rl];
    __syncthreads();
    if (rl == 0) return;
    const int b = s_rp[wv][0], e = s_rp[wv][rl];
    // kPermUnroll chunks per pass: their loads, searches and inv gathers are
    // independent and in flight together
    for (int q0 = b + lane; q0 < e; q0 += kWave * kPermUnroll) {
        int cc[kPermUnroll], dd[kPermUnroll], jj[kPermUnroll];
        T vv[kPermUnroll];
#pragma unroll
        for (int u = 0; u < kPermUnroll; ++u) {
            const int q = q0 + u * kWave;
            cc[u] = (q < e) ? ci[q] : 0;
            vv[u] = (q < e) ? av[q] : T(0);
        }
#pragma unroll
        for (int u = 0; u < kPermUnroll; ++u) {
            const int q = q0 + u * kWave;
            int lo = 0;  // last row whose start is <= q
#pragma unroll
            for (int st = kCopyRows / 2; st > 0; st >>= 1) {
                const int mid = lo + st;
                if (mid < rl && s_rp[wv][mid] <= q) lo = mid;
            }
            dd[u] = s_dst[wv][lo] + (q - s_rp[wv][lo]);
        }
#pragma unroll
        for (int u = 0; u < kPermUnroll; ++u) jj[u] = (q0 + u * kWave < e) ? inv[cc[u]] : 0;
#pragma unroll
        for (int u = 0; u < kPermUnroll; ++u)
            if (q0 + u * kWave < e) {
                colpp[dd[u]] = jj[u];
                valpp[dd[u]] = vv[u];
            }
    }
    if (Xp) {
        // the start rows of these natural rows at their permuted positions
        constexpr int E = 16 / sizeof(T);
        const int cpr = K / E;  // chunks per row (K >= E here)
        for (int q = lane; q < rl * cpr; q += kWave) {
            const int r = q / cpr, k0 = (q % cpr) * E;
            const int64_t nat = r0 + r;
            uint64_t z = splitmix64_state(seed, (uint64_t)(nat * K + k0));
            Frag<T, E> f;
#pragma unroll
            for (int u = 0; u < E; ++u, z += kSplitmixGamma)
                f.v[u] = (T)uniform_pm1(splitmix64_mix(z));
            store_frag<T, E>(Xp + (int64_t)s_inv[wv][r] * K + k0, f);
        }
    }
}

// Xp[p] = hash start of natural row rowlist[p] (or X0[rowlist[p]] if given).
// A thread writes kStartChunks 16-byte chunks, chunk h of every thread of
// the block at consecutive addresses, so each store instruction of a wave
// fills whole cache lines; the row-list loads of a thread are issued
// together.  K is a power of two: row and column of a panel value come from
// shifts.
constexpr int kStartChunks = 8;
template <typename T>
constexpr int kStartLog2E = (sizeof(T) == 4) ? 2 : 1;  // log2 of the values per chunk

template <typename T>
__global__ __launch_bounds__(kBlock) void start_perm_kernel(int64_t total, int kshift,
                                                            const int* __restrict__ rowlist,
                                                            uint64_t seed, const T* __restrict__ X0,
                                                            T* __restrict__ Xp) {
    constexpr int E = 16 / sizeof(T);
    const int64_t kmask = ((int64_t)1 << kshift) - 1;
    // a chunk's values lie in one panel row when K >= E (a launch-wide
    // condition): its source run is contiguous and the hash state is formed
    // once and stepped by one counter
    const bool one_row = kshift >= kStartLog2E<T>;
    int64_t o[kStartChunks], s0[kStartChunks];
#pragma unroll
    for (int h = 0; h < kStartChunks; ++h) {
        o[h] = (((int64_t)blockIdx.x * kStartChunks + h) * kBlock + threadIdx.x) * E;
        const int64_t c = o[h] < total ? o[h] : total - 1;
        s0[h] = ((int64_t)rowlist[c >> kshift] << kshift) | (c & kmask);
    }
#pragma unroll
    for (int h = 0; h < kStartChunks; ++h) {
        if (o[h] >= total) break;
        Frag<T, E> f;
        if (one_row) {
            if (X0) {
#pragma unroll
                for (int q = 0; q < E; ++q) f.v[q] = X0[s0[h] + q];
            } else {
                uint64_t z = splitmix64_state(seed, (uint64_t)s0[h]);
#pragma unroll
                for (int q = 0; q < E; ++q, z += kSplitmixGamma)
                    f.v[q] = (T)uniform_pm1(splitmix64_mix(z));
            }
        } else {
#pragma unroll
            for (int q = 0; q < E; ++q) {
                const int64_t c = o[h] + q < total ? o[h] + q : total - 1;
                const int64_t sq = ((int64_t)rowlist[c >> kshift] << kshift) | (c & kmask);
                f.v[q] = X0 ? X0[sq] : (T)uniform_pm1(splitmix64_at(seed, (uint64_t)sq));
            }
        }
        if (o[h] + E <= total) {
            store_frag<T, E>(Xp + o[h], f);
        } else {
            for (int q = 0; q < E && o[h] + q < total; ++q) Xp[o[h] + q] = f.v[q];
        }
    }
}

// X[rowlist[p]] = Xp[p]
template <typename T>
__global__ __launch_bounds__(kBlock) void unpermute_kernel(int64_t total, int kshift,
                                                           const int* __restrict__ rowlist,
                                                           const T* __restrict__ Xp,
                                                           T* __restrict__ X) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= total) return;
    const int64_t kmask = ((int64_t)1 << kshift) - 1;
    X[((int64_t)rowlist[c >> kshift] << kshift) | (c & kmask)] = Xp[c];
}

static int log2_of(int K) {
    int s = 0;
    while ((1 << s) < K) ++s;
    return s;
}

// One colour phase in the permuted layout.  Rows p in [seg[c], seg[c+1]):
//   x_new = x - (A z) / a_ii,  z_jp = Xnew_p[jp] if jp < seg[c] else Xold_p[jp].
// Xnew_p receives the row when write_perm; Xnat (if not null) receives it at
// its natural position (the last sweep writes the caller's output directly).
// The phase of colour 0 also carries the held rows (invalid colour).
template <typename T, int K, int LPR>
__global__ __launch_bounds__(kBlock) void gs_phase_perm_kernel(
    const int* __restrict__ rpp, const int* __restrict__ colpp, const T* __restrict__ valpp, int c,
    int nc, const int* __restrict__ rowlist, const int* __restrict__ seg,
    const T* __restrict__ Xold, T* __restrict__ Xnew, T* __restrict__ Xnat, int write_perm,
    int iter, int xcd, unsigned* status) {
    using S = Shape<T, K, LPR>;
    constexpr int V = S::V, C = S::C;
    const int lane = threadIdx.x & (kWave - 1);
    const int g = lane / LPR, l = lane % LPR;
    const int wv = threadIdx.x / kWave;
    const int b0 = seg[c], b1 = seg[c + 1];
    const int64_t rows_per_tile = (int64_t)S::RPB * iter;
    const int64_t ntiles = (b1 - b0 + rows_per_tile - 1) / rows_per_tile;
    const int64_t tile = map_tile(ntiles, xcd);
    __shared__ CsrStage<T> stg;
    if (tile >= 0 && tile < ntiles) {
        for (int it = 0; it < iter; ++it) {
            const int64_t pw = b0 + tile * rows_per_tile + (int64_t)it * S::RPB + wv * S::RPW;
            if (pw >= b1) break;  // whole wavefront
            const int64_t pe = (pw + S::RPW < b1) ? pw + S::RPW : (int64_t)b1;
            int64_t s0;
            int cnt;
            wave_lds_sync();
            stage_csr(stg, wv, lane, (int64_t)rpp[pw], (int64_t)rpp[pe], colpp, valpp, s0, cnt);
            wave_lds_sync();
            const int64_t p = pw + g;
            if (p >= b1) continue;
            T y[V], d;
            Frag<T, V> xi;
            row_spmm_staged<S, T, K>(
                (int)p, rpp[p], rpp[p + 1], stg, wv, s0, cnt, colpp, valpp, l,
                [&](int jp) { return (jp < b0) ? (const T*)Xnew : Xold; }, y, d, xi);
            Frag<T, V> out;
            if (d == T(0)) {
                out = load_lane<T, V, C>(Xold + (size_t)p * K + l * V);
                if (l == 0) flag(status, AD_STAT_ZERO_DIAG);
            } else {
#pragma unroll
                for (int q = 0; q < V; ++q) out.v[q] = xi.v[q] - y[q] / d;
            }
            if (write_perm) store_lane<T, V, C>(Xnew + (size_t)p * K + l * V, out);
            if (Xnat) store_lane<T, V, C>(Xnat + (size_t)rowlist[p] * K + l * V, out);
        }
    }
    if (c == 0) {  // rows with an invalid colour are held fixed
        const int q0 = seg[nc], q1 = seg[nc + 1];
        const int64_t stride = (int64_t)gridDim.x * S::RPB;
        for (int64_t p = q0 + (int64_t)blockIdx.x * S::RPB + wv * S::RPW + g; p < q1; p += stride) {
            const Frag<T, V> v = load_lane<T, V, C>(Xold + (size_t)p * K + l * V);
            store_lane<T, V, C>(Xnew + (size_t)p * K + l * V, v);
            if (Xnat) store_lane<T, V, C>(Xnat + (size_t)rowlist[p] * K + l * V, v);
        }
    }
}

template <typename T, int K, int LPR>
static void gsp_go(const PermCsr& P, int c, int nc, const void* Xold, void* Xnew, void* Xnat,
                   int write_perm, unsigned* st, const LaunchCfg& cfg, hipStream_t s) {
    using S = Shape<T, K, LPR>;
    const int64_t rpt = (int64_t)S::RPB * cfg.iter;
    const int64_t ntiles = (P.n + rpt - 1) / rpt;
    const int grid = grid_for_tiles(ntiles, cfg.xcd_map);
    gs_phase_perm_kernel<T, K, LPR><<<dim3(grid), dim3(kBlock), 0, s>>>(
        P.rpp, P.colpp, (const T*)P.valpp, c, nc, P.rowlist, P.seg, (const T*)Xold, (T*)Xnew,
        (T*)Xnat, write_perm, cfg.iter, cfg.xcd_map, st);
}

template <typename T>
static int gsp_dispatch(int K, const PermCsr& P, int c, int nc, const void* Xold, void* Xnew,
                        void* Xnat, int write_perm, unsigned* st, const LaunchCfg& cfg,
                        hipStream_t s) {
    return with_k<T>(K, [&](auto kc) {
        constexpr int KK = decltype(kc)::value;
        return with_lpr<T, KK>(cfg.lpr, [&](auto lc) {
            constexpr int L = decltype(lc)::value;
            gsp_go<T, KK, L>(P, c, nc, Xold, Xnew, Xnat, write_perm, st, cfg, s);
        });
    });
}

int launch_gs_phase_perm(int dtype, int K, const PermCsr& P, int c, int ncolors, const void* Xold,
                         void* Xnew, void* Xnat, int write_perm, unsigned* status,
                         const LaunchCfg& cfg, hipStream_t s) {
    if (P.n == 0) return AD_OK;
    const int rc = (dtype == AD_F32)
                       ? gsp_dispatch<float>(K, P, c, ncolors, Xold, Xnew, Xnat, write_perm,
                                             status, cfg, s)
                       : gsp_dispatch<double>(K, P, c, ncolors, Xold, Xnew, Xnat, write_perm,
                                              status, cfg, s);
    if (rc) return rc;
    AD_HIP(hipGetLastError());
    return AD_OK;
}

// The colour-major entries of P (whose rowlist, row pointers and inverse inv
// the partition wrote); with Xp, also the hash start panel (seed, K columns)
// in colour-major row order.
int launch_perm_setup(int dtype, const ad_csr* A, PermCsr& P, int32_t* inv, hipStream_t s,
                      int K, uint64_t seed, void* Xp) {
    const int n = A->n;
    if (n == 0) return AD_OK;
    const int64_t rows_per_block = (int64_t)kCopyRows * kWavesPerBlock;
    const unsigned cb = (unsigned)((n + rows_per_block - 1) / rows_per_block);
    if (dtype == AD_F32)
        permute_entries_kernel<float><<<dim3(cb), dim3(kBlock), 0, s>>>(
            n, A->row_ptr, A->col, (const float*)A->val, inv, P.rpp, (int32_t*)P.colpp,
            (float*)P.valpp, K, seed, (float*)Xp);
    else
        permute_entries_kernel<double><<<dim3(cb), dim3(kBlock), 0, s>>>(
            n, A->row_ptr, A->col, (const double*)A->val, inv, P.rpp, (int32_t*)P.colpp,
            (double*)P.valpp, K, seed, (double*)Xp);
    AD_HIP(hipGetLastError());
    return AD_OK;
}

int launch_start_perm(int dtype, int n, int K, const int32_t* rowlist, uint64_t seed,
                      const void* X0, void* Xp, hipStream_t s) {
    const int64_t m = (int64_t)n * K;
    if (m == 0) return AD_OK;
    const int64_t per_block = (int64_t)(dtype == AD_F32 ? 4 : 2) * kStartChunks * kBlock;
    const unsigned b = (unsigned)((m + per_block - 1) / per_block);
    if (dtype == AD_F32)
        start_perm_kernel<float><<<dim3(b), dim3(kBlock), 0, s>>>(m, log2_of(K), rowlist, seed,
                                                                  (const float*)X0, (float*)Xp);
    else
        start_perm_kernel<double><<<dim3(b), dim3(kBlock), 0, s>>>(m, log2_of(K), rowlist, seed,
                                                                   (const double*)X0, (double*)Xp);
    AD_HIP(hipGetLastError());
    return AD_OK;
}

int launch_unpermute(int dtype, int n, int K, const int32_t* rowlist, const void* Xp, void* X,
                     hipStream_t s) {
    const int64_t m = (int64_t)n * K;
    if (m == 0) return AD_OK;
    const unsigned b = (unsigned)((m + kBlock - 1) / kBlock);
    if (dtype == AD_F32)
        unpermute_kernel<float><<<dim3(b), dim3(kBlock), 0, s>>>(m, log2_of(K), rowlist,
                                                                 (const float*)Xp, (float*)X);
    else
        unpermute_kernel<double><<<dim3(b), dim3(kBlock), 0, s>>>(m, log2_of(K), rowlist,
                                                                  (const double*)Xp, (double*)X);
    AD_HIP(hipGetLastError());
    return AD_OK;
}

}  // namespace ad
