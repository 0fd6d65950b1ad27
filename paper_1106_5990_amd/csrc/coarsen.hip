// coarsen.hip -- compatible-relaxation coarsening (Sec. 3.2 and Sec. 4.2,
// Algorithm 1): F-relaxation runs, the rate estimate, the candidate set and
// the independent set of the candidates on the strength graph.
//
// F-relaxation (eq:frelax) is the colour-phase Gauss-Seidel of the test
// vectors with every C row given no colour, so it stays at its start value
// 0; F rows start from the constant 1.  The panel has two identical columns
// (the sweep kernels take K >= 2); column 0 is the CR vector.
//
// Rate and candidates (eq:meas1, the remark after Algorithm 1): per-block
// partial sums over F of u^2, the F count and max |u|, reduced in a fixed
// order; rho_f = (sqrt(sum u^2) / sqrt(|F|))^(1/nu) on the host; sigma_i =
// |u_i| / max_F |u| > tol marks the candidates.
//
// Independent set: the greedy maximal set of the candidates in decreasing
// priority (|S_i^T|, h_i, i) on the symmetric closure of the strength graph,
// h_i = splitmix64 output i+1 of the stage's seed.  It is computed by rounds
// of local maxima: an undecided candidate joins when no undecided or chosen
// neighbour outranks it, then undecided neighbours of chosen points drop
// out.  With fixed distinct priorities these rounds choose exactly the
// greedy set (the highest undecided candidate is always a local maximum, and
// a point is dropped only next to a chosen point that outranks it), and the
// in-place state updates are race-free: a point is written only by its own
// thread, and a neighbour read as undecided or as chosen in the same round
// outranks the reader either way.
#include <math.h>

#include <vector>

#include "device.h"
#include "internal.h"

namespace ad {

// fcol[i] = -1 on C (held), color[i] on F; U0 row i = (1, 1) on F, (0, 0) on C.
template <typename T>
__global__ __launch_bounds__(kBlock) void cr_start_kernel(int n, const int* __restrict__ color,
                                                          const uint8_t* __restrict__ cf,
                                                          int* __restrict__ fcol,
                                                          T* __restrict__ U0) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const bool c = cf[i] != 0;
    fcol[i] = c ? -1 : color[i];
    U0[2 * i] = c ? T(0) : T(1);
    U0[2 * i + 1] = c ? T(0) : T(1);
}

constexpr int kNormPer = 4;  // rows per thread in the partial pass

// part[3b .. 3b+2] = (|F|, sum_F u^2, max_F |u|) over block b's rows, u =
// column 0 of U (n x 2).  Fixed order: rows in a thread, then a wave
// butterfly, then the waves in order.
template <typename T>
__global__ __launch_bounds__(kBlock) void cr_norm_partials_kernel(int n,
                                                                  const uint8_t* __restrict__ cf,
                                                                  const T* __restrict__ U,
                                                                  double* __restrict__ part) {
    __shared__ double sh[3][kWavesPerBlock];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    double cnt = 0.0, sq = 0.0, mx = 0.0;
    const int64_t base = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * kNormPer;
#pragma unroll
    for (int q = 0; q < kNormPer; ++q) {
        const int64_t i = base + q;
        if (i < n && !cf[i]) {
            const double u = (double)U[2 * i];
            cnt += 1.0;
            sq += u * u;
            mx = fabs(u) > mx ? fabs(u) : mx;
        }
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        cnt += __shfl_xor(cnt, o, kWave);
        sq += __shfl_xor(sq, o, kWave);
        const double m2 = __shfl_xor(mx, o, kWave);
        mx = m2 > mx ? m2 : mx;
    }
    if (lane == 0) {
        sh[0][wv] = cnt;
        sh[1][wv] = sq;
        sh[2][wv] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0, m = 0.0;
        for (int q = 0; q < kWavesPerBlock; ++q) {
            a += sh[0][q];
            b += sh[1][q];
            m = sh[2][q] > m ? sh[2][q] : m;
        }
        part[3 * blockIdx.x] = a;
        part[3 * blockIdx.x + 1] = b;
        part[3 * blockIdx.x + 2] = m;
    }
}

// out[0..2] from the partials of nb blocks (one workgroup of 1024 threads).
__global__ __launch_bounds__(1024) void cr_norm_final_kernel(int64_t nb,
                                                             const double* __restrict__ part,
                                                             double* __restrict__ out) {
    __shared__ double acc[3][1024];
    const int t = threadIdx.x;
    const int64_t per = (nb + 1023) / 1024;
    double a = 0.0, b = 0.0, m = 0.0;
    for (int64_t q = t * per; q < nb && q < (t + 1) * per; ++q) {
        a += part[3 * q];
        b += part[3 * q + 1];
        m = part[3 * q + 2] > m ? part[3 * q + 2] : m;
    }
    acc[0][t] = a;
    acc[1][t] = b;
    acc[2][t] = m;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (t < o) {
            acc[0][t] += acc[0][t + o];
            acc[1][t] += acc[1][t + o];
            acc[2][t] = acc[2][t + o] > acc[2][t] ? acc[2][t + o] : acc[2][t];
        }
        __syncthreads();
    }
    if (t == 0) {
        out[0] = acc[0][0];
        out[1] = acc[1][0];
        out[2] = acc[2][0];
    }
}

// z_i = 1 for F points with |u_i| / max_F |u| > tol.
template <typename T>
__global__ __launch_bounds__(kBlock) void cr_candidates_kernel(int n,
                                                               const uint8_t* __restrict__ cf,
                                                               const T* __restrict__ U, int stride,
                                                               const double* __restrict__ norms,
                                                               double tol,
                                                               uint8_t* __restrict__ z) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double m = norms[2];
    const double u = (double)U[(int64_t)stride * i];
    z[i] = (uint8_t)(!cf[i] && m > 0.0 && fabs(u) / m > tol);
}

// ---------------------------------------------------------------- independent set
// (lam_j, h_j, j) > (lam_i, h_i, i)
__device__ __forceinline__ bool outranks(int lj, uint64_t hj, int j, int li, uint64_t hi, int i) {
    if (lj != li) return lj > li;
    if (hj != hi) return hj > hi;
    return j > i;
}

// key[i] = (h_i, lam_i = strong entries in column i); state 1 for
// candidates, else 0.
__global__ __launch_bounds__(kBlock) void mis_init_kernel(int n, const int64_t* __restrict__ cp,
                                                          const int* __restrict__ tent,
                                                          const uint8_t* __restrict__ strong,
                                                          const uint8_t* __restrict__ z,
                                                          uint64_t seed, MisKey* __restrict__ key,
                                                          int8_t* __restrict__ state) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int c = 0;
    for (int64_t f = cp[i]; f < cp[i + 1]; ++f) c += strong[tent[f]] != 0;
    MisKey k;
    k.h = splitmix64_at(seed, (uint64_t)i);
    k.lam = c;
    k.pad = 0;
    key[i] = k;
    state[i] = z[i] ? 1 : 0;
}

// Calls f(j) for every neighbour j != i with a strong entry (i, j) or
// (j, i), until f returns true (then true).  With a structurally symmetric
// pattern the k-th entry of column i is (row i's k-th column, i), so both
// directions of an edge are read in one pass over row i.
template <typename F>
__device__ __forceinline__ bool any_strong_neighbour(int i, bool sym, const int* __restrict__ rp,
                                                     const int* __restrict__ ci,
                                                     const uint8_t* __restrict__ strong,
                                                     const int64_t* __restrict__ cp,
                                                     const int* __restrict__ trow,
                                                     const int* __restrict__ tent, F&& f) {
    const int e0 = rp[i], e1 = rp[i + 1];
    if (sym) {
        const int64_t f0 = cp[i];
        for (int e = e0; e < e1; ++e) {
            const int j = ci[e];
            if (j == i || !(strong[e] || strong[tent[f0 + (e - e0)]])) continue;
            if (f(j)) return true;
        }
        return false;
    }
    for (int e = e0; e < e1; ++e) {
        const int j = ci[e];
        if (j == i || !strong[e]) continue;
        if (f(j)) return true;
    }
    for (int64_t g = cp[i]; g < cp[i + 1]; ++g) {
        const int j = trow[g];
        if (j == i || !strong[tent[g]]) continue;
        if (f(j)) return true;
    }
    return false;
}

// An undecided candidate with no undecided or chosen neighbour that
// outranks it is chosen (state 2).  Neighbours: strong (i, j) in row i and
// strong (j, i) in column i, j != i.
__global__ __launch_bounds__(kBlock) void mis_select_kernel(
    int n, const int* __restrict__ rp, const int* __restrict__ ci,
    const uint8_t* __restrict__ strong, const int64_t* __restrict__ cp,
    const int* __restrict__ trow, const int* __restrict__ tent, const int* __restrict__ asym,
    const MisKey* __restrict__ key, int8_t* state) {
    const int64_t i64 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i64 >= n) return;
    const int i = (int)i64;
    if (state[i] != 1) return;
    const MisKey ki = key[i];
    const bool beaten = any_strong_neighbour(i, *asym == 0, rp, ci, strong, cp, trow, tent, [&](int j) {
        if (state[j] == 0) return false;
        const MisKey kj = key[j];
        return outranks(kj.lam, kj.h, j, ki.lam, ki.h, i);
    });
    if (!beaten) state[i] = 2;
}

// Undecided candidates next to a chosen point drop out (state 0); the rest
// are counted into *left.
__global__ __launch_bounds__(kBlock) void mis_drop_kernel(
    int n, const int* __restrict__ rp, const int* __restrict__ ci,
    const uint8_t* __restrict__ strong, const int64_t* __restrict__ cp,
    const int* __restrict__ trow, const int* __restrict__ tent, const int* __restrict__ asym,
    int8_t* state, int* left) {
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    const int64_t i64 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i64 < n && state[i64] == 1) {
        const int i = (int)i64;
        const bool out = any_strong_neighbour(i, *asym == 0, rp, ci, strong, cp, trow, tent,
                                              [&](int j) { return state[j] == 2; });
        if (out) state[i] = 0;
        else atomicAdd(&cnt, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0 && cnt) atomicAdd(left, cnt);
}

// sel[i] = chosen; cf[i] |= chosen (cf may be null); *chosen += the count.
__global__ __launch_bounds__(kBlock) void mis_apply_kernel(int n, const int8_t* __restrict__ state,
                                                           uint8_t* __restrict__ sel,
                                                           uint8_t* __restrict__ cf, int* chosen) {
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) {
        const bool c = state[i] == 2;
        if (sel) sel[i] = (uint8_t)c;
        if (cf && c) cf[i] = 1;
        if (c) atomicAdd(&cnt, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0 && cnt) atomicAdd(chosen, cnt);
}

// fm[i] = 1 on F (cf[i] == 0)
__global__ __launch_bounds__(kBlock) void cr_fmask_kernel(int n, const uint8_t* __restrict__ cf,
                                                          uint8_t* __restrict__ fm) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) fm[i] = (uint8_t)(cf[i] == 0);
}

static unsigned blocks_for(int64_t m, int64_t per) {
    return (unsigned)((m + per - 1) / per > 0 ? (m + per - 1) / per : 1);
}

int cr_norm_blocks(int n) { return (int)blocks_for(n, (int64_t)kBlock * kNormPer); }

int launch_cr_start(int dtype, int n, const int* color, const uint8_t* cf, int* fcol, void* U0,
                    hipStream_t s) {
    if (n == 0) return AD_OK;
    if (dtype == AD_F32)
        cr_start_kernel<float><<<dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s>>>(n, color, cf, fcol,
                                                                                 (float*)U0);
    else
        cr_start_kernel<double><<<dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s>>>(n, color, cf, fcol,
                                                                                  (double*)U0);
    AD_HIP(hipGetLastError());
    return AD_OK;
}

int launch_cr_fmask(int n, const uint8_t* cf, uint8_t* fm, hipStream_t s) {
    if (n == 0) return AD_OK;
    cr_fmask_kernel<<<dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s>>>(n, cf, fm);
    AD_HIP(hipGetLastError());
    return AD_OK;
}

int launch_cr_norms(int dtype, int n, const uint8_t* cf, const void* U, double* part,
                    double* norms, hipStream_t s) {
    const int nb = cr_norm_blocks(n);
    if (dtype == AD_F32)
        cr_norm_partials_kernel<float><<<dim3(nb), dim3(kBlock), 0, s>>>(n, cf, (const float*)U, part);
    else
        cr_norm_partials_kernel<double><<<dim3(nb), dim3(kBlock), 0, s>>>(n, cf, (const double*)U,
                                                                          part);
    cr_norm_final_kernel<<<dim3(1), dim3(1024), 0, s>>>(nb, part, norms);
    AD_HIP(hipGetLastError());
    return AD_OK;
}

int launch_cr_candidates(int dtype, int n, const uint8_t* cf, const void* U, int stride,
                         const double* norms, double tol, uint8_t* z, hipStream_t s) {
    if (n == 0) return AD_OK;
    if (dtype == AD_F32)
        cr_candidates_kernel<float><<<dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s>>>(
            n, cf, (const float*)U, stride, norms, tol, z);
    else
        cr_candidates_kernel<double><<<dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s>>>(
            n, cf, (const double*)U, stride, norms, tol, z);
    AD_HIP(hipGetLastError());
    return AD_OK;
}

// The rounds of the independent set (synchronises the stream once per
// round).  *count receives the size of the set.
int run_independent_set(int n, const int* rp, const int* ci, const uint8_t* strong,
                        const int64_t* cp, const int* trow, const int* tent, const int* asym,
                        const uint8_t* z, uint64_t seed, MisKey* key, int8_t* state, int* left,
                        uint8_t* sel, uint8_t* cf, int64_t* count, hipStream_t s) {
    *count = 0;
    if (n == 0) return AD_OK;
    const unsigned nb = blocks_for(n, kBlock);
    mis_init_kernel<<<dim3(nb), dim3(kBlock), 0, s>>>(n, cp, tent, strong, z, seed, key, state);
    AD_HIP(hipGetLastError());
    // every round chooses the highest undecided candidate, so n rounds bound
    // the loop; the host looks at the count of undecided points after every
    // kMisRounds rounds (rounds after the last one find nothing to do)
    constexpr int kMisRounds = 4;
    for (int64_t round = 0; round <= n; round += kMisRounds) {
        for (int r = 0; r < kMisRounds; ++r) {
            int rc = launch_fill_i32(left, 1, 0, s);
            if (rc) return rc;
            mis_select_kernel<<<dim3(nb), dim3(kBlock), 0, s>>>(n, rp, ci, strong, cp, trow, tent,
                                                                asym, key, state);
            mis_drop_kernel<<<dim3(nb), dim3(kBlock), 0, s>>>(n, rp, ci, strong, cp, trow, tent,
                                                              asym, state, left);
        }
        AD_HIP(hipGetLastError());
        int h_left = 0;
        AD_HIP(hipMemcpyAsync(&h_left, left, sizeof h_left, hipMemcpyDeviceToHost, s));
        AD_HIP(hipStreamSynchronize(s));
        if (h_left == 0) break;
    }
    int rc = launch_fill_i32(left, 1, 0, s);
    if (rc) return rc;
    mis_apply_kernel<<<dim3(nb), dim3(kBlock), 0, s>>>(n, state, sel, cf, left);
    AD_HIP(hipGetLastError());
    int chosen = 0;
    AD_HIP(hipMemcpyAsync(&chosen, left, sizeof chosen, hipMemcpyDeviceToHost, s));
    AD_HIP(hipStreamSynchronize(s));
    *count = chosen;
    return AD_OK;
}

}  // namespace ad
