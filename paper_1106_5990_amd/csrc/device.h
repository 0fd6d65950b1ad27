// device.h -- device-side building blocks shared by the libalgdist kernels.
//
// Work mapping used by every per-row kernel: a row of the n x K panel is
// K * sizeof(T) contiguous bytes.  A "row group" of LPR lanes covers one
// panel row, each lane holding V = min(K, 16 / sizeof(T)) consecutive
// entries (one 16-byte load: float4 or double2), so one wavefront (64
// lanes) works on RPW = 64 / LPR rows at once and a gathered neighbour row
// is read as one fully used 16-byte-per-lane request.  Reductions over K
// are xor-butterflies inside the row group; they leave the identical
// (commutatively equal) sum in every lane of the group.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ad {

constexpr int kWave = 64;
constexpr int kBlock = 256;  // threads per workgroup of the per-row kernels
constexpr int kWavesPerBlock = kBlock / kWave;

template <typename T> struct MaxVec;
template <> struct MaxVec<float> { static constexpr int v = 4; };
template <> struct MaxVec<double> { static constexpr int v = 2; };

template <typename T, int K>
struct Shape {
    static constexpr int V = (K < MaxVec<T>::v) ? K : MaxVec<T>::v;  // entries per lane
    static constexpr int LPR = K / V;                                  // lanes per row
    static constexpr int RPW = kWave / LPR;                            // rows per wavefront
    static constexpr int RPB = RPW * kWavesPerBlock;                   // rows per block step
    static_assert(K % V == 0 && (LPR & (LPR - 1)) == 0, "K must be a power of two");
};

template <typename T, int V>
struct Frag {
    T v[V];
};

// Load V consecutive entries starting at p (p aligned to V * sizeof(T)).
template <typename T, int V>
__device__ __forceinline__ Frag<T, V> load_frag(const T* __restrict__ p) {
    Frag<T, V> f;
    typedef T vec_t __attribute__((ext_vector_type(V)));
    vec_t x = *reinterpret_cast<const vec_t*>(p);
#pragma unroll
    for (int q = 0; q < V; ++q) f.v[q] = x[q];
    return f;
}

template <typename T, int V>
__device__ __forceinline__ void store_frag(T* __restrict__ p, const Frag<T, V>& f) {
    typedef T vec_t __attribute__((ext_vector_type(V)));
    vec_t x;
#pragma unroll
    for (int q = 0; q < V; ++q) x[q] = f.v[q];
    *reinterpret_cast<vec_t*>(p) = x;
}

// Sum over the LPR lanes of a row group (groups are aligned lane ranges).
template <int LPR, typename U>
__device__ __forceinline__ U group_sum(U x) {
#pragma unroll
    for (int o = LPR / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
    return x;
}

template <int LPR, typename U>
__device__ __forceinline__ U group_min(U x) {
#pragma unroll
    for (int o = LPR / 2; o > 0; o >>= 1) {
        U y = __shfl_xor(x, o, kWave);
        x = (y < x) ? y : x;
    }
    return x;
}

// XCD-aware tile assignment.  Workgroups are dispatched round-robin over the
// 8 XCDs (blockIdx % 8), each XCD with its own L2.  Give XCD x the contiguous
// tile range [x * per, (x + 1) * per) so that neighbouring rows -- whose
// panel rows the gathers re-read -- stay in one L2.  Returns -1 for a
// workgroup with no tile.  The grid must hold >= 8 * ceil(ntiles / 8) blocks.
__device__ __forceinline__ int64_t xcd_tile(int64_t ntiles) {
    const int64_t per = (ntiles + 7) / 8;
    const int64_t b = blockIdx.x;
    const int64_t q = b / 8;
    if (q >= per) return -1;
    const int64_t t = (b % 8) * per + q;
    return (t < ntiles) ? t : -1;
}

__device__ __forceinline__ void flag(unsigned* status, unsigned bit) {
    atomicOr(status, bit);
}

// splitmix64 (Steele, Lea, Flood 2014): state += 0x9e3779b97f4a7c15, then
// the xor-shift-multiply finaliser.  Output number c + 1 of the generator
// seeded with s is finalise(s + (c + 1) * gamma).
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t c) {
    uint64_t z = seed + (c + 1ull) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double uniform_pm1(uint64_t z) {
    return 2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0;
}

}  // namespace ad
