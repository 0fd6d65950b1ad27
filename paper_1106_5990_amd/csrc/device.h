// device.h -- device-side building blocks shared by the libalgdist kernels.
//
// Work mapping used by the per-row kernels: a row of the n x K panel is
// K * sizeof(T) contiguous bytes.  A "row group" of LPR adjacent lanes
// covers one panel row, each lane holding V = K / LPR consecutive entries
// (16-byte chunk loads: float4 or double2), so one wavefront (64 lanes)
// works on RPW = 64 / LPR rows at once and a gathered neighbour row is read
// as LPR * V * sizeof(T) contiguous bytes.  Reductions over K are
// xor-butterflies inside the row group; they leave the identical
// (commutatively equal) sum in every lane of the group.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ad {

constexpr int kWave = 64;
constexpr int kBlock = 256;  // threads per workgroup of the per-row kernels
constexpr int kWavesPerBlock = kBlock / kWave;

// Lanes per row (LPR) is a launch choice: each lane of a row group holds
// V = K / LPR consecutive panel entries, read as 16-byte chunks.  Allowed
// shapes keep V within 64 bytes of registers (16 floats, 8 doubles) and at
// least 8 bytes, and V >= vmax / 4 unless V = K (tiny K).
template <typename T>
constexpr int vmax_of() { return 64 / (int)sizeof(T); }

template <typename T>
constexpr bool lpr_ok(int K, int L) {
    return L >= 1 && L <= kWave && K % L == 0 && (K / L) <= vmax_of<T>() &&
           (K / L) * (int)sizeof(T) >= 8 && ((K / L) >= vmax_of<T>() / 4 || (K / L) == K);
}

// Default LPR before tuning: 32 bytes per lane where the shape allows it.
template <typename T>
constexpr int lpr_default(int K) {
    for (int L = 1; L <= kWave; L *= 2)
        if (lpr_ok<T>(K, L) && (K / L) * (int)sizeof(T) <= 32) return L;
    for (int L = kWave; L >= 1; L /= 2)
        if (lpr_ok<T>(K, L)) return L;
    return 1;
}

template <typename T, int K, int LPR_>
struct Shape {
    static constexpr int LPR = LPR_;                        // lanes per row
    static constexpr int V = K / LPR;                       // entries per lane
    static constexpr int C = (V * (int)sizeof(T) <= 16) ? V : 16 / (int)sizeof(T);  // per load
    static constexpr int RPW = kWave / LPR;                 // rows per wavefront
    static constexpr int RPB = RPW * kWavesPerBlock;        // rows per block step
    static_assert(lpr_ok<T>(K, LPR_), "unsupported lanes-per-row for this K");
    static_assert((LPR & (LPR - 1)) == 0, "LPR must be a power of two");
};

template <typename T, int V>
struct Frag {
    T v[V];
};

// Load V consecutive entries starting at p (p aligned to V * sizeof(T), V a
// power of two with V * sizeof(T) <= 16).
template <typename T, int V>
__device__ __forceinline__ Frag<T, V> load_frag(const T* __restrict__ p) {
    Frag<T, V> f;
    if constexpr (V == 1) {
        f.v[0] = *p;
    } else {
        typedef T vec_t __attribute__((ext_vector_type(V)));
        vec_t x = *reinterpret_cast<const vec_t*>(p);
#pragma unroll
        for (int q = 0; q < V; ++q) f.v[q] = x[q];
    }
    return f;
}

template <typename T, int V>
__device__ __forceinline__ void store_frag(T* __restrict__ p, const Frag<T, V>& f) {
    if constexpr (V == 1) {
        *p = f.v[0];
    } else {
        typedef T vec_t __attribute__((ext_vector_type(V)));
        vec_t x;
#pragma unroll
        for (int q = 0; q < V; ++q) x[q] = f.v[q];
        *reinterpret_cast<vec_t*>(p) = x;
    }
}

// A lane's V entries of a panel row, as V / C chunk loads.
template <typename T, int V, int C>
__device__ __forceinline__ Frag<T, V> load_lane(const T* __restrict__ p) {
    Frag<T, V> f;
#pragma unroll
    for (int c = 0; c < V / C; ++c) {
        Frag<T, C> x = load_frag<T, C>(p + c * C);
#pragma unroll
        for (int q = 0; q < C; ++q) f.v[c * C + q] = x.v[q];
    }
    return f;
}

template <typename T, int V, int C>
__device__ __forceinline__ void store_lane(T* __restrict__ p, const Frag<T, V>& f) {
#pragma unroll
    for (int c = 0; c < V / C; ++c) {
        Frag<T, C> x;
#pragma unroll
        for (int q = 0; q < C; ++q) x.v[q] = f.v[c * C + q];
        store_frag<T, C>(p + c * C, x);
    }
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

// Tile assignment over the 8 XCDs (workgroups are dispatched round-robin:
// block b runs on XCD b % 8, each XCD with its own L2).  mode:
//   0      tile = block index: consecutive tiles on different XCDs;
//   1      XCD x takes the contiguous tile range [x * per, (x + 1) * per);
//   c >= 2 chunks of 8c consecutive tiles, XCD x taking tiles
//          [x * c, (x + 1) * c) of each chunk: neighbouring tiles -- whose
//          panel rows the gathers re-read -- share an L2 while all XCDs work
//          on one region of memory at a time.
// Returns -1 for a workgroup with no tile; the grid is grid_for_tiles(ntiles, mode).
__device__ __forceinline__ int64_t map_tile(int64_t ntiles, int mode) {
    const int64_t b = blockIdx.x;
    int64_t t;
    if (mode <= 0) {
        t = b;
    } else if (mode == 1) {
        const int64_t per = (ntiles + 7) / 8;
        const int64_t q = b / 8;
        if (q >= per) return -1;
        t = (b % 8) * per + q;
    } else {
        const int64_t span = 8 * (int64_t)mode;
        const int64_t r = b % span;
        t = (b - r) + (r % 8) * mode + r / 8;
    }
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
