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

// v itself, as a value the compiler cannot see through: conversions of it
// are formed where they are used instead of being hoisted and kept live.
template <typename T>
__device__ __forceinline__ T opaque(T v) {
    asm volatile("" : "+v"(v));
    return v;
}

// An FP64 value as the FP32 path carries it: its FP32 rounding plus the
// FP32 rounding of the remainder (48 significant bits, relative error at
// most 2^-48); the value itself on the FP64 path.
template <typename T>
__device__ __forceinline__ double carried(double x) {
    if constexpr (sizeof(T) == 8) {
        return x;
    } else {
        const T hi = (T)x;
        return (double)hi + (double)(T)(x - (double)hi);
    }
}

// 1/sqrt(x) for x > 0 in FP64: the hardware estimate refined by two Newton
// steps y <- y + y (1/2 - (x/2) y^2) (each doubles the correct bits), within
// a few ulps of the correctly rounded value; tiny x (where the estimate
// may flush) takes the division.
__device__ __forceinline__ double rsqrt_fp64(double x) {
    if (x < 0x1p-1000) return 1.0 / sqrt(x);
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    y = fma(y, fma(-hx * y, y, 0.5), y);
    y = fma(y, fma(-hx * y, y, 0.5), y);
    return y;
}

// The value of partner lane i ^ m(O) for a butterfly level of offset O.
// Inside a 16-lane row the exchange is a DPP move (no LDS round trip):
// O = 1, 2 swap lanes within a quad (m = 1, 2), O = 4 mirrors each 8-lane
// half (m = 7), O = 8 mirrors the row (m = 15); larger offsets use the
// cross-lane permute (m = O).  The masks of any run O = LPR/2, ..., 1 span
// the group's lane indices, so the butterfly reaches every lane, and at each
// level a lane and its partner add the same two values: every lane of the
// group ends with the bitwise identical result.
template <int O>
__device__ __forceinline__ int lane_swap_i32(int x) {
    if constexpr (O == 1) return __builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, true);  // [1,0,3,2]
    else if constexpr (O == 2) return __builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, true);  // [2,3,0,1]
    else if constexpr (O == 4) return __builtin_amdgcn_mov_dpp(x, 0x141, 0xF, 0xF, true);  // half mirror
    else if constexpr (O == 8) return __builtin_amdgcn_mov_dpp(x, 0x140, 0xF, 0xF, true);  // mirror
    else return __shfl_xor(x, O, kWave);
}

template <int O, typename U>
__device__ __forceinline__ U lane_swap(U x) {
    static_assert(sizeof(U) == 4 || sizeof(U) == 8, "32- or 64-bit values");
    if constexpr (sizeof(U) == 4) {
        return __builtin_bit_cast(U, lane_swap_i32<O>(__builtin_bit_cast(int, x)));
    } else {
        const int64_t b = __builtin_bit_cast(int64_t, x);
        const int lo = lane_swap_i32<O>((int)(uint32_t)b);
        const int hi = lane_swap_i32<O>((int)(b >> 32));
        return __builtin_bit_cast(U, (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
    }
}

template <int O, int LPR, typename U>
__device__ __forceinline__ U group_sum_from(U x) {
    if constexpr (O == 0) {
        return x;
    } else {
        x += lane_swap<O>(x);
        return group_sum_from<O / 2, LPR>(x);
    }
}

// Sum over the LPR lanes of a row group (groups are aligned lane ranges;
// every lane of the group must be active).
template <int LPR, typename U>
__device__ __forceinline__ U group_sum(U x) {
    return group_sum_from<LPR / 2, LPR>(x);
}

template <int O, typename U>
__device__ __forceinline__ U group_min_from(U x) {
    if constexpr (O == 0) {
        return x;
    } else {
        const U y = lane_swap<O>(x);
        x = (y < x) ? y : x;
        return group_min_from<O / 2>(x);
    }
}

template <int LPR, typename U>
__device__ __forceinline__ U group_min(U x) {
    return group_min_from<LPR / 2>(x);
}

template <int O, typename U>
__device__ __forceinline__ U group_max_from(U x) {
    if constexpr (O == 0) {
        return x;
    } else {
        const U y = lane_swap<O>(x);
        x = (y > x) ? y : x;
        return group_max_from<O / 2>(x);
    }
}

template <int G, typename U>
__device__ __forceinline__ U group_max(U x) {
    return group_max_from<G / 2>(x);
}

// The 32-bit value of lane k of this lane's aligned group of G (2 or 4)
// lanes (DPP quad permute).
template <int G, int k>
__device__ __forceinline__ int group_bcast(int x) {
    static_assert((G == 2 || G == 4) && k < G, "groups of 2 or 4 lanes");
    constexpr int ctrl = (G == 4) ? k * 0x55 : (k | (k << 2) | ((2 + k) << 4) | ((2 + k) << 6));
    return __builtin_amdgcn_mov_dpp(x, ctrl, 0xF, 0xF, true);
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
constexpr uint64_t kSplitmixGamma = 0x9e3779b97f4a7c15ull;

// The output mix applied to the state z.
__device__ __forceinline__ uint64_t splitmix64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// State before output c; consecutive outputs step it by kSplitmixGamma, so
// a run of them costs one multiply for the first and an add for each next.
__device__ __forceinline__ uint64_t splitmix64_state(uint64_t seed, uint64_t c) {
    return seed + (c + 1ull) * kSplitmixGamma;
}

__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t c) {
    return splitmix64_mix(splitmix64_state(seed, c));
}

__device__ __forceinline__ double uniform_pm1(uint64_t z) {
    return 2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0;
}

}  // namespace ad
