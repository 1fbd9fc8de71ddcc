// Device-side helpers for gfx950 (64-lane wavefronts).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "hgp_internal.h"

namespace hgp {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }
__device__ __forceinline__ int wave_id() { return (int)(threadIdx.x / kWave); }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        T t = __shfl_xor(v, o, kWave);
        v = t > v ? t : v;
    }
    return v;
}

__device__ __forceinline__ unsigned long long wave_or(unsigned long long v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v |= __shfl_xor(v, o, kWave);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        T t = __shfl_xor(v, o, kWave);
        v = t < v ? t : v;
    }
    return v;
}

// Inclusive prefix sum across the wave.
// Loads of values that other threads update with device atomics (performed in
// L2): device-scope relaxed loads, so a workgroup that runs several dependent
// steps never reads an older copy held in its vector L1 cache.
template <typename T>
__device__ __forceinline__ T load_l2(const T* p) {
    return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Value of lane `src` (wave-uniform) broadcast through scalar registers: unlike
// __shfl, no LDS permute traffic.
__device__ __forceinline__ int bcast(int v, int src) { return __builtin_amdgcn_readlane(v, src); }
__device__ __forceinline__ unsigned bcast(unsigned v, int src) {
    return (unsigned)__builtin_amdgcn_readlane((int)v, src);
}
__device__ __forceinline__ long long bcast(long long v, int src) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, src);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)((unsigned long long)v >> 32), src);
    return (long long)(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ long bcast(long v, int src) { return (long)bcast((long long)v, src); }
__device__ __forceinline__ unsigned long long bcast(unsigned long long v, int src) {
    return (unsigned long long)bcast((long long)v, src);
}
__device__ __forceinline__ unsigned long bcast(unsigned long v, int src) {
    return (unsigned long)bcast((long long)v, src);
}

// Work item of round r for workgroup b of a persistent grid of G workgroups.
// Workgroups go to the 8 XCDs round robin (b to XCD b % 8), so item b of each
// round would put consecutive items, which share most of their inputs (a
// node's neighbours, an h-edge's rows), on eight different L2 caches.  Here
// each XCD takes a contiguous run of G / 8 items per round.  A bijection on
// each round's G items; grids not a multiple of 8 keep the plain order.
__device__ __forceinline__ i64 xcd_item(i64 r, int b, int G) {
    if (G & 7) return r * G + b;
    return r * G + (i64)(b & 7) * (G >> 3) + (b >> 3);
}

// List entries one wave takes at a time in the windowed kernels (one per lane,
// kept by ballot): the list of n entries spread evenly over the grid's waves,
// at most kWave.  Long lists use full windows; a short one (a coarse level)
// gets narrow windows, so it still reaches every wave of the grid instead of
// leaving most of the chip idle.  Host grids are sized for kWindowMin.
constexpr int kWindowMin = 8;
__device__ __forceinline__ i64 wave_window(i64 n, i64 waves) {
    const i64 w = (n + waves - 1) / waves;
    return w < 1 ? 1 : (w > kWave ? kWave : w);
}

// Orders shared-memory writes of one wave before later reads of other lanes of
// the same wave.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const int l = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        T t = __shfl_up(v, o, kWave);
        if (l >= o) v += t;
    }
    return v;
}

// Comparisons that pick between two (key, id) pairs are written with bitwise
// operators on operands already in registers, so the device compiler emits
// selects instead of short-circuit branches: a short-circuit form, where the
// condition guards updates of two variables, was compiled into code that lost
// one of the updates on some lanes.
template <typename K>
__device__ __forceinline__ bool lex_gt(K k1, i32 i1, K k2, i32 i2) {
    return ((int)(k1 > k2) | ((int)(k1 == k2) & (int)(i1 > i2))) != 0;
}

// (k1, i1) beats (k2, i2) where id < 0 marks an empty entry.
template <typename K>
__device__ __forceinline__ bool lex_better(K k1, i32 i1, K k2, i32 i2) {
    return ((int)(i1 >= 0) & ((int)(i2 < 0) | (int)lex_gt(k1, i1, k2, i2))) != 0;
}

// Lexicographic max of (key, id) across the wave; every lane receives it.
__device__ __forceinline__ void wave_lexmax(u64& key, i32& id) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const u64 k2 = __shfl_xor(key, o, kWave);
        const i32 i2 = __shfl_xor(id, o, kWave);
        const bool t = lex_gt(k2, i2, key, id);
        key = t ? k2 : key;
        id = t ? i2 : id;
    }
}

// Same over signed keys with id < 0 marking an empty entry.
__device__ __forceinline__ void wave_lexmax_i64(i64& key, i32& id) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const i64 k2 = __shfl_xor(key, o, kWave);
        const i32 i2 = __shfl_xor(id, o, kWave);
        const bool t = lex_better(k2, i2, key, id);
        key = t ? k2 : key;
        id = t ? i2 : id;
    }
}

// Block-wide sum (blockDim.x a multiple of 64, at most 1024).  `red` is
// shared scratch of at least 16 entries.  Every thread receives the total.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* red) {
    v = wave_sum(v);
    const int nw = blockDim.x / kWave;
    __syncthreads();
    if (lane_id() == 0) red[wave_id()] = v;
    __syncthreads();
    T t = 0;
    for (int w = 0; w < nw; ++w) t += red[w];
    __syncthreads();
    return t;
}

// Block-wide exclusive prefix sum of one value per thread; *total receives
// the block total.  `red` holds at least 16 entries.
template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T* red, T* total) {
    T inc = wave_incl_scan(v);
    const int nw = blockDim.x / kWave;
    __syncthreads();
    if (lane_id() == kWave - 1) red[wave_id()] = inc;
    __syncthreads();
    T off = 0, tot = 0;
    for (int w = 0; w < nw; ++w) {
        if (w < wave_id()) off += red[w];
        tot += red[w];
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

// Order-preserving map of a signed 64-bit value onto unsigned.
__device__ __forceinline__ u64 enc_i64(i64 x) { return (u64)x ^ 0x8000000000000000ull; }
__device__ __forceinline__ i64 dec_i64(u64 x) { return (i64)(x ^ 0x8000000000000000ull); }

// SplitMix64 output mixing function (Steele, Lea, Flood, OOPSLA 2014).
__device__ __forceinline__ u64 splitmix_mix(u64 z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Remainder by an invariant 64-bit divisor d >= 1 with one multiply-high
// (Granlund and Montgomery, "Division by invariant integers using
// multiplication", PLDI 1994, Fig. 4.1): with l = ceil(log2 d) and
// m = floor(2^64 (2^l - d) / d) + 1, q = (t + ((n - t) >> min(l,1))) >> max(l-1,0)
// where t = mulhi(m, n), is floor(n / d) for every 64-bit n.
struct DivU64 {
    u64 d, m;
    u32 sh1, sh2;
};

__device__ __forceinline__ DivU64 divu64_make(u64 d) {
    u32 l = 0;
    while (l < 64 && (1ull << l) < d) ++l;  // ceil(log2 d)
    DivU64 r;
    r.d = d;
    const unsigned __int128 two_l = (unsigned __int128)1 << l;
    r.m = (u64)((((unsigned __int128)(two_l - d)) << 64) / d) + 1;
    r.sh1 = l < 1 ? l : 1;
    r.sh2 = l > 0 ? l - 1 : 0;
    return r;
}

__device__ __forceinline__ u64 divu64_rem(u64 n, const DivU64& f) {
    const u64 t = __umul64hi(f.m, n);
    const u64 q = (t + ((n - t) >> f.sh1)) >> f.sh2;
    return n - q * f.d;
}

// Symmetric histogram noise of Sec. V-C: hash of the unordered pair {a, b}
// and the seed, reduced into [0, cap]; `f` divides by cap + 1.
__device__ __forceinline__ u64 pair_noise(u64 seed, i32 a, i32 b, const DivU64& f) {
    const u64 lo = (u64)(u32)(a < b ? a : b);
    const u64 hi = (u64)(u32)(a < b ? b : a);
    return divu64_rem(splitmix_mix(seed ^ splitmix_mix((lo << 32) | hi)), f);
}

// Normalised h-edge weight omega(e)/|e| in 16-bit fixed point, at least 1.
__device__ __forceinline__ u64 norm_weight(i32 w, i64 card) {
    const u64 t = ((u64)(u32)w << 16) / (u64)card;
    return t ? t : 1;
}

// Bitonic sort of s[0 .. npad) in shared memory, npad a power of two; all
// threads of the block take part.
__device__ __forceinline__ void block_bitonic_sort_u32(u32* s, int npad) {
    for (int k = 2; k <= npad; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < npad; i += blockDim.x) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const u32 a = s[i], b = s[ixj];
                    const bool up = (i & k) == 0;
                    if ((a > b) == up) {
                        s[i] = b;
                        s[ixj] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Bitonic sort, ascending, of 64 * KPL keys held in one wave: lane l holds
// positions KPL*l .. KPL*l + KPL - 1 in v[0 .. KPL).  Partners KPL or more
// positions apart are in other lanes (same register, exchanged by shuffles);
// closer ones are in the same lane.  Fully unrolled: no barriers, no shared
// memory.
template <int KPL>
__device__ __forceinline__ void wave_bitonic_sort(u32 (&v)[KPL]) {
    constexpr int N = 64 * KPL;
    const int lane = lane_id();
#pragma unroll
    for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= KPL) {
#pragma unroll
                for (int r = 0; r < KPL; ++r) {
                    const int i = lane * KPL + r;
                    const u32 o = (u32)__shfl_xor((int)v[r], j / KPL, kWave);
                    const bool keep_min = ((i & j) == 0) == ((i & k) == 0);
                    const u32 mn = v[r] < o ? v[r] : o, mx = v[r] < o ? o : v[r];
                    v[r] = keep_min ? mn : mx;
                }
            } else {
#pragma unroll
                for (int r = 0; r < KPL; ++r) {
                    const int rp = r ^ j;
                    if (rp > r) {
                        const int i = lane * KPL + r;
                        const bool up = (i & k) == 0;
                        const u32 a = v[r], b = v[rp];
                        const bool sw = (a > b) == up;
                        v[r] = sw ? b : a;
                        v[rp] = sw ? a : b;
                    }
                }
            }
        }
    }
}

__host__ __device__ __forceinline__ int next_pow2(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

}  // namespace hgp
