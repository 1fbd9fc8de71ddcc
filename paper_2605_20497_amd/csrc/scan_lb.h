// Single-pass prefix sum with decoupled look-back, shared by the plain scans
// (k_prim.hip) and the kernels that fuse a scan with its producer and its
// consumer (the chain rounds' compaction).
#pragma once

#include "dev_util.h"

namespace hgp {

// Single-pass prefix sum with decoupled look-back (Merrill and Garland,
// "Single-pass Parallel Prefix Scan with Decoupled Look-back", NVIDIA technical
// report NVR-2016-002).  A tile is kLbBlock * kLbItems items; each wave scans a
// contiguous run of kWave * kLbItems of them, lane l holding items l, l + 64,
// ... (coalesced loads and stores).  A block takes its tile from a ticket
// counter, so every tile with a smaller index belongs to a block already
// running.  It publishes its aggregate, sums its predecessors' published
// values 64 tiles at a time (stopping at the nearest tile that has published
// its inclusive prefix), then publishes its own inclusive prefix.
//
// Each published value is two status words, one per 32-bit half, each
// carrying the scan's tag and a ready bit beside its half, so a word read
// whole is either this scan's final half or not ready, and no ordering between
// words is needed.  The words are written and read with relaxed device-scope
// atomics: release and acquire at device scope would write back and
// invalidate the XCD's whole L2 on every publish and poll.  Tags make values
// left by earlier scans unreadable, so nothing is cleared between scans (the
// host zeroes the state when the 31-bit tag wraps).  A wait that runs out
// (kLbSpinMax polls) sets the error word, which the host checks, instead of
// waiting for ever.
constexpr int kLbBlock = 256;
constexpr int kLbItems = 16;
constexpr i64 kLbTile = (i64)kLbBlock * kLbItems;
constexpr u32 kLbSpinMax = 1u << 22;
constexpr u64 kLbTagLimit = 1ull << 31;

struct ScanState {
    unsigned long long* ticket;
    u64* err;
    u64* word;  // per tile: aggregate (low, high half), inclusive prefix (low, high half)
};

__device__ __forceinline__ u64 lb_word(u64 tag, u32 half) { return (tag << 33) | (1ull << 32) | (u64)half; }
__device__ __forceinline__ bool lb_ready(u64 w, u64 tag) { return (w >> 32) == ((tag << 1) | 1ull); }
__device__ __forceinline__ i64 lb_join(u64 lo, u64 hi) { return (i64)(((hi & 0xFFFFFFFFull) << 32) | (lo & 0xFFFFFFFFull)); }

__device__ __forceinline__ void lb_publish(const ScanState& st, i64 t, u64 tag, int incl, i64 v) {
    u64* w = st.word + 4 * t + 2 * incl;
    __hip_atomic_store(w, lb_word(tag, (u32)(u64)v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(w + 1, lb_word(tag, (u32)((u64)v >> 32)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ u64 lb_load(const u64* p) {
    return __hip_atomic_load(const_cast<u64*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum of the items of tiles 0 .. t-1, on every lane of the calling wave
// (t >= 1; tile 0 publishes its inclusive prefix without looking back).
__device__ inline i64 lb_look_back(const ScanState& st, i64 t, u64 tag) {
    const int lane = lane_id();
    i64 prefix = 0;
    for (i64 hi = t;; hi -= kWave) {
        const i64 j = hi - 1 - lane;  // lane 0: the nearest tile
        const u64* w = st.word + 4 * (j >= 0 ? j : 0);
        u64 a0 = 0, a1 = 0, c0 = 0, c1 = 0;
        int has_incl = 0, has_agg = 0;
        for (u32 spins = 0;; ++spins) {
            a0 = lb_load(w);
            a1 = lb_load(w + 1);
            c0 = lb_load(w + 2);
            c1 = lb_load(w + 3);
            has_incl = (int)(j >= 0) & (int)lb_ready(c0, tag) & (int)lb_ready(c1, tag);
            has_agg = (int)(j >= 0) & (int)lb_ready(a0, tag) & (int)lb_ready(a1, tag);
            if (__all((int)(j < 0) | has_incl | has_agg)) break;
            if (spins == kLbSpinMax) {
                if (lane == 0) __hip_atomic_store(st.err, (u64)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return prefix;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        // the window holds tile 0 (inclusive) whenever some j < 0, so stop < kWave then
        const u64 im = __ballot(has_incl);
        const int stop = im ? __builtin_ctzll(im) : kWave;
        i64 v = 0;
        if ((j >= 0) & (lane <= stop)) v = lane == stop ? lb_join(c0, c1) : lb_join(a0, a1);
        prefix += wave_sum(v);
        if (im) return prefix;
    }
}

// One tile of a look-back scan over n items, in a kernel of kLbBlock threads
// launched with `tiles` = ceil(n / kLbTile) blocks.  load(i) gives item i
// (i < n); store(i, prefix, item) receives the exclusive prefix of item i;
// total(sum) runs once, on the tile holding the last item.  With on == false
// the block only takes its ticket (the host counts tickets per launch).
template <typename Load, typename Store, typename Total>
__device__ __forceinline__ void lookback_scan_tile(i64 n, const ScanState& st, u64 tag, u64 ticket0, i64 tiles,
                                                   bool on, Load load, Store store, Total total) {
    constexpr int kWaves = kLbBlock / kWave;
    __shared__ i64 s_wsum[kWaves];
    __shared__ i64 s_tile, s_prefix;
    const int lane = lane_id(), w = wave_id();
    if (threadIdx.x == 0) s_tile = (i64)(atomicAdd(st.ticket, 1ull) - ticket0);
    __syncthreads();
    const i64 t = s_tile;
    if ((t < 0) | (t >= tiles)) {  // the host's ticket count is off: report, touch nothing
        if (threadIdx.x == 0) __hip_atomic_store(st.err, (u64)2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    if (!on) return;
    const i64 seg = t * kLbTile + (i64)w * (kWave * kLbItems) + lane;
    i64 x[kLbItems], e[kLbItems];
#pragma unroll
    for (int k = 0; k < kLbItems; ++k) {
        const i64 i = seg + (i64)k * kWave;
        x[k] = i < n ? load(i) : 0;
    }
    // exclusive sums within the wave's run
    i64 run = 0;
#pragma unroll
    for (int k = 0; k < kLbItems; ++k) {
        const i64 inc = wave_incl_scan(x[k]);
        e[k] = run + inc - x[k];
        run += bcast((long long)inc, kWave - 1);
    }
    if (lane == 0) s_wsum[w] = run;
    __syncthreads();
    i64 woff = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) {
        const i64 sq = s_wsum[q];
        woff += q < w ? sq : 0;
        tot += sq;
    }
    if (w == 0) {
        i64 prefix = 0;
        if (t == 0) {
            if (lane == 0) lb_publish(st, 0, tag, 1, tot);
        } else {
            if (lane == 0) lb_publish(st, t, tag, 0, tot);
            prefix = lb_look_back(st, t, tag);
            if (lane == 0) lb_publish(st, t, tag, 1, prefix + tot);
        }
        if (lane == 0) s_prefix = prefix;
    }
    __syncthreads();
    const i64 off = s_prefix + woff;
#pragma unroll
    for (int k = 0; k < kLbItems; ++k) {
        const i64 i = seg + (i64)k * kWave;
        if (i < n) store(i, off + e[k], x[k]);
    }
    if ((threadIdx.x == 0) & ((t + 1) * kLbTile >= n)) total(s_prefix + tot);
}

// Scan state for one launch over n >= 1 items: grows the context's state when
// needed and hands out the launch's tag and first ticket.
struct ScanLaunch {
    ScanState st;
    u64 tag, ticket0;
    i64 tiles;
};
ScanLaunch scan_launch(Ctx* c, i64 n);

}  // namespace hgp
