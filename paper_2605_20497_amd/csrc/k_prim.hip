// Parallel primitives: prefix sums, fills and gathers.  The stable radix sort
// is in k_sort.hip.

#include "dev_util.h"

namespace hgp {

namespace {

// Single-pass prefix sum with decoupled look-back (Merrill and Garland,
// "Single-pass Parallel Prefix Scan with Decoupled Look-back", NVIDIA technical
// report NVR-2016-002).  A tile is kLbBlock * kLbItems items; each wave scans a
// contiguous run of kWave * kLbItems of them, lane l holding items l, l + 64,
// ... (coalesced loads and stores).  A block takes its tile from a ticket
// counter, so every tile with a smaller index belongs to a block already
// running.  It publishes its aggregate, sums its predecessors' published
// values 64 tiles at a time (stopping at the nearest tile that has published
// its inclusive prefix), then publishes its own inclusive prefix.  Status words
// carry the scan's tag, so values left by earlier scans are never taken as
// this scan's and nothing is cleared between scans.  A wait that runs out
// (kLbSpinMax polls) sets the error word, which the host checks, instead of
// waiting for ever.
constexpr int kLbBlock = 256;
constexpr int kLbItems = 16;
constexpr i64 kLbTile = (i64)kLbBlock * kLbItems;
constexpr u32 kLbSpinMax = 1u << 22;

struct ScanState {
    unsigned long long* ticket;
    u64* err;
    u64* flag;  // (tag << 2) | 1 (aggregate published) or 2 (inclusive prefix published)
    i64* agg;
    i64* incl;
};

__device__ __forceinline__ void lb_publish(const ScanState& st, i64 t, u64 tag, u64 kind, i64 v) {
    __hip_atomic_store(kind == 2 ? st.incl + t : st.agg + t, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(st.flag + t, (tag << 2) | kind, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum of the items of tiles 0 .. t-1, on every lane of the calling wave
// (t >= 1; tile 0 publishes its inclusive prefix without looking back).
__device__ i64 lb_look_back(const ScanState& st, i64 t, u64 tag) {
    const int lane = lane_id();
    i64 prefix = 0;
    for (i64 hi = t;; hi -= kWave) {
        const i64 j = hi - 1 - lane;  // lane 0: the nearest tile
        u64 f = 0;
        for (u32 spins = 0;; ++spins) {
            f = j >= 0 ? __hip_atomic_load(st.flag + j, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) : 0;
            if (__all((int)(j < 0) | (int)((f >> 2) == tag))) break;
            if (spins == kLbSpinMax) {
                if (lane == 0) __hip_atomic_store(st.err, (u64)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return prefix;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        // the window holds tile 0 (inclusive) whenever some j < 0, so stop < kWave then
        const u64 im = __ballot((int)(j >= 0) & (int)((f & 3u) == 2u));
        const int stop = im ? __builtin_ctzll(im) : kWave;
        i64 v = 0;
        if ((j >= 0) & (lane <= stop))
            v = __hip_atomic_load(lane == stop ? st.incl + j : st.agg + j, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
        prefix += wave_sum(v);
        if (im) return prefix;
    }
}

template <typename Tin, typename Tout>
__global__ __launch_bounds__(kLbBlock) void k_scan_lookback(const Tin* __restrict__ in, i64 n, Tout* out,
                                                             ScanState st, u64 tag, u64 ticket0, i64 tiles) {
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
    const i64 seg = t * kLbTile + (i64)w * (kWave * kLbItems) + lane;
    i64 e[kLbItems];
#pragma unroll
    for (int k = 0; k < kLbItems; ++k) {
        const i64 i = seg + (i64)k * kWave;
        e[k] = i < n ? (i64)in[i] : 0;
    }
    // exclusive sums within the wave's run
    i64 run = 0;
#pragma unroll
    for (int k = 0; k < kLbItems; ++k) {
        const i64 x = e[k];
        const i64 inc = wave_incl_scan(x);
        e[k] = run + inc - x;
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
            if (lane == 0) lb_publish(st, 0, tag, 2, tot);
        } else {
            if (lane == 0) lb_publish(st, t, tag, 1, tot);
            prefix = lb_look_back(st, t, tag);
            if (lane == 0) lb_publish(st, t, tag, 2, prefix + tot);
        }
        if (lane == 0) s_prefix = prefix;
    }
    __syncthreads();
    const i64 off = s_prefix + woff;
#pragma unroll
    for (int k = 0; k < kLbItems; ++k) {
        const i64 i = seg + (i64)k * kWave;
        if (i < n) out[i] = (Tout)(off + e[k]);
    }
    if ((threadIdx.x == 0) & ((t + 1) * kLbTile >= n)) out[n] = (Tout)(s_prefix + tot);
}

template <typename T>
__global__ void k_fill(T* p, T v, i64 n) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) p[i] = v;
}

// One grid row per buffer of the list.
__global__ void k_fill_many(FillList L) {
    const FillItem f = L.it[blockIdx.y];
    u32* p = (u32*)f.p;
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < f.n; i += (i64)gridDim.x * blockDim.x) p[i] = f.v;
}

__global__ void k_iota(i32* p, i64 n) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) p[i] = (i32)i;
}

__global__ void k_gather(const i32* __restrict__ src, const i32* __restrict__ idx, i32* dst, i64 n) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
        dst[i] = src[idx[i]];
}

// The scan state with room for `tiles` tiles, zeroed when (re)allocated.
ScanState scan_state(Ctx* c, i64 tiles) {
    if (c->scan_tiles < tiles) {
        const i64 cap = std::max<i64>({tiles, 2 * c->scan_tiles, 4096});
        c->release(c->b_scan);
        const size_t bytes = 16 + (size_t)cap * 24;
        c->b_scan = c->alloc(bytes);
        HIPC(hipMemsetAsync(c->b_scan.p, 0, bytes, c->stream));
        c->scan_tiles = cap;
        c->scan_ticket = 0;
    }
    u64* base = (u64*)c->b_scan.p;
    return ScanState{(unsigned long long*)base, base + 1, base + 2, (i64*)(base + 2 + c->scan_tiles),
                     (i64*)(base + 2 + 2 * c->scan_tiles)};
}

template <typename Tin, typename Tout>
void scan_impl(Ctx* c, const Tin* in, Tout* out, i64 n) {
    if (n <= 0) {
        HIPC(hipMemsetAsync(out, 0, sizeof(Tout), c->stream));
        return;
    }
    const i64 tiles = ceil_div(n, kLbTile);
    const ScanState st = scan_state(c, tiles);
    const u64 tag = ++c->scan_tag;
    const u64 ticket0 = c->scan_ticket;
    c->scan_ticket += (u64)tiles;
    LAUNCH(c, KF_SCAN, (k_scan_lookback<Tin, Tout>), (int)tiles, kLbBlock, 0, in, n, out, st, tag, ticket0, tiles);
}

}  // namespace

void scan_excl_i64(Ctx* c, const i64* in, i64* out, i64 n) { scan_impl<i64, i64>(c, in, out, n); }
void scan_excl_i32_to_i64(Ctx* c, const i32* in, i64* out, i64 n) { scan_impl<i32, i64>(c, in, out, n); }
void scan_excl_i32(Ctx* c, const i32* in, i32* out, i64 n) { scan_impl<i32, i32>(c, in, out, n); }

void fill_i32(Ctx* c, i32* p, i32 v, i64 n) {
    if (n > 0) LAUNCH(c, KF_MISC, k_fill<i32>, grid_for(n, 256, 4096), 256, 0, p, v, n);
}
void fill_many(Ctx* c, std::initializer_list<FillItem> items) {
    FillList L{};
    int k = 0;
    i64 mx = 0;
    for (const FillItem& it : items) {
        if (it.n <= 0) continue;
        if (k == kFillMax) fail(HGP_E_INVALID, "fill_many: more than kFillMax buffers");
        L.it[k++] = it;
        mx = std::max(mx, it.n);
    }
    if (k > 0) LAUNCH(c, KF_MISC, k_fill_many, dim3(grid_for(mx, 256, 4096), k), 256, 0, L);
}
void fill_i64(Ctx* c, i64* p, i64 v, i64 n) {
    if (n > 0) LAUNCH(c, KF_MISC, k_fill<i64>, grid_for(n, 256, 4096), 256, 0, p, v, n);
}
void iota_i32(Ctx* c, i32* p, i64 n) {
    if (n > 0) LAUNCH(c, KF_MISC, k_iota, grid_for(n, 256, 4096), 256, 0, p, n);
}
void gather_i32(Ctx* c, const i32* src, const i32* idx, i32* dst, i64 n) {
    if (n > 0) LAUNCH(c, KF_MISC, k_gather, grid_for(n, 256, 4096), 256, 0, src, idx, dst, n);
}

void check_scan_state(Ctx* c) {
    if (!c->b_scan.p) return;
    i64 err = 0;
    read_back(c, (const u64*)c->b_scan.p + 1, &err, 1, 8);
    if (err != 0) {
        release_scan_state(c);  // the next scan starts from a zeroed state
        fail(HGP_E_DEVICE, "a prefix-sum look-back wait ran out");
    }
}

void release_scan_state(Ctx* c) {
    c->release(c->b_scan);
    c->scan_tiles = 0;
    c->scan_ticket = 0;
}

void read_back(Ctx* c, const void* dev, i64* host, int count, int elem_bytes) {
    HIPC(hipMemcpyAsync(c->host_scalars, dev, (size_t)count * elem_bytes, hipMemcpyDeviceToHost, c->stream));
    HIPC(hipStreamSynchronize(c->stream));
    for (int i = 0; i < count; ++i) {
        if (elem_bytes == 8) host[i] = ((i64*)c->host_scalars)[i];
        else host[i] = ((i32*)c->host_scalars)[i];
    }
}

}  // namespace hgp
