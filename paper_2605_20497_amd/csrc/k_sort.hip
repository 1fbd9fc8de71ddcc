// Stable LSD radix sort of (key, value) pairs on the low `bits` bits of the
// key: 8-bit digits, one pass per digit.
//
// A pass over n > kSortTile elements takes three launches:
//  - k_rs_count: per tile of kSortTile elements, its digit counts (per-wave
//    histograms in shared memory, summed), stored digit-major: cnt[d][tile];
//  - an exclusive scan of cnt in that order, giving each (digit, tile) its
//    first output position (all tiles' digit-0 elements first, in tile order);
//  - k_rs_scatter: per tile, a stable rank of every element within its digit
//    (each wave ranks its contiguous quarter 64 elements at a time, lanes
//    holding the same digit found with eight ballots; one pass then orders
//    the waves), the tile reordered by digit in shared memory, then each
//    digit's run written to its output position by consecutive threads at
//    consecutive addresses.
// Up to kSortTile elements are sorted in one workgroup (k_rs_small): every
// pass in shared memory, with the same stable ranking.
#include "dev_util.h"

namespace hgp {

namespace {

constexpr int kSortThreads = 256;
constexpr int kSortChunks = 16;
constexpr int kSortTile = kSortThreads * kSortChunks;  // 4,096 elements per tile
constexpr int kBuckets = 256;
constexpr int kSortWaves = kSortThreads / kWave;

__device__ __forceinline__ u32 digit_of(u32 k, int shift) { return (k >> shift) & 255u; }
__device__ __forceinline__ u32 digit_of(u64 k, int shift) { return (u32)(k >> shift) & 255u; }

// Lanes of this wave holding the same digit d (among lanes with `valid`).
__device__ __forceinline__ u64 digit_peers(u32 d, int valid) {
    u64 m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const u64 ones = __ballot((int)((d >> b) & 1u));
        m &= ((d >> b) & 1u) ? ones : ~ones;
    }
    return m;
}

template <typename K>
__global__ __launch_bounds__(kSortThreads) void k_rs_count(i64 n, const K* __restrict__ keys, int shift,
                                                           u32* cnt, i64 ntiles) {
    __shared__ u32 h[kSortWaves][kBuckets];
    const int wv = wave_id();
    for (int i = threadIdx.x; i < kSortWaves * kBuckets; i += kSortThreads) (&h[0][0])[i] = 0;
    __syncthreads();
    const i64 base = (i64)blockIdx.x * kSortTile;
#pragma unroll 4
    for (int c = 0; c < kSortChunks; ++c) {
        const i64 i = base + (i64)c * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[wv][digit_of(keys[i], shift)], 1u);
    }
    __syncthreads();
    const int d = threadIdx.x;
    u32 s = 0;
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) s += h[w][d];
    cnt[(i64)d * ntiles + blockIdx.x] = s;
}

// Stable ranks of one tile (up to kSortTile elements from `kin`/`vin`) into
// shared memory ordered by digit.  dstart[d] = first tile position of digit
// d, which the caller has filled.  Each wave ranks its own contiguous quarter
// of the tile, kSortChunks rounds of 64 elements against digit counters of its
// own (wave-level ordering only, no block barrier per round); one block-wide
// pass then offsets each wave's counts by those of the waves before it, so
// equal digits keep their input order.  The elements stay in registers
// between the two phases.  wc[kSortWaves][kBuckets] is scratch.
template <typename K, typename V>
__device__ __forceinline__ void rank_tile(i64 nt, const K* __restrict__ kin, const V* __restrict__ vin, int shift,
                                          const u32* dstart, u32 (*wc)[kBuckets], K* sk, V* sv) {
    static_assert(kBuckets == kSortThreads, "one thread per digit in the cross-wave pass");
    const int lane = lane_id(), wv = wave_id();
    const u64 lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    u32* mine = wc[wv];
    for (int d = lane; d < kBuckets; d += kWave) mine[d] = 0;
    const i64 w0 = (i64)wv * (kWave * kSortChunks) + lane;  // this lane's first element
    K kk[kSortChunks];
    V vv[kSortChunks];
#pragma unroll
    for (int c = 0; c < kSortChunks; ++c) {
        const i64 i = w0 + (i64)c * kWave;
        const bool valid = i < nt;
        kk[c] = valid ? kin[i] : (K)0;
        vv[c] = valid ? vin[i] : (V)0;
    }
    wave_sync();  // counters cleared
    u32 rr[kSortChunks];
#pragma unroll
    for (int c = 0; c < kSortChunks; ++c) {
        const int valid = (int)(w0 + (i64)c * kWave < nt);
        const u32 d = digit_of(kk[c], shift);
        const u64 peers = digit_peers(d, valid);
        const u32 r = (u32)__popcll(peers & lt);
        const u32 before = mine[d];
        rr[c] = before + r;
        wave_sync();  // every lane has read its digit's count before the first lane of the digit moves it
        if (valid & (int)(r == 0)) mine[d] = before + (u32)__popcll(peers);
        wave_sync();
    }
    __syncthreads();
    {
        // digit t: exclusive prefix of the waves' counts, in wave order
        const int t = threadIdx.x;
        u32 acc = 0;
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) {
            const u32 x = wc[w][t];
            wc[w][t] = acc;
            acc += x;
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kSortChunks; ++c) {
        if (w0 + (i64)c * kWave < nt) {
            const u32 d = digit_of(kk[c], shift);
            const u32 pos = dstart[d] + mine[d] + rr[c];
            sk[pos] = kk[c];
            sv[pos] = vv[c];
        }
    }
    __syncthreads();  // the tile is in shared memory, and wc is free again
}

// Exclusive scan of one value per thread over the block (256 threads).
__device__ __forceinline__ u32 block_excl_u32(u32 x, u32* tmp) {
    const int lane = lane_id(), wv = wave_id();
    const u32 inc = wave_incl_scan(x);
    if (lane == kWave - 1) tmp[wv] = inc;
    __syncthreads();
    u32 off = 0;
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) off += w < wv ? tmp[w] : 0u;
    __syncthreads();
    return off + inc - x;
}

template <typename K, typename V>
struct SortShared {
    K sk[kSortTile];
    V sv[kSortTile];
    u32 wc[kSortWaves][kBuckets];
    u32 dstart[kBuckets];
    u32 gpos[kBuckets];
    u32 tmp[kSortWaves];
};

template <typename K, typename V>
__global__ __launch_bounds__(kSortThreads) void k_rs_scatter(i64 n, const K* __restrict__ kin, K* kout,
                                                             const V* __restrict__ vin, V* vout, int shift,
                                                             const u32* __restrict__ cnt,
                                                             const u32* __restrict__ pos, i64 ntiles) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    SortShared<K, V>& sh = *reinterpret_cast<SortShared<K, V>*>(smem_raw);
    const i64 base = (i64)blockIdx.x * kSortTile;
    const i64 nt = min((i64)kSortTile, n - base);
    const int d = threadIdx.x;
    const u32 c = cnt[(i64)d * ntiles + blockIdx.x];
    sh.gpos[d] = pos[(i64)d * ntiles + blockIdx.x];
    sh.dstart[d] = block_excl_u32(c, sh.tmp);
    __syncthreads();
    rank_tile<K, V>(nt, kin + base, vin + base, shift, sh.dstart, sh.wc, sh.sk, sh.sv);
    // each digit's run to its output position: consecutive positions of the
    // reordered tile go to consecutive addresses
    for (int j = threadIdx.x; j < nt; j += kSortThreads) {
        const K k = sh.sk[j];
        const u32 dj = digit_of(k, shift);
        const i64 o = (i64)sh.gpos[dj] + (j - (i64)sh.dstart[dj]);
        kout[o] = k;
        vout[o] = sh.sv[j];
    }
}

// Whole sort of at most kSortTile elements in one workgroup.
template <typename K, typename V>
__global__ __launch_bounds__(kSortThreads) void k_rs_small(i64 n, const K* __restrict__ kin, K* kout,
                                                           const V* __restrict__ vin, V* vout, int bits) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    SortShared<K, V>& sh = *reinterpret_cast<SortShared<K, V>*>(smem_raw);
    K* bk = reinterpret_cast<K*>(&sh + 1);  // second buffer pair after the first
    V* bv = reinterpret_cast<V*>(bk + kSortTile);
    const K* src_k = kin;
    const V* src_v = vin;
    // digits on which the keys differ (the others need no pass)
    u64 o = 0, a = ~0ull;
    for (i64 i = threadIdx.x; i < n; i += kSortThreads) {
        o |= (u64)kin[i];
        a &= (u64)kin[i];
    }
#pragma unroll
    for (int sh2 = kWave / 2; sh2 > 0; sh2 >>= 1) {
        o |= __shfl_xor(o, sh2, kWave);
        a &= __shfl_xor(a, sh2, kWave);
    }
    __shared__ u64 s_or[kSortWaves], s_and[kSortWaves];
    if (lane_id() == 0) {
        s_or[wave_id()] = o;
        s_and[wave_id()] = a;
    }
    __syncthreads();
    u64 varying = 0;
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) varying |= s_or[w] ^ s_and[w];
    int npass = 0;
    for (int shift = 0; shift < bits; shift += 8) {
        if (((varying >> shift) & 255u) == 0) continue;  // same digit everywhere: the order stays
        // digit counts of the current order, then their starts
        for (int w = 0; w < kSortWaves; ++w) sh.wc[w][threadIdx.x] = 0;
        __syncthreads();
        for (int c = 0; c < kSortChunks; ++c) {
            const i64 i = (i64)c * kSortThreads + threadIdx.x;
            if (i < n) atomicAdd(&sh.wc[wave_id()][digit_of(src_k[i], shift)], 1u);
        }
        __syncthreads();
        u32 s = 0;
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) s += sh.wc[w][threadIdx.x];
        __syncthreads();
        sh.dstart[threadIdx.x] = block_excl_u32(s, sh.tmp);
        __syncthreads();
        // alternate between the two shared buffer pairs
        const bool to_first = (npass++ % 2) == 0;
        K* dk = to_first ? sh.sk : bk;
        V* dv = to_first ? sh.sv : bv;
        rank_tile<K, V>(n, src_k, src_v, shift, sh.dstart, sh.wc, dk, dv);
        src_k = dk;
        src_v = dv;
    }
    for (i64 j = threadIdx.x; j < n; j += kSortThreads) {
        kout[j] = src_k[j];
        vout[j] = src_v[j];
    }
}

// OR and AND of all keys: a digit where they agree is the same for every key,
// and a stable pass over it leaves the order as it is.
template <typename K>
__global__ __launch_bounds__(kSortThreads) void k_rs_varying(i64 n, const K* __restrict__ keys,
                                                             unsigned long long* orand) {
    u64 o = 0, a = ~0ull;
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) {
        const u64 k = (u64)keys[i];
        o |= k;
        a &= k;
    }
#pragma unroll
    for (int sh = kWave / 2; sh > 0; sh >>= 1) {
        o |= __shfl_xor(o, sh, kWave);
        a &= __shfl_xor(a, sh, kWave);
    }
    if (lane_id() == 0) {
        atomicOr(&orand[0], (unsigned long long)o);
        atomicAnd(&orand[1], (unsigned long long)a);
    }
}

enum { WS_RS_KEYS = 56, WS_RS_VALS = 57, WS_RS_CNT = 58, WS_RS_POS = 59, WS_RS_BITS = 55 };

template <typename K, typename V>
void radix_sort(Ctx* c, const K* kin, K* kout, const V* vin, V* vout, i64 n, int bits) {
    if (n <= 0) return;
    if (bits < 1) bits = 1;
    const int nk = (int)(8 * sizeof(K));
    if (bits > nk) bits = nk;
    if (n <= kSortTile) {
        const size_t lds = sizeof(SortShared<K, V>) + (sizeof(K) + sizeof(V)) * kSortTile;
        LAUNCH(c, KF_SORT, (k_rs_small<K, V>), 1, kSortThreads, lds, n, kin, kout, vin, vout, bits);
        return;
    }
    const i64 ntiles = ceil_div(n, kSortTile);
    // Only digits on which the keys differ need a pass.
    unsigned long long* orand = wsp<unsigned long long>(c, WS_RS_BITS, 2);
    fill_many(c, {{orand, 2, 0u}, {orand + 1, 2, ~0u}});
    LAUNCH(c, KF_SORT, (k_rs_varying<K>), grid_for(n, kSortThreads, c->num_cu * 4), kSortThreads, 0, n, kin, orand);
    i64 oa[2];
    read_back(c, orand, oa, 2, 8);
    const u64 varying = ((u64)oa[0] ^ (u64)oa[1]) & (bits >= 64 ? ~0ull : ((1ull << bits) - 1));
    int shifts[8], passes = 0;
    for (int sh = 0; sh < bits; sh += 8)
        if ((varying >> sh) & 255u) shifts[passes++] = sh;
    if (passes == 0) {  // already in order: every key is the same on the sorted bits
        HIPC(hipMemcpyAsync(kout, kin, sizeof(K) * (size_t)n, hipMemcpyDeviceToDevice, c->stream));
        HIPC(hipMemcpyAsync(vout, vin, sizeof(V) * (size_t)n, hipMemcpyDeviceToDevice, c->stream));
        return;
    }
    K* tk = wsp<K>(c, WS_RS_KEYS, (size_t)n);
    V* tv = wsp<V>(c, WS_RS_VALS, (size_t)n);
    u32* cnt = wsp<u32>(c, WS_RS_CNT, (size_t)kBuckets * ntiles);
    u32* pos = wsp<u32>(c, WS_RS_POS, (size_t)kBuckets * ntiles + 1);
    const size_t lds = sizeof(SortShared<K, V>);
    const K* sk = kin;
    const V* sv = vin;
    for (int p = 0; p < passes; ++p) {
        // the last pass lands in kout; earlier ones alternate so that it does
        K* dk = ((passes - 1 - p) % 2 == 0) ? kout : tk;
        V* dv = ((passes - 1 - p) % 2 == 0) ? vout : tv;
        LAUNCH(c, KF_SORT, (k_rs_count<K>), (int)ntiles, kSortThreads, 0, n, sk, shifts[p], cnt, ntiles);
        scan_excl_i32(c, (const i32*)cnt, (i32*)pos, (i64)kBuckets * ntiles);
        LAUNCH(c, KF_SORT, (k_rs_scatter<K, V>), (int)ntiles, kSortThreads, lds, n, sk, dk, sv, dv, shifts[p],
               (const u32*)cnt, (const u32*)pos, ntiles);
        sk = dk;
        sv = dv;
    }
}

}  // namespace

void sort_pairs_u32(Ctx* c, const u32* kin, u32* kout, const i32* vin, i32* vout, i64 n, int bits) {
    radix_sort<u32, i32>(c, kin, kout, vin, vout, n, bits);
}

void sort_pairs_u32_u64(Ctx* c, const u32* kin, u32* kout, const u64* vin, u64* vout, i64 n, int bits) {
    radix_sort<u32, u64>(c, kin, kout, vin, vout, n, bits);
}

void sort_pairs_u64(Ctx* c, const u64* kin, u64* kout, const i32* vin, i32* vout, i64 n, int bits) {
    radix_sort<u64, i32>(c, kin, kout, vin, vout, n, bits);
}

}  // namespace hgp
