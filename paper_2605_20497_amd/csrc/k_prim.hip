// Parallel primitives: prefix sums, fills and gathers.  The stable radix sort
// is in k_sort.hip.

#include "dev_util.h"
#include "scan_lb.h"

namespace hgp {

namespace {

template <typename Tin, typename Tout>
__global__ __launch_bounds__(kLbBlock) void k_scan_lookback(const Tin* __restrict__ in, i64 n, Tout* out,
                                                             ScanState st, u64 tag, u64 ticket0, i64 tiles) {
    lookback_scan_tile(
        n, st, tag, ticket0, tiles, true, [&](i64 i) { return (i64)in[i]; },
        [&](i64 i, i64 prefix, i64) { out[i] = (Tout)prefix; }, [&](i64 sum) { out[n] = (Tout)sum; });
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
template <typename Tin, typename Tout>
void scan_impl(Ctx* c, const Tin* in, Tout* out, i64 n) {
    if (n <= 0) {
        HIPC(hipMemsetAsync(out, 0, sizeof(Tout), c->stream));
        return;
    }
    const ScanLaunch sl = scan_launch(c, n);
    LAUNCH(c, KF_SCAN, (k_scan_lookback<Tin, Tout>), (int)sl.tiles, kLbBlock, 0, in, n, out, sl.st, sl.tag,
           sl.ticket0, sl.tiles);
}

}  // namespace

ScanLaunch scan_launch(Ctx* c, i64 n) {
    const i64 tiles = ceil_div(n, kLbTile);
    if (c->scan_tiles < tiles || c->scan_tag + 1 >= kLbTagLimit) {
        // (re)allocated or, once the tags run out, cleared: zero status words
        // are older than any tag
        const i64 cap = std::max<i64>({tiles, c->scan_tiles, 4096});
        const size_t bytes = 16 + (size_t)cap * 32;
        if (c->scan_tiles < cap) {
            c->release(c->b_scan);
            c->b_scan = c->alloc(bytes);
        }
        HIPC(hipMemsetAsync(c->b_scan.p, 0, bytes, c->stream));
        c->scan_tiles = cap;
        c->scan_ticket = 0;
        c->scan_tag = 0;
    }
    u64* base = (u64*)c->b_scan.p;
    ScanLaunch sl;
    sl.st = ScanState{(unsigned long long*)base, base + 1, base + 2};
    sl.tag = ++c->scan_tag;
    sl.ticket0 = c->scan_ticket;
    sl.tiles = tiles;
    c->scan_ticket += (u64)tiles;
    return sl;
}

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
