// Parallel primitives: prefix sums, fills and gathers.  The stable radix sort
// is in k_sort.hip.

#include "dev_util.h"

namespace hgp {

namespace {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

enum { WS_SCAN_PART = 1 };

template <typename Tin, typename Tacc>
__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(const Tin* __restrict__ in, i64 n, Tacc* part) {
    __shared__ Tacc red[16];
    const i64 base = (i64)blockIdx.x * kScanTile;
    Tacc s = 0;
    for (int i = threadIdx.x; i < kScanTile; i += kScanBlock) {
        const i64 idx = base + i;
        if (idx < n) s += (Tacc)in[idx];
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

template <typename Tacc>
__global__ __launch_bounds__(1024) void k_scan_partials(Tacc* part, int nb) {
    __shared__ Tacc red[16];
    Tacc carry = 0;
    for (int base = 0; base < nb; base += 1024) {
        const int i = base + threadIdx.x;
        const Tacc v = i < nb ? part[i] : 0;
        Tacc tot;
        const Tacc ex = block_excl_scan(v, red, &tot);
        if (i < nb) part[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) part[nb] = carry;
}

template <typename Tin, typename Tacc, typename Tout>
__global__ __launch_bounds__(kScanBlock) void k_scan_down(const Tin* __restrict__ in, i64 n,
                                                          const Tacc* __restrict__ part, Tout* out) {
    __shared__ Tacc red[16];
    const i64 base = (i64)blockIdx.x * kScanTile + (i64)threadIdx.x * kScanItems;
    Tacc v[kScanItems];
    Tacc s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? (Tacc)in[base + k] : 0;
        s += v[k];
    }
    Tacc tot;
    const Tacc ex = block_excl_scan(s, red, &tot);
    Tacc run = part[blockIdx.x] + ex;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = (Tout)run;
        run += v[k];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = (Tout)part[gridDim.x];
}

// Whole scan in one workgroup, for arrays small enough that three launches
// would cost more than the work.
constexpr int kScanSingleMax = 1 << 16;

template <typename Tin, typename Tacc, typename Tout>
__global__ __launch_bounds__(1024) void k_scan_single(const Tin* __restrict__ in, i64 n, Tout* out) {
    __shared__ Tacc red[16];
    constexpr i64 kTile = 1024 * kScanItems;
    // the next tile's items are loaded before the current tile is scanned;
    // indices past the end read the last element (n >= 1) and count as 0
    auto load = [&](i64 base0, Tacc (&v)[kScanItems]) {
        const i64 base = base0 + (i64)threadIdx.x * kScanItems;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            const Tacc x = (Tacc)in[min(base + k, n - 1)];
            v[k] = base + k < n ? x : (Tacc)0;
        }
    };
    Tacc nx[kScanItems];
    load(0, nx);
    Tacc carry = 0;
    for (i64 base0 = 0; base0 < n; base0 += kTile) {
        Tacc v[kScanItems];
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) v[k] = nx[k];
        if (base0 + kTile < n) load(base0 + kTile, nx);
        const i64 base = base0 + (i64)threadIdx.x * kScanItems;
        Tacc s = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) s += v[k];
        Tacc tot;
        Tacc run = carry + block_excl_scan(s, red, &tot);
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            if (base + k < n) out[base + k] = (Tout)run;
            run += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) out[n] = (Tout)carry;
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

template <typename Tin, typename Tacc, typename Tout>
void scan_impl(Ctx* c, const Tin* in, Tout* out, i64 n) {
    if (n <= 0) {
        HIPC(hipMemsetAsync(out, 0, sizeof(Tout), c->stream));
        return;
    }
    if (n <= kScanSingleMax) {
        LAUNCH(c, KF_SCAN, (k_scan_single<Tin, Tacc, Tout>), 1, 1024, 0, in, n, out);
        return;
    }
    const int nb = (int)ceil_div(n, kScanTile);
    Tacc* part = wsp<Tacc>(c, WS_SCAN_PART, (size_t)nb + 1);
    LAUNCH(c, KF_SCAN, (k_scan_reduce<Tin, Tacc>), nb, kScanBlock, 0, in, n, part);
    LAUNCH(c, KF_SCAN, (k_scan_partials<Tacc>), 1, 1024, 0, part, nb);
    LAUNCH(c, KF_SCAN, (k_scan_down<Tin, Tacc, Tout>), nb, kScanBlock, 0, in, n, (const Tacc*)part, out);
}

}  // namespace

void scan_excl_i64(Ctx* c, const i64* in, i64* out, i64 n) { scan_impl<i64, i64, i64>(c, in, out, n); }
void scan_excl_i32_to_i64(Ctx* c, const i32* in, i64* out, i64 n) { scan_impl<i32, i64, i64>(c, in, out, n); }
void scan_excl_i32(Ctx* c, const i32* in, i32* out, i64 n) { scan_impl<i32, i64, i32>(c, in, out, n); }

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

void read_back(Ctx* c, const void* dev, i64* host, int count, int elem_bytes) {
    HIPC(hipMemcpyAsync(c->host_scalars, dev, (size_t)count * elem_bytes, hipMemcpyDeviceToHost, c->stream));
    HIPC(hipStreamSynchronize(c->stream));
    for (int i = 0; i < count; ++i) {
        if (elem_bytes == 8) host[i] = ((i64*)c->host_scalars)[i];
        else host[i] = ((i32*)c->host_scalars)[i];
    }
}

}  // namespace hgp
