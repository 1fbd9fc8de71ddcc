// Hypergraph structure kernels: validation of the input (Sec. II-A), the
// node -> h-edge incidence of the dual compressed layout (Sec. IV-B), coarse
// h-edges through the cluster map with pin deduplication (Sec. V-E), and the
// per-h-edge rows of pins(p,e) / pins_in(p,e) (Sec. II-B, Sec. VI-B).
#include "dev_util.h"

namespace hgp {

namespace {

enum { WS_KEYS = 10, WS_KEYS_OUT = 11, WS_VALS = 12, WS_PIN_EDGE = 13, WS_EDGE_TMP = 14, WS_CARD = 15, WS_NSRC = 16 };

// Error bits reported by validation.
enum {
    VE_OFFSETS = 1, VE_EMPTY = 2, VE_NSRC = 4, VE_RANGE = 8, VE_ORDER = 16, VE_OVERLAP = 32, VE_WEIGHT = 64,
    VE_TOO_BIG = 128, VE_NODE_WEIGHT = 256
};
constexpr int kMaxCard = 4096;

// One wave per h-edge.  out[0] |= error bits, out[1] += sum of h-edge
// weights, out[3] = max |e|.
__global__ __launch_bounds__(256) void k_validate_edges(i32 N, i32 E, const i64* __restrict__ he_off,
                                                        const i32* __restrict__ he_nsrc,
                                                        const i32* __restrict__ pins, const i32* __restrict__ hw,
                                                        i64 P, unsigned long long* out) {
    const int lane = lane_id();
    const int wpb = blockDim.x / kWave;
    unsigned long long err = 0, wsum = 0, cmax = 0, wmax = 0;
    for (i64 e = (i64)blockIdx.x * wpb + wave_id(); e < E; e += (i64)gridDim.x * wpb) {
        const i64 a = he_off[e], b = he_off[e + 1];
        if (a < 0 || b > P || b < a) { err |= VE_OFFSETS; continue; }
        if (e == 0 && a != 0) err |= VE_OFFSETS;
        if (e == E - 1 && b != P) err |= VE_OFFSETS;
        const i64 card = b - a;
        if (card == 0) { err |= VE_EMPTY; continue; }
        if (card > kMaxCard) err |= VE_TOO_BIG;
        cmax = cmax > (unsigned long long)card ? cmax : (unsigned long long)card;
        const i32 w = hw ? hw[e] : 1;
        if (w < 1) err |= VE_WEIGHT;
        if (lane == 0) wsum += (unsigned long long)(w > 0 ? w : 0);
        wmax = wmax > (unsigned long long)(w > 0 ? w : 0) ? wmax : (unsigned long long)(w > 0 ? w : 0);
        const i32 ns = he_nsrc[e];
        if (ns < 0 || ns > card) { err |= VE_NSRC; continue; }
        const i64 d0 = a + ns;
        bool bad_range = false;
        for (i64 j = a + lane; j < b; j += kWave) {
            const i32 m = pins[j];
            if (m < 0 || m >= N) { bad_range = true; continue; }
            if (j != a && j != d0) {
                const i32 prev = pins[j - 1];
                if (prev >= m) err |= VE_ORDER;
            }
        }
        if (bad_range) err |= VE_RANGE;
        if (__any(bad_range)) continue;
        // src ∩ dst via binary search of each source in the destination block.
        for (i64 j = a + lane; j < d0; j += kWave) {
            const i32 m = pins[j];
            i64 lo = d0, hi = b;
            while (lo < hi) {
                const i64 mid = (lo + hi) >> 1;
                if (pins[mid] < m) lo = mid + 1;
                else hi = mid;
            }
            const i32 at = pins[lo < b ? lo : b - 1];  // the block is non-empty: j < d0 <= b - 1 here
            if ((int)(lo < b) & (int)(at == m)) err |= VE_OVERLAP;
        }
    }
    err = wave_or(err);
    wsum = wave_sum(wsum);
    cmax = wave_max(cmax);
    wmax = wave_max(wmax);
    if (lane == 0) {
        if (err) atomicOr(&out[0], err);
        atomicAdd(&out[1], wsum);
        atomicMax(&out[3], cmax);
        atomicMax(&out[4], wmax);
    }
}

__global__ __launch_bounds__(256) void k_validate_nodes(i32 N, const i32* __restrict__ nw, unsigned long long* out) {
    unsigned long long err = 0, s = 0;
    for (i64 n = (i64)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (i64)gridDim.x * blockDim.x) {
        const i32 w = nw ? nw[n] : 1;
        if (w < 1) err |= VE_NODE_WEIGHT;
        else s += (unsigned long long)w;
    }
    s = wave_sum(s);
    err = wave_or(err);
    if (lane_id() == 0) {
        if (err) atomicOr(&out[0], err);
        atomicAdd(&out[2], s);
    }
}

// Incidence keys: one wave per h-edge; key = 2*node + (pin is a source),
// value = h-edge id.  A stable sort by key then lists, per node, inbound
// h-edges first and each block ascending (Sec. IV-B).
// Sort keys 2n + [source] and values (h-edge << 32) | pin position, so the
// sorted values give both the incidence entry and its pin slot.
__global__ __launch_bounds__(256) void k_pin_keys(i32 E, const i64* __restrict__ he_off,
                                                  const i32* __restrict__ he_nsrc, const i32* __restrict__ pins,
                                                  u32* keys, u64* vals) {
    const int lane = lane_id();
    const int wpb = blockDim.x / kWave;
    for (i64 e = (i64)blockIdx.x * wpb + wave_id(); e < E; e += (i64)gridDim.x * wpb) {
        const i64 a = he_off[e], b = he_off[e + 1], d0 = a + he_nsrc[e];
        for (i64 j = a + lane; j < b; j += kWave) {
            const i32 n = pins[j];
            keys[j] = ((u32)n << 1) | (j < d0 ? 1u : 0u);
            vals[j] = ((u64)(u32)e << 32) | (u64)(u32)j;
        }
    }
}

// Mean h-edge size below which the flat key kernel is used.
constexpr i64 kPinKeysFlatMean = 32;

// The same keys for levels of small h-edges (a few pins on average), where a
// wave per h-edge leaves most lanes idle: each wave takes 64 consecutive
// h-edges, whose pins form one contiguous range, and walks that range 64 pins
// at a time; a lane finds its pin's h-edge by a binary search over the
// window's start offsets (relative to the window, so 32 bits).
__global__ __launch_bounds__(256) void k_pin_keys_flat(i32 E, const i64* __restrict__ he_off,
                                                       const i32* __restrict__ he_nsrc, const i32* __restrict__ pins,
                                                       u32* keys, u64* vals) {
    const int lane = lane_id();
    const int wpb = blockDim.x / kWave;
    for (i64 base = ((i64)blockIdx.x * wpb + wave_id()) * kWave; base < E; base += (i64)gridDim.x * wpb * kWave) {
        const i64 e = base + lane;
        const int in = (int)(e < E);
        const i64 A = he_off[base];
        const i64 B = he_off[min(base + kWave, (i64)E)];
        const i64 a = he_off[in ? e : E];  // lanes past the end start at B and own nothing
        const i32 rel = (i32)(a - A);
        const i32 srel = rel + (in ? he_nsrc[e] : 0);  // first destination pin, window-relative
        for (i64 j0 = A; j0 < B; j0 += kWave) {
            const i64 j = j0 + lane;
            const i32 jr = (i32)(j - A);
            int o = 0;  // the last lane whose h-edge starts at or before pin j
#pragma unroll
            for (int step = kWave / 2; step >= 1; step >>= 1) {
                const int cand = o + step;
                const i32 sc = __shfl(rel, cand, kWave);
                o = sc <= jr ? cand : o;
            }
            const i32 so = __shfl(srel, o, kWave);
            if (j < B) {
                const i32 n = pins[j];
                keys[j] = ((u32)n << 1) | (jr < so ? 1u : 0u);
                vals[j] = ((u64)(u32)(base + o) << 32) | (u64)(u32)j;
            }
        }
    }
}

__global__ void k_pins16(i64 P, const i32* __restrict__ pins, unsigned short* p16) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (i64)gridDim.x * blockDim.x)
        p16[i] = (unsigned short)pins[i];
}

// h-edge of every incidence entry from its pin position.
__global__ void k_inc_edges(i64 P, const u64* __restrict__ sv, i32* inc, i32* inc_pos) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (i64)gridDim.x * blockDim.x) {
        const u64 v = sv[i];
        inc[i] = (i32)(v >> 32);
        inc_pos[i] = (i32)(u32)v;
    }
}

// Incidence offsets and inbound counts from the sorted keys: node n's entries
// start at the first key >= 2n; its outbound ones at the first key >= 2n+1.
__global__ void k_inc_offsets(i32 N, i64 P, const u32* __restrict__ skeys, i64* inc_off, i32* nin) {
    for (i64 n = (i64)blockIdx.x * blockDim.x + threadIdx.x; n <= N; n += (i64)gridDim.x * blockDim.x) {
        i64 pos[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const u64 key = 2ull * (u64)n + (u64)t;
            i64 l = 0, h = P;
            while (l < h) {
                const i64 mid = (l + h) >> 1;
                const int lt = (int)((u64)skeys[mid] < key);
                l = lt ? mid + 1 : l;
                h = lt ? h : mid;
            }
            pos[t] = l;
        }
        inc_off[n] = pos[0];
        if (n < N) nin[n] = (i32)(pos[1] - pos[0]);
    }
}

// H-edges of at most kSmallEdge pins are handled one lane each, their keys
// sorted in registers by an odd-even transposition network (ascending).
constexpr int kSmallEdge = 8;

template <int S>
__device__ __forceinline__ void reg_sort(u32 (&k)[S]) {
#pragma unroll
    for (int r = 0; r < S; ++r)
#pragma unroll
        for (int i = r & 1; i + 1 < S; i += 2) {
            const u32 x = k[i], y = k[i + 1];
            k[i] = x < y ? x : y;
            k[i + 1] = x < y ? y : x;
        }
}

// Coarse pins of one h-edge per block (Sec. V-E): map pins through gamma,
// sort (id, is_source) in shared memory, keep each coarse id once; an id seen
// among destinations is a destination, otherwise a source.  Written at the
// old offset (|e'| <= |e|); card/nsrc receive the new counts.
__global__ __launch_bounds__(256) void k_contract_edges(i32 E, const i64* __restrict__ he_off,
                                                        const i32* __restrict__ he_nsrc,
                                                        const i32* __restrict__ pins, const i32* __restrict__ gamma,
                                                        i32* tmp, i32* card_out, i32* nsrc_out, int skip_le,
                                                        unsigned long long* bytes) {
    extern __shared__ u32 keys[];
    __shared__ i32 red[16];
    __shared__ i32 s_list[256];
    __shared__ int s_n;
    u64 acc = 0;  // algorithmic bytes of the h-edges this block handled
    // h-edges blockDim.x at a time; those of more than skip_le pins are listed
    // in shared memory and handled one after another
    for (i64 base = (i64)blockIdx.x * blockDim.x; base < E; base += (i64)gridDim.x * blockDim.x) {
      if (threadIdx.x == 0) s_n = 0;
      __syncthreads();
      {
        const i64 el = base + threadIdx.x;
        if ((el < E) && (he_off[el + 1] - he_off[el] > (i64)skip_le)) s_list[atomicAdd(&s_n, 1)] = (i32)el;
      }
      __syncthreads();
      const int nl = s_n;
      for (int li = 0; li < nl; ++li) {
        const i64 e = s_list[li];
        const i64 a = he_off[e];
        const int card = (int)(he_off[e + 1] - a), ns = he_nsrc[e];
        const int npad = next_pow2(card);
        for (int i = threadIdx.x; i < npad; i += blockDim.x)
            keys[i] = i < card ? (((u32)gamma[pins[a + i]] << 1) | (i < ns ? 1u : 0u)) : 0xFFFFFFFFu;
        __syncthreads();
        block_bitonic_sort_u32(keys, npad);
        // count sources first, then write sources and destinations.
        i32 nsrc_new = 0;
        for (int base = 0; base < card; base += blockDim.x) {
            const int i = base + threadIdx.x;
            const int ic = i < card ? i : 0;
            const u32 kc = keys[ic], kp = keys[ic > 0 ? ic - 1 : 0];
            const bool head = ((int)(i < card) & ((int)(i == 0) | (int)((kc >> 1) != (kp >> 1)))) != 0;
            nsrc_new += block_sum((i32)(head & ((kc & 1u) != 0)), red);
        }
        i32 run_s = 0, run_d = 0;
        for (int base = 0; base < card; base += blockDim.x) {
            const int i = base + threadIdx.x;
            const int ic = i < card ? i : 0;
            const u32 kc = keys[ic], kp = keys[ic > 0 ? ic - 1 : 0];
            const bool head = ((int)(i < card) & ((int)(i == 0) | (int)((kc >> 1) != (kp >> 1)))) != 0;
            const bool fs = head & ((kc & 1u) != 0), fd = head & ((kc & 1u) == 0);
            i32 ts, td;
            const i32 xs = block_excl_scan((i32)fs, red, &ts);
            const i32 xd = block_excl_scan((i32)fd, red, &td);
            if (fs) tmp[a + run_s + xs] = (i32)(kc >> 1);
            if (fd) tmp[a + nsrc_new + run_d + xd] = (i32)(kc >> 1);
            run_s += ts;
            run_d += td;
        }
        if (threadIdx.x == 0) {
            card_out[e] = run_s + run_d;
            nsrc_out[e] = run_s;
        }
        // offsets and |src| read, pins and their cluster ids read, the
        // coarse pins and the two counts written
        acc += 20 + 8 * (u64)card + 4 * (u64)(run_s + run_d);
        __syncthreads();
      }
    }
    if ((bytes != nullptr) & (threadIdx.x == 0) & (acc != 0)) atomicAdd(bytes, (unsigned long long)acc);
}

// Compacts per-h-edge segments written at old offsets into the new layout.
// Each wave takes a window of up to 64 h-edges (64 whenever the grid, sized
// for 64 per wave, is not capped): segments of at most kSmallEdge pins are copied
// one lane each, longer ones by the whole wave (kept by ballot).
__global__ __launch_bounds__(256) void k_pack_edges(i32 E, const i64* __restrict__ old_off,
                                                    const i64* __restrict__ new_off, const i32* __restrict__ tmp,
                                                    i32* out, unsigned long long* bytes) {
    const int lane = lane_id();
    const int wpb = blockDim.x / kWave;
    const i64 nw = (i64)gridDim.x * wpb, win = wave_window(E, nw);
    u64 acc = 0;
    for (i64 base = ((i64)blockIdx.x * wpb + wave_id()) * win; base < E; base += nw * win) {
        const i64 el = base + lane;
        const int in = (int)(lane < win) & (int)(el < E);
        const i64 ec = in ? el : 0;
        const i64 al = old_off[ec], ol = new_off[ec];
        const i64 nl = in ? new_off[ec + 1] - ol : 0;
        if (nl <= kSmallEdge) {
            i32 v[kSmallEdge];
#pragma unroll
            for (int j = 0; j < kSmallEdge; ++j) v[j] = j < nl ? tmp[al + j] : 0;
#pragma unroll
            for (int j = 0; j < kSmallEdge; ++j)
                if (j < nl) out[ol + j] = v[j];
        }
        acc += in ? 16 + 8 * (u64)nl : 0;  // both offsets; each pin read once and written once
        u64 todo = __ballot((int)(nl > kSmallEdge));
        while (todo) {
            const int src = __builtin_ctzll(todo);
            todo &= todo - 1;
            const i64 a = __shfl(al, src, kWave), o = __shfl(ol, src, kWave), n = __shfl(nl, src, kWave);
            for (i64 j = lane; j < n; j += kWave) out[o + j] = tmp[a + j];
        }
    }
    const u64 tot = bytes != nullptr ? (u64)wave_sum((i64)acc) : 0;
    if ((bytes != nullptr) & (lane == 0) & (tot != 0)) atomicAdd(bytes, (unsigned long long)tot);
}

// Algorithmic bytes of one h-edge's rows: offsets, |src| and lambda (16), its
// pins and their partition ids read (8 per pin), part / cnt / cnt_in written
// (12 per row), plus the 16-bit copy (2 per row) and the `single` bytes (1 per
// pin) when asked for.
__device__ __forceinline__ u64 phi_edge_bytes(int card, int rows, bool single, bool part16) {
    return 16 + 8 * (u64)card + (12 + (part16 ? 2 : 0)) * (u64)rows + (single ? (u64)card : 0);
}

// pins(p,e) and pins_in(p,e) of one h-edge per block: sort (rho(pin), is_dst)
// in shared memory and run-length count.  Rows are written at the h-edge's pin
// offset, ascending p; len[e] = lambda(e).
// With `single` non-null, also writes one byte per pin slot: 1 when the
// pin's partition holds no other pin of the h-edge (pins(rho(m), e) = 1).
// Shared memory then holds two more arrays (the unsorted keys and the row of
// each sorted position).
__global__ __launch_bounds__(256) void k_phi(i32 E, const i64* __restrict__ he_off, const i32* __restrict__ he_nsrc,
                                             const i32* __restrict__ pins, const i32* __restrict__ rho,
                                             i32* part, i32* cnt, i32* cnt_in, i32* len, unsigned char* single,
                                             unsigned short* part16, const i32* __restrict__ elist,
                                             const u32* __restrict__ ecount, int npad_max, int skip_le,
                                             unsigned long long* bytes) {
    extern __shared__ u32 sm[];
    __shared__ i32 red[16];
    __shared__ i32 s_list[256];
    __shared__ int s_n;
    u64 acc = 0;
    const i64 ne = elist ? (i64)*ecount : (i64)E;
    // list entries blockDim.x at a time; h-edges of more than skip_le pins are
    // listed in shared memory and handled one after another
    for (i64 base = (i64)blockIdx.x * blockDim.x; base < ne; base += (i64)gridDim.x * blockDim.x) {
      if (threadIdx.x == 0) s_n = 0;
      __syncthreads();
      {
        const i64 il = base + threadIdx.x;
        if (il < ne) {
            const i64 el = elist ? (i64)elist[il] : il;
            if (he_off[el + 1] - he_off[el] > (i64)skip_le) s_list[atomicAdd(&s_n, 1)] = (i32)el;
        }
      }
      __syncthreads();
      const int nl = s_n;
      for (int li = 0; li < nl; ++li) {
        const i64 e = s_list[li];
        const i64 a = he_off[e];
        const int card = (int)(he_off[e + 1] - a), ns = he_nsrc[e];
        const int npad = next_pow2(card);
        u32* keys = sm;
        i32* c_all = (i32*)(sm + npad);
        i32* c_in = c_all + npad;
        i32* rpart = (i32*)(sm + 3 * npad_max);       // partition of each row
        u32* orig = sm + 4 * npad_max;                // unsorted keys (with `single`)
        i32* rowat = (i32*)(sm + 5 * npad_max);       // row of each sorted position
        for (int i = threadIdx.x; i < npad; i += blockDim.x) {
            const u32 k = i < card ? (((u32)rho[pins[a + i]] << 1) | (i >= ns ? 1u : 0u)) : 0xFFFFFFFFu;
            keys[i] = k;
            if (single) orig[i] = k;
            c_all[i] = 0;
            c_in[i] = 0;
        }
        __syncthreads();
        block_bitonic_sort_u32(keys, npad);
        i32 rows = 0;
        for (int base = 0; base < card; base += blockDim.x) {
            const int i = base + threadIdx.x;
            const int ic = i < card ? i : 0;
            const u32 kc = keys[ic], kp = keys[ic > 0 ? ic - 1 : 0];
            const bool head = ((int)(i < card) & ((int)(i == 0) | (int)((kc >> 1) != (kp >> 1)))) != 0;
            i32 tot;
            const i32 x = block_excl_scan((i32)head, red, &tot);
            if (i < card) {
                const i32 r = rows + x + (head ? 1 : 0) - 1;  // row of element i
                if (head) {
                    part[a + r] = (i32)(kc >> 1);
                    rpart[r] = (i32)(kc >> 1);
                }
                atomicAdd(&c_all[r], 1);
                if (kc & 1u) atomicAdd(&c_in[r], 1);
                if (single) rowat[i] = r;
            }
            rows += tot;
        }
        __syncthreads();
        for (int r = threadIdx.x; r < rows; r += blockDim.x) {
            cnt[a + r] = c_all[r];
            cnt_in[a + r] = c_in[r];
            // 16-bit copy for the gains sweep: partition id, top bit where pins(p,e) = 1
            if (part16) part16[a + r] = (unsigned short)((u32)rpart[r] | (c_all[r] == 1 ? 0x8000u : 0u));
        }
        if (single) {
            for (int i = threadIdx.x; i < card; i += blockDim.x) {
                const u32 k = orig[i];
                int lo = 0, hi = card;  // first sorted position with key >= k (the key is present)
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    const int lt = (int)(keys[mid] < k);
                    lo = lt ? mid + 1 : lo;
                    hi = lt ? hi : mid;
                }
                single[a + i] = (unsigned char)(c_all[rowat[lo]] == 1 ? 1 : 0);
            }
        }
        if (threadIdx.x == 0) len[e] = rows;
        acc += phi_edge_bytes(card, rows, single != nullptr, part16 != nullptr);
        __syncthreads();
      }
    }
    if ((bytes != nullptr) & (threadIdx.x == 0) & (acc != 0)) atomicAdd(bytes, (unsigned long long)acc);
}

// ---- one wave per h-edge of at most 256 pins --------------------------------
// The h-edge's keys are sorted in registers (wave_bitonic_sort, KPL keys per
// lane, blocked), runs are found by comparing each key with its predecessor,
// and outputs are placed by wave scans: no block barriers and no shared
// memory for the sort.  Results are those of the block kernels above.
constexpr int kWaveEdgeMax = 256;

// In-lane inclusive prefix of flags and the wave-exclusive offset of the lane.
template <int KPL>
__device__ __forceinline__ i32 lane_offsets(const int (&f)[KPL], i32 (&pre)[KPL], i32& total) {
    i32 c = 0;
#pragma unroll
    for (int r = 0; r < KPL; ++r) {
        c += f[r];
        pre[r] = c;
    }
    const i32 incl = wave_incl_scan(c);
    total = __shfl(incl, kWave - 1, kWave);
    return incl - c;
}

template <int KPL>
__device__ __forceinline__ void contract_edge_wave(i64 a, int card, int ns, const i32* __restrict__ pins,
                                                   const i32* __restrict__ gamma, i32* tmp, i32& ncard, i32& nsrc) {
    const int lane = lane_id();
    u32 v[KPL];
#pragma unroll
    for (int r = 0; r < KPL; ++r) {
        const int pos = lane * KPL + r;
        v[r] = pos < card ? (((u32)gamma[pins[a + pos]] << 1) | (pos < ns ? 1u : 0u)) : 0xFFFFFFFFu;
    }
    wave_bitonic_sort<KPL>(v);
    const u32 last = (u32)__shfl_up((int)v[KPL - 1], 1, kWave);
    int fs[KPL], fd[KPL];
#pragma unroll
    for (int r = 0; r < KPL; ++r) {
        const int pos = lane * KPL + r;
        const u32 prev = r > 0 ? v[r - 1] : last;
        const int head = (int)(pos < card) & ((int)(pos == 0) | (int)((v[r] >> 1) != (prev >> 1)));
        fs[r] = head & (int)((v[r] & 1u) != 0);  // a cluster with a destination pin is a destination
        fd[r] = head & (int)((v[r] & 1u) == 0);
    }
    i32 ps[KPL], pd[KPL], ts, td;
    const i32 os = lane_offsets<KPL>(fs, ps, ts);
    const i32 od = lane_offsets<KPL>(fd, pd, td);
#pragma unroll
    for (int r = 0; r < KPL; ++r) {
        if (fs[r]) tmp[a + os + ps[r] - 1] = (i32)(v[r] >> 1);
        if (fd[r]) tmp[a + ts + od + pd[r] - 1] = (i32)(v[r] >> 1);
    }
    ncard = ts + td;
    nsrc = ts;
}

__global__ __launch_bounds__(256) void k_contract_edges_wave(i32 E, const i64* __restrict__ he_off,
                                                             const i32* __restrict__ he_nsrc,
                                                             const i32* __restrict__ pins,
                                                             const i32* __restrict__ gamma, i32* tmp, i32* card_out,
                                                             i32* nsrc_out, unsigned long long* bytes) {
    const int wpb = blockDim.x / kWave;
    const int lane = lane_id();
    const i64 nw = (i64)gridDim.x * wpb, win = wave_window(E, nw);
    u64 acc = 0;
    // a window of h-edges at a time; those of kSmallEdge < |e| <= kWaveEdgeMax
    // pins are kept by ballot (smaller ones: k_contract_small, larger: the
    // block kernel)
    for (i64 base = ((i64)blockIdx.x * wpb + wave_id()) * win; base < E; base += nw * win) {
      const i64 el = base + lane;
      const int in = (int)(lane < win) & (int)(el < E);
      const i64 ec = in ? el : 0;
      const i64 al = he_off[ec];
      const int cl = (int)(he_off[ec + 1] - al), nsl = he_nsrc[ec];
      u64 todo = __ballot(in & (int)(cl > kSmallEdge) & (int)(cl <= kWaveEdgeMax));
      while (todo) {
        const int src = __builtin_ctzll(todo);
        todo &= todo - 1;
        const i64 e = base + src;
        const i64 a = __shfl(al, src, kWave);
        const int card = __shfl(cl, src, kWave), ns = __shfl(nsl, src, kWave);
        i32 nc, nsv;
        if (card <= 64) contract_edge_wave<1>(a, card, ns, pins, gamma, tmp, nc, nsv);
        else if (card <= 128) contract_edge_wave<2>(a, card, ns, pins, gamma, tmp, nc, nsv);
        else contract_edge_wave<4>(a, card, ns, pins, gamma, tmp, nc, nsv);
        if (lane == 0) {
            card_out[e] = nc;
            nsrc_out[e] = nsv;
        }
        // offsets and |src| read, pins and their cluster ids read, the
        // coarse pins and the two counts written
        acc += 20 + 8 * (u64)card + 4 * (u64)nc;
      }
    }
    if ((bytes != nullptr) & (lane == 0) & (acc != 0)) atomicAdd(bytes, (unsigned long long)acc);
}

// Coarse pins of h-edges of at most kSmallEdge pins, one lane per h-edge: the
// keys (cluster << 1 | source flag) sorted in registers, each cluster kept
// once, sources first; the same result as contract_edge_wave.
__global__ __launch_bounds__(256) void k_contract_small(i32 E, const i64* __restrict__ he_off,
                                                        const i32* __restrict__ he_nsrc, const i32* __restrict__ pins,
                                                        const i32* __restrict__ gamma, i32* tmp, i32* card_out,
                                                        i32* nsrc_out, unsigned long long* bytes) {
    constexpr int S = kSmallEdge;
    u64 acc = 0;
    for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += (i64)gridDim.x * blockDim.x) {
        const i64 a = he_off[e];
        const int card = (int)(he_off[e + 1] - a);
        if (card > S) continue;
        if (card <= 0) {
            card_out[e] = 0;
            nsrc_out[e] = 0;
            acc += 20;
            continue;
        }
        const int ns = he_nsrc[e];
        i32 m[S];
        u32 k[S];
#pragma unroll
        for (int j = 0; j < S; ++j) m[j] = pins[a + (j < card ? j : 0)];
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const u32 g = (u32)gamma[m[j]];
            k[j] = j < card ? ((g << 1) | (j < ns ? 1u : 0u)) : 0xFFFFFFFFu;
        }
        reg_sort<S>(k);
        int ts = 0;
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const int head = (int)(j < card) & ((int)(j == 0) | (int)((k[j] >> 1) != (k[j > 0 ? j - 1 : 0] >> 1)));
            ts += head & (int)((k[j] & 1u) != 0);
        }
        int os = 0, od = 0;
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const int head = (int)(j < card) & ((int)(j == 0) | (int)((k[j] >> 1) != (k[j > 0 ? j - 1 : 0] >> 1)));
            if (head) {
                if (k[j] & 1u) tmp[a + os++] = (i32)(k[j] >> 1);
                else tmp[a + ts + od++] = (i32)(k[j] >> 1);
            }
        }
        card_out[e] = os + od;
        nsrc_out[e] = os;
        acc += 20 + 8 * (u64)card + 4 * (u64)(os + od);
    }
    const u64 tot = bytes != nullptr ? (u64)wave_sum((i64)acc) : 0;
    if ((bytes != nullptr) & (lane_id() == 0) & (tot != 0)) atomicAdd(bytes, (unsigned long long)tot);
}

// Phi rows of one h-edge in one wave.  Shared memory per wave: the sorted
// keys and the row of each sorted position (for `single`), the row counts.
struct PhiWaveShared {
    u32 keys[kWaveEdgeMax];
    i32 rowat[kWaveEdgeMax];
    i32 c_all[kWaveEdgeMax];
    i32 c_in[kWaveEdgeMax];
    i32 rpart[kWaveEdgeMax];  // partition of each row
};

template <int KPL>
__device__ __forceinline__ void phi_edge_wave(PhiWaveShared& sh, i64 a, int card, int ns, const i32* __restrict__ pins,
                                              const i32* __restrict__ rho, i32* part, i32* cnt, i32* cnt_in,
                                              unsigned char* single, unsigned short* part16, i32& rows) {
    const int lane = lane_id();
    u32 v[KPL], orig[KPL];
#pragma unroll
    for (int r = 0; r < KPL; ++r) {
        const int pos = lane * KPL + r;
        v[r] = pos < card ? (((u32)rho[pins[a + pos]] << 1) | (pos >= ns ? 1u : 0u)) : 0xFFFFFFFFu;
        orig[r] = v[r];
        sh.c_all[pos] = 0;
        sh.c_in[pos] = 0;
    }
    wave_bitonic_sort<KPL>(v);
    const u32 last = (u32)__shfl_up((int)v[KPL - 1], 1, kWave);
    int hd[KPL];
#pragma unroll
    for (int r = 0; r < KPL; ++r) {
        const int pos = lane * KPL + r;
        const u32 prev = r > 0 ? v[r - 1] : last;
        hd[r] = (int)(pos < card) & ((int)(pos == 0) | (int)((v[r] >> 1) != (prev >> 1)));
    }
    i32 pre[KPL];
    const i32 off = lane_offsets<KPL>(hd, pre, rows);
    wave_sync();  // counters cleared
#pragma unroll
    for (int r = 0; r < KPL; ++r) {
        const int pos = lane * KPL + r;
        if (pos < card) {
            const i32 row = off + pre[r] - 1;
            if (hd[r]) {
                part[a + row] = (i32)(v[r] >> 1);
                sh.rpart[row] = (i32)(v[r] >> 1);
            }
            atomicAdd(&sh.c_all[row], 1);
            if (v[r] & 1u) atomicAdd(&sh.c_in[row], 1);
            sh.keys[pos] = v[r];
            sh.rowat[pos] = row;
        }
    }
    wave_sync();
    for (int r = lane; r < rows; r += kWave) {
        cnt[a + r] = sh.c_all[r];
        cnt_in[a + r] = sh.c_in[r];
        // 16-bit copy for the gains sweep: partition id, top bit where pins(p,e) = 1
        if (part16) part16[a + r] = (unsigned short)((u32)sh.rpart[r] | (sh.c_all[r] == 1 ? 0x8000u : 0u));
    }
    if (single) {
#pragma unroll
        for (int r = 0; r < KPL; ++r) {
            const int pos = lane * KPL + r;
            if (pos < card) {
                const u32 k = orig[r];
                int lo = 0, hi = card;  // first sorted position with key >= k (the key is present)
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    const int lt = (int)(sh.keys[mid] < k);
                    lo = lt ? mid + 1 : lo;
                    hi = lt ? hi : mid;
                }
                single[a + pos] = (unsigned char)(sh.c_all[sh.rowat[lo]] == 1 ? 1 : 0);
            }
        }
    }
    wave_sync();  // shared memory is reused by the wave's next h-edge
}

// With elist, only the h-edges it lists (*ecount of them) are rebuilt.
__global__ __launch_bounds__(256) void k_phi_wave(i32 E, const i64* __restrict__ he_off,
                                                  const i32* __restrict__ he_nsrc, const i32* __restrict__ pins,
                                                  const i32* __restrict__ rho, i32* part, i32* cnt, i32* cnt_in,
                                                  i32* len, unsigned char* single, unsigned short* part16,
                                                  const i32* __restrict__ elist, const u32* __restrict__ ecount,
                                                  unsigned long long* bytes) {
    __shared__ PhiWaveShared sh[4];
    const int wpb = blockDim.x / kWave;
    const int lane = lane_id();
    PhiWaveShared& my = sh[wave_id()];
    u64 acc = 0;
    const i64 ne = elist ? (i64)*ecount : (i64)E;
    const i64 nw = (i64)gridDim.x * wpb, win = wave_window(ne, nw);
    // a window of list entries at a time; h-edges of kSmallEdge < |e| <=
    // kWaveEdgeMax pins are kept by ballot (smaller ones: k_phi_small, larger:
    // k_phi)
    for (i64 base = ((i64)blockIdx.x * wpb + wave_id()) * win; base < ne; base += nw * win) {
      const i64 il = base + lane;
      const int in = (int)(lane < win) & (int)(il < ne);
      const i64 el = in ? (elist ? (i64)elist[il] : il) : 0;
      const i64 al = he_off[el];
      const int cl = (int)(he_off[el + 1] - al), nsl = he_nsrc[el];
      u64 todo = __ballot(in & (int)(cl > kSmallEdge) & (int)(cl <= kWaveEdgeMax));
      while (todo) {
        const int src = __builtin_ctzll(todo);
        todo &= todo - 1;
        const i64 e = __shfl(el, src, kWave);
        const i64 a = __shfl(al, src, kWave);
        const int card = __shfl(cl, src, kWave), ns = __shfl(nsl, src, kWave);
        i32 rows;
        if (card <= 64) phi_edge_wave<1>(my, a, card, ns, pins, rho, part, cnt, cnt_in, single, part16, rows);
        else if (card <= 128) phi_edge_wave<2>(my, a, card, ns, pins, rho, part, cnt, cnt_in, single, part16, rows);
        else phi_edge_wave<4>(my, a, card, ns, pins, rho, part, cnt, cnt_in, single, part16, rows);
        if (lane == 0) len[e] = rows;
        acc += phi_edge_bytes(card, rows, single != nullptr, part16 != nullptr);
      }
    }
    if ((bytes != nullptr) & (lane == 0) & (acc != 0)) atomicAdd(bytes, (unsigned long long)acc);
}

// Phi rows of h-edges of at most kSmallEdge pins, one lane per h-edge: the
// keys (partition << 1 | destination flag) sorted in registers and
// run-length counted; the same rows as phi_edge_wave.
__global__ __launch_bounds__(256) void k_phi_small(i32 E, const i64* __restrict__ he_off,
                                                   const i32* __restrict__ he_nsrc, const i32* __restrict__ pins,
                                                   const i32* __restrict__ rho, i32* part, i32* cnt, i32* cnt_in,
                                                   i32* len, unsigned char* single, unsigned short* part16,
                                                   const i32* __restrict__ elist, const u32* __restrict__ ecount,
                                                   unsigned long long* bytes) {
    constexpr int S = kSmallEdge;
    u64 acc = 0;
    const i64 ne = elist ? (i64)*ecount : (i64)E;
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < ne; i += (i64)gridDim.x * blockDim.x) {
        const i64 e = elist ? (i64)elist[i] : i;
        const i64 a = he_off[e];
        const int card = (int)(he_off[e + 1] - a);
        if (card > S) continue;
        if (card <= 0) {
            len[e] = 0;
            acc += phi_edge_bytes(0, 0, single != nullptr, part16 != nullptr);
            continue;
        }
        const int ns = he_nsrc[e];
        i32 m[S];
        u32 k[S], orig[S];
#pragma unroll
        for (int j = 0; j < S; ++j) m[j] = pins[a + (j < card ? j : 0)];
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const u32 pr = (u32)rho[m[j]];
            k[j] = j < card ? ((pr << 1) | (j >= ns ? 1u : 0u)) : 0xFFFFFFFFu;
            orig[j] = k[j];
        }
        reg_sort<S>(k);
        int rows = 0;
        i32 ca = 0, ci = 0;
#pragma unroll
        for (int j = 0; j < S; ++j) {
            if (j < card) {
                ca += 1;
                ci += (int)(k[j] & 1u);
                const int last = (int)(j + 1 == card) | (int)(j + 1 < S && (k[j + 1 < S ? j + 1 : j] >> 1) != (k[j] >> 1));
                if (last) {
                    part[a + rows] = (i32)(k[j] >> 1);
                    cnt[a + rows] = ca;
                    cnt_in[a + rows] = ci;
                    // 16-bit copy for the gains sweep: partition id, top bit where pins(p,e) = 1
                    if (part16) part16[a + rows] = (unsigned short)((k[j] >> 1) | (ca == 1 ? 0x8000u : 0u));
                    ++rows;
                    ca = 0;
                    ci = 0;
                }
            }
        }
        len[e] = rows;
        if (single) {
#pragma unroll
            for (int j = 0; j < S; ++j) {
                if (j < card) {
                    int same = 0;
#pragma unroll
                    for (int o = 0; o < S; ++o) same += (int)(o < card) & (int)((orig[o] >> 1) == (orig[j] >> 1));
                    single[a + j] = (unsigned char)(same == 1 ? 1 : 0);
                }
            }
        }
        acc += phi_edge_bytes(card, rows, single != nullptr, part16 != nullptr);
    }
    const u64 tot = bytes != nullptr ? (u64)wave_sum((i64)acc) : 0;
    if ((bytes != nullptr) & (lane_id() == 0) & (tot != 0)) atomicAdd(bytes, (unsigned long long)tot);
}

int bits_for(u64 v) {
    int b = 0;
    while (b < 64 && (v >> b) != 0) ++b;
    return b;
}

}  // namespace

void validate_graph(Ctx* c, i32 N, i32 E, const i64* he_off, const i32* he_nsrc, const i32* pins, const i32* hw,
                    const i32* nw, i64 P, i64* d_out) {
    HIPC(hipMemsetAsync(d_out, 0, 5 * sizeof(i64), c->stream));
    if (E > 0)
        LAUNCH(c, KF_VALIDATE, k_validate_edges, grid_for(E, 4, c->num_cu * 16), 256, 0, N, E, he_off, he_nsrc,
               pins, hw, P, (unsigned long long*)d_out);
    LAUNCH(c, KF_VALIDATE, k_validate_nodes, grid_for(N, 256, c->num_cu * 4), 256, 0, N, nw,
           (unsigned long long*)d_out);
}

void build_incidence(Ctx* c, Level& L) {
    const i64 P = L.P;
    u32* keys = wsp<u32>(c, WS_KEYS, P);
    u32* keys_out = wsp<u32>(c, WS_KEYS_OUT, P);
    u64* vals = wsp<u64>(c, WS_VALS, P);
    u64* vals_out = wsp<u64>(c, WS_PIN_EDGE, P);
    if (P > 0x7FFFFFFF) fail(HGP_E_UNSUPPORTED, "more than 2^31 - 1 pins in one level");
    L.b_inc_nin = c->alloc(sizeof(i32) * (size_t)L.N);
    L.b_inc_off = c->alloc(sizeof(i64) * ((size_t)L.N + 1));
    L.b_inc = c->alloc(sizeof(i32) * (size_t)(P > 0 ? P : 1));
    L.b_inc_pos = c->alloc(sizeof(i32) * (size_t)(P > 0 ? P : 1));
    if (L.E > 0) {
        if (P < (i64)kPinKeysFlatMean * L.E)  // a few pins per h-edge: flat over each window's pins
            LAUNCH(c, KF_TRANSPOSE, k_pin_keys_flat, grid_for(ceil_div((i64)L.E, (i64)kWave), 4, c->num_cu * 16), 256,
                   0, L.E, L.he_off(), L.he_nsrc(), L.pins(), keys, vals);
        else
            LAUNCH(c, KF_TRANSPOSE, k_pin_keys, grid_for(L.E, 4, c->num_cu * 16), 256, 0, L.E, L.he_off(),
                   L.he_nsrc(), L.pins(), keys, vals);
    }
    // Stable sort by (node, source flag): per node its inbound h-edges first,
    // each group in ascending h-edge order, since pins are stored by h-edge.
    sort_pairs_u32_u64(c, keys, keys_out, vals, vals_out, P, bits_for(2ull * (u64)L.N));
    if (L.N <= 65536 && P > 0) {
        L.b_pins16 = c->alloc(sizeof(unsigned short) * (size_t)P);
        LAUNCH(c, KF_TRANSPOSE, k_pins16, grid_for(P, 256, c->num_cu * 8), 256, 0, P, (const i32*)L.pins(),
               (unsigned short*)L.b_pins16.p);
    }
    if (P > 0)
        LAUNCH(c, KF_TRANSPOSE, k_inc_edges, grid_for(P, 256, c->num_cu * 8), 256, 0, P, (const u64*)vals_out,
               L.inc(), L.inc_pos());
    LAUNCH(c, KF_TRANSPOSE, k_inc_offsets, grid_for((i64)L.N + 1, 256, c->num_cu * 8), 256, 0, L.N, P,
           (const u32*)keys_out, L.inc_off(), L.inc_nin());
}

void contract_edges(Ctx* c, const Level& L, const i32* gamma, Level& out) {
    const i32 E = L.E;
    out.E = E;
    out.b_he_off = c->alloc(sizeof(i64) * ((size_t)E + 1));
    out.b_he_nsrc = c->alloc(sizeof(i32) * (size_t)(E > 0 ? E : 1));
    i32* tmp = wsp<i32>(c, WS_EDGE_TMP, (size_t)L.P + 1);
    i32* card = wsp<i32>(c, WS_CARD, (size_t)E + 1);
    if (E > 0) {
        // the input's largest h-edge bounds every level (|e'| <= |e|)
        const int npad = next_pow2(c->max_card);
        LAUNCH(c, KF_CONTRACT_EDGES, k_contract_small, grid_for(E, 256, c->num_cu * 8), 256, 0, E, L.he_off(),
               L.he_nsrc(), L.pins(), gamma, tmp, card, out.he_nsrc(), prof_bytes(c, KF_CONTRACT_EDGES));
        if (c->max_card > kSmallEdge)
            LAUNCH(c, KF_CONTRACT_EDGES, k_contract_edges_wave, grid_for(ceil_div((i64)E, (i64)kWindowMin), 4,
                   c->num_cu * 16), 256, 0, E, L.he_off(), L.he_nsrc(), L.pins(), gamma, tmp, card, out.he_nsrc(),
                   prof_bytes(c, KF_CONTRACT_EDGES));
        if (c->max_card > kWaveEdgeMax)
            LAUNCH(c, KF_CONTRACT_EDGES, k_contract_edges, grid_for(E, 256, c->num_cu * 16), 256,
                   sizeof(u32) * npad, E, L.he_off(), L.he_nsrc(), L.pins(), gamma, tmp, card, out.he_nsrc(),
                   kWaveEdgeMax, prof_bytes(c, KF_CONTRACT_EDGES));
    }
    scan_excl_i32_to_i64(c, card, out.he_off(), E);
    i64 P2 = 0;
    read_back(c, out.he_off() + E, &P2, 1, 8);
    out.P = P2;
    out.b_pins = c->alloc(sizeof(i32) * (size_t)(P2 > 0 ? P2 : 1));
    if (E > 0)
        LAUNCH(c, KF_PACK, k_pack_edges, grid_for(ceil_div((i64)E, (i64)kWave), 4, c->num_cu * 16), 256, 0, E,
               L.he_off(),
               (const i64*)out.he_off(), (const i32*)tmp, out.pins(), prof_bytes(c, KF_PACK));
}

// Pin roles of one h-edge per block, staged in shared memory (|e| <= 4,096):
// mode 1 writes the destination block first and makes it the sources; mode 2
// merges the two sorted blocks into one (each pin's place is its index in its
// own block plus the count of smaller pins in the other; the blocks are
// disjoint) with no sources.
__global__ __launch_bounds__(256) void k_retarget(i32 E, const i64* __restrict__ he_off, i32* he_nsrc, i32* pins,
                                                  int mode) {
    __shared__ i32 sp[kMaxCard];
    for (i64 e = blockIdx.x; e < E; e += gridDim.x) {
        const i64 a = he_off[e];
        const int card = (int)(he_off[e + 1] - a), ns = he_nsrc[e], nd = card - ns;
        for (int i = threadIdx.x; i < card; i += blockDim.x) sp[i] = pins[a + i];
        __syncthreads();
        for (int i = threadIdx.x; i < card; i += blockDim.x) {
            const i32 v = sp[i];
            const int src = (int)(i < ns);
            int pos;
            if (mode == 1) {
                pos = src ? nd + i : i - ns;
            } else {
                const int lo0 = src ? ns : 0, hi0 = src ? card : ns;  // the other block
                int lo = lo0, hi = hi0;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    const int lt = (int)(sp[mid] < v);
                    lo = lt ? mid + 1 : lo;
                    hi = lt ? hi : mid;
                }
                pos = (src ? i : i - ns) + (lo - lo0);
            }
            pins[a + pos] = v;
        }
        if (threadIdx.x == 0) he_nsrc[e] = mode == 1 ? nd : 0;
        __syncthreads();
    }
}

void retarget_pins(Ctx* c, Level& L, int mode) {
    if (L.E == 0) return;
    LAUNCH(c, KF_VALIDATE, k_retarget, grid_for(L.E, 1, c->num_cu * 16), 256, 0, L.E, L.he_off(), L.he_nsrc(),
           L.pins(), mode);
}

void build_phi(Ctx* c, const Level& L, const i32* rho, i32* part, i32* cnt, i32* cnt_in, i32* len,
               unsigned char* single, unsigned short* part16, const i32* elist, const u32* ecount) {
    if (L.E == 0) return;
    const int npad = next_pow2(c->max_card);
    // h-edges of at most kSmallEdge pins one lane each, up to kWaveEdgeMax one
    // wave each, larger ones one block each
    LAUNCH(c, KF_PHI, k_phi_small, grid_for(L.E, 256, c->num_cu * 8), 256, 0, L.E, L.he_off(), L.he_nsrc(),
           L.pins(), rho, part, cnt, cnt_in, len, single, part16, elist, ecount, prof_bytes(c, KF_PHI));
    if (c->max_card > kSmallEdge)
        LAUNCH(c, KF_PHI, k_phi_wave, grid_for(ceil_div((i64)L.E, (i64)kWindowMin), 4, c->num_cu * 16), 256, 0, L.E,
               L.he_off(), L.he_nsrc(), L.pins(), rho, part, cnt, cnt_in, len, single, part16, elist, ecount,
               prof_bytes(c, KF_PHI));
    if (c->max_card > kWaveEdgeMax)
        LAUNCH(c, KF_PHI, k_phi, grid_for(L.E, 256, c->num_cu * 16), 256, sizeof(u32) * (single ? 6 : 4) * npad, L.E,
               L.he_off(), L.he_nsrc(), L.pins(), rho, part, cnt, cnt_in, len, single, part16, elist, ecount, npad,
               kWaveEdgeMax, prof_bytes(c, KF_PHI));
}

}  // namespace hgp
