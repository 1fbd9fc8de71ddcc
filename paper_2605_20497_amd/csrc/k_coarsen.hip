// Coarsening of one level (Sec. V): candidate-pair proposal with the neighbour
// histogram, Pi rounds of exact maximum-weight matching on the proposal
// pseudo-forest, best-effort pairing of isolated nodes, the cluster map gamma
// and the coarse hypergraph.
#include <algorithm>

#include <type_traits>

#include "dev_util.h"
#include "top_select.h"

namespace hgp {

namespace {

enum {
    WS_STATS = 30, WS_T = 31, WS_S = 32, WS_PARENT = 33, WS_J0 = 34, WS_J1 = 35, WS_D0 = 36, WS_D1 = 37,
    WS_ACC_A = 38, WS_ACC_BV = 39, WS_ACC_BC = 40, WS_SS0 = 41, WS_SS10 = 42, WS_ISO_FLAG = 43, WS_ISO_POS = 44,
    WS_ISO_KEYS = 45, WS_ISO_KEYS2 = 46, WS_ISO_VALS = 47, WS_ISO_VALS2 = 48, WS_REP = 49, WS_CID = 50,
    WS_BND = 51, WS_TE = 52, WS_CM1 = 53
};

// stats: [0] max_n sum_{e in I(n)} t(e); [1] max |in(n)|; [2] sum of t(e) over
// h-edges with >= 2 pins; [3] their count; [4] noise cap; [5] max depth;
// [6] merged pairs; [7] scratch.
// Per node, from the per-h-edge t(e) and |e| - 1 written by k_edge_tsum.
__global__ __launch_bounds__(256) void k_node_tsum(i32 N, const i64* __restrict__ inc_off,
                                                   const i32* __restrict__ inc_nin, const i32* __restrict__ inc,
                                                   const u64* __restrict__ te, const i32* __restrict__ cm1,
                                                   const i32* __restrict__ nw, unsigned long long* stats) {
    const int lane = lane_id();
    const int wpb = blockDim.x / kWave;
    unsigned long long mx = 0, mn = 0, mw = 0, mb = 0;
    for (i64 n = (i64)blockIdx.x * wpb + wave_id(); n < N; n += (i64)gridDim.x * wpb) {
        u64 s = 0, nb = 0;
        const i64 k0 = inc_off[n], k1 = inc_off[n + 1];
        for (i64 kb = k0; kb < k1; kb += 4 * kWave) {
            i32 ee[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const i64 k = kb + u * kWave + lane;
                ee[u] = k < k1 ? inc[k] : -1;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (ee[u] >= 0) {
                    s += te[ee[u]];
                    nb += (u64)cm1[ee[u]];
                }
            }
        }
        s = wave_sum(s);
        nb = wave_sum(nb);
        mx = mx > s ? mx : s;
        mb = mb > nb ? mb : nb;
        const unsigned long long ni = (unsigned long long)inc_nin[n];
        mn = mn > ni ? mn : ni;
        const unsigned long long wn = (unsigned long long)nw[n];
        mw = mw > wn ? mw : wn;
    }
    if (lane == 0) {
        atomicMax(&stats[0], mx);
        atomicMax(&stats[1], mn);
        atomicMax(&stats[11], mw);
        atomicMax(&stats[12], mb);  // largest neighbour bound sum_{e in I(n)} (|e| - 1)
    }
}

__global__ __launch_bounds__(256) void k_edge_tsum(i32 E, const i64* __restrict__ he_off, const i32* __restrict__ hw,
                                                   unsigned long long* stats, u64* te, i32* cm1) {
    __shared__ unsigned long long red[16];
    unsigned long long s = 0, c = 0, sq = 0, tmax = 0;
    for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += (i64)gridDim.x * blockDim.x) {
        const i64 card = he_off[e + 1] - he_off[e];
        const u64 t = norm_weight(hw[e], card > 0 ? card : 1);
        te[e] = t;
        cm1[e] = (i32)(card - 1);
        if (card >= 2) {
            s += t;
            c += 1;
        }
        sq += (u64)card * (u64)card;
        tmax = tmax > t ? tmax : t;
    }
    s = block_sum(s, red);
    c = block_sum(c, red);
    sq = block_sum(sq, red);
    tmax = wave_max(tmax);
    if (lane_id() == 0) atomicMax(&stats[14], tmax);  // largest normalised weight
    if (threadIdx.x == 0) {
        atomicAdd(&stats[2], s);
        atomicAdd(&stats[3], c);
        atomicAdd(&stats[13], sq);  // sum_e |e|^2: pin visits of the sparse proposal
    }
}

// Noise cap: a tenth of the mean normalised weight of h-edges with >= 2 pins.
// stats[8..10]: the divide-by-(cap + 1) constants used by the noise.
__global__ void k_noise_cap(unsigned long long* stats) {
    const u64 cap = stats[3] ? stats[2] / (10ull * stats[3]) : 0ull;
    stats[4] = cap;
    const DivU64 f = divu64_make(cap + 1);
    stats[8] = f.m;
    stats[9] = ((u64)f.sh2 << 32) | f.sh1;
    stats[10] = f.d;
}

__device__ __forceinline__ DivU64 noise_div(const unsigned long long* stats) {
    DivU64 f;
    f.m = stats[8];
    f.sh1 = (u32)stats[9];
    f.sh2 = (u32)(stats[9] >> 32);
    f.d = stats[10];
    return f;
}

// Candidate proposal (Sec. V-C): one block per node.  The block sweeps n's
// incident h-edges and their pins and accumulates, per neighbour m, the packed
// value (eta(n,m) << ib) + inter(n,m) in a shared-memory histogram indexed by
// m.  Neighbour ids are split into ranges of R that fit the histogram; every
// range is one pass over the pins.  The pins of one h-edge are distinct, and
// h-edges run on different waves, so updates are shared-memory atomics.  After
// each pass the block scans the bins and keeps the best PI valid neighbours
// (Eq. proposal_graph: sizes, and |in(n) ∪ in(m)| through inter) by (score
// desc, id desc), score = eta + symmetric noise (top_select.h).
//
// Pin sweep: each wave owns a batch of up to 64 incident h-edges (one per
// lane).  Their pin segments for the current pass (all sources, plus the
// destinations whose ids fall in the pass's range) are concatenated into one
// index space through a per-wave offset table in shared memory, and every lane
// walks that space with stride 64, kProposeU loads in flight at a time, so a
// wave keeps many loads outstanding whatever the h-edge sizes.
constexpr int kProposeU = 8;
constexpr int kProposeWaves = 4;       // waves per block with a 64 KiB histogram
constexpr int kProposeWavesBig = 8;    // waves per block with a 128 KiB histogram (one block per CU)
constexpr int kScanVec = 2;  // 16-byte vectors of bins per thread per step of the bin scan
// Batches whose segments average at least kLongSegment pins are instead swept
// by propose_group, several h-edges at a time.
constexpr int kLongSegment = 32;

template <typename BIN, int WAVES>
struct SegTable {
    i32 start[WAVES][kWave];    // first flat index of the lane's segment
    i32 src_end[WAVES][kWave];  // flat index where its destinations begin
    i64 sbase[WAVES][kWave];    // pin position = base + flat index
    i64 dbase[WAVES][kWave];
    BIN add[WAVES][kWave];      // per source pin
    BIN add_in[WAVES][kWave];   // per destination pin
};

// The sweep's offset tables and the scan's queues are never live together.
template <typename BIN, int WAVES>
union ProposeShared {
    SegTable<BIN, WAVES> tab;
    SelQueue<BIN> q[WAVES];
};

// Histogram allocation in bins: R rounded up to whole scan vectors of a block.
__host__ __device__ inline int propose_bins_alloc(int R) { return (R + 255) / 256 * 256; }

template <typename BIN>
__device__ __forceinline__ BIN vec_bin(const uint4& w, int i);
template <>
__device__ __forceinline__ u32 vec_bin<u32>(const uint4& w, int i) {
    return i == 0 ? w.x : i == 1 ? w.y : i == 2 ? w.z : w.w;
}
template <>
__device__ __forceinline__ unsigned long long vec_bin<unsigned long long>(const uint4& w, int i) {
    return i == 0 ? ((unsigned long long)w.y << 32 | w.x) : ((unsigned long long)w.w << 32 | w.z);
}

// Grouped pin sweep of one wave batch (lane l holds h-edge l's metadata):
// h-edges G at a time; each h-edge's sources and this pass's destinations form
// one index space [0, cs + cd) (destination q at offset q + dsh from the
// h-edge start), read GU * 64 entries per h-edge and chunk, so G * GU loads per
// lane are in flight.  Destinations lie in the pass's id range (pass bounds);
// sources are tested.  The sweep is software pipelined: the loads of the next
// chunk are issued before the updates of the current one, in two register sets
// used alternately.
template <int G, int GU, typename BIN>
struct GroupChunk {
    i32 m[G][GU];    // pin id, n when the entry is past the h-edge's segment
    BIN ad[G][GU];   // histogram increment of the entry
    u32 src;         // bit g * GU + u: the entry is a source
};

// Issues the loads of chunk (i0, q0); returns the group's longest segment.
template <int G, int GU, typename BIN, typename PIN>
__device__ __forceinline__ i32 group_load(int i0, i32 q0, int nb, int lane, i32 n, const PIN* __restrict__ pins,
                                          i64 e0, i32 cs, i32 cd, i32 dsh, BIN add, BIN add_in,
                                          GroupChunk<G, GU, BIN>& c) {
    i32 maxt = 0;
    u32 srcm = 0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int sl = min(i0 + g, kWave - 1);
        const PIN* rp = pins + bcast(e0, sl);  // wave-uniform row base
        const i32 ns = bcast(cs, sl);
        const i32 nt = i0 + g < nb ? ns + bcast(cd, sl) : 0;
        const i32 sh = bcast(dsh, sl);
        const BIN sa = bcast(add, sl), sai = bcast(add_in, sl);
        maxt = max(maxt, nt);
#pragma unroll
        for (int u = 0; u < GU; ++u) {
            const i32 q = q0 + u * kWave + lane;
            const int is_src = (int)(q < ns);
            c.m[g][u] = q < nt ? (i32)rp[q + (is_src ? 0 : sh)] : n;
            c.ad[g][u] = is_src ? sa : sai;
            srcm |= (u32)is_src << (g * GU + u);
        }
    }
    c.src = srcm;
    return maxt;
}

template <int G, int GU, typename BIN>
__device__ __forceinline__ void group_apply(const GroupChunk<G, GU, BIN>& c, i32 n, i32 lo, i32 hi, BIN* bins) {
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int u = 0; u < GU; ++u) {
            const i32 m = c.m[g][u];
            const int is_src = (int)((c.src >> (g * GU + u)) & 1u);
            const int ok = (int)(m != n) & (!is_src | (int)((u32)(m - lo) < (u32)(hi - lo)));
            if (ok) atomicAdd(&bins[m - lo], c.ad[g][u]);
        }
}

template <int G, int GU, typename BIN, typename PIN>
__device__ __forceinline__ void propose_group(int nb, int lane, i32 n, i32 lo, i32 hi, const PIN* __restrict__ pins,
                                              i64 e0, i32 cs, i32 cd, i32 dsh, BIN add, BIN add_in, BIN* bins) {
    if (nb <= 0) return;
    GroupChunk<G, GU, BIN> c0, c1;
    int i0 = 0;
    i32 q0 = 0;
    // chunk order: GU * 64 entries of the group at a time, then the next group
    auto next = [&](i32 mt) {
        q0 += GU * kWave;
        if (q0 >= mt) {
            i0 += G;
            q0 = 0;
        }
    };
    i32 mt = group_load<G, GU>(i0, q0, nb, lane, n, pins, e0, cs, cd, dsh, add, add_in, c0);
    while (true) {
        next(mt);
        if (i0 < nb) mt = group_load<G, GU>(i0, q0, nb, lane, n, pins, e0, cs, cd, dsh, add, add_in, c1);
        group_apply(c0, n, lo, hi, bins);
        if (i0 >= nb) break;
        next(mt);
        if (i0 < nb) mt = group_load<G, GU>(i0, q0, nb, lane, n, pins, e0, cs, cd, dsh, add, add_in, c0);
        group_apply(c1, n, lo, hi, bins);
        if (i0 >= nb) break;
    }
}

template <typename BIN, int PI, typename PIN, int WAVES>
__global__ __launch_bounds__(WAVES * kWave) void k_propose(
    i32 N, const i64* __restrict__ inc_off, const i32* __restrict__ inc_nin, const i32* __restrict__ inc,
    const i64* __restrict__ he_off, const i32* __restrict__ he_nsrc, const PIN* __restrict__ pins,
    const i32* __restrict__ hw, const i32* __restrict__ nw, i64 omega, i64 delta, u64 seed,
    const unsigned long long* __restrict__ stats, int ib, i32* cand, u64* score, int R,
    const i32* __restrict__ bnd) {
    constexpr int kBinsPerVec = 16 / (int)sizeof(BIN);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    BIN* bins = (BIN*)smem_raw;  // R bins: one pass covers R consecutive neighbour ids
    uint4* bins4 = (uint4*)smem_raw;
    __shared__ u64 red_s[16];
    __shared__ i32 red_m[16];
    __shared__ ProposeShared<BIN, WAVES> sh;
    __shared__ unsigned long long s_floor;
    SelNode sn;
    sn.seed = seed;
    sn.cap = stats[4];
    sn.ndiv = noise_div(stats);
    sn.ib = ib;
    sn.omega = omega;
    sn.delta = delta;
    sn.nw = nw;
    sn.inc_nin = inc_nin;
    sn.floor = &s_floor;
    sn.union_floor = 1;
    const int npass = (int)((N + R - 1) / R);
    const int lane = lane_id(), wv = wave_id(), nwv = blockDim.x / kWave;
    const int nalloc4 = propose_bins_alloc(R) / kBinsPerVec;
    for (int i = threadIdx.x; i < nalloc4; i += blockDim.x) bins4[i] = make_uint4(0u, 0u, 0u, 0u);
    __syncthreads();
    for (i64 r = 0;; ++r) {
        const i64 nx = xcd_item(r, blockIdx.x, gridDim.x);  // neighbouring nodes on one XCD
        if (nx >= N) break;
        const i32 n = (i32)nx;
        TopList<PI> top;
        top.clear();
        const i64 a = inc_off[n], b = inc_off[n + 1];
        const i32 nin_n = inc_nin[n];
        const i64 nw_n = nw[n];
        sn.n = n;
        sn.nin_n = nin_n;
        sn.nw_n = nw_n;
        if (threadIdx.x == 0) s_floor = 0;  // read after the sweep's barrier
        // When even the heaviest and most-connected node fits with n, every
        // pair (n, m) is valid and the scan needs no per-neighbour loads.
        sn.all_valid = (int)(nw_n + (i64)stats[11] <= omega) & (int)((i64)nin_n + (i64)stats[1] <= delta);
        // h-edges per wave batch: spread the node's h-edges evenly over the waves.
        const i64 deg = b - a;
        const i64 chunk = deg <= (i64)nwv * kWave ? (deg + nwv - 1) / nwv : (i64)kWave;
        const bool one_batch = deg <= (i64)nwv * kWave;
        i32 e = 0;
        i64 e0 = 0, e1v = 0, d0v = 0;
        BIN add = 0, add_in = 0;
        int valid = 0;
        for (int pass = 0; pass < npass && a < b; ++pass) {
            const i32 lo = pass * R;
            const i32 hi = min(N, lo + R);
            for (i64 kb = a + (i64)wv * chunk; kb < b; kb += (i64)nwv * chunk) {
                if ((pass == 0) | !one_batch) {
                    const i64 k = kb + lane;
                    valid = (int)(lane < chunk) & (int)(k < b);
                    e = inc[valid ? k : kb];
                    e0 = he_off[e];
                    e1v = he_off[e + 1];
                    d0v = e0 + he_nsrc[e];
                    add = ((BIN)norm_weight(hw[e], e1v - e0)) << ib;
                    add_in = add + (((k - a) < nin_n) ? (BIN)1 : (BIN)0);  // destinations of e lie in in(n)
                }
                i64 dlo = d0v, dhi = e1v;
                if (npass > 1) {
                    dlo = e0 + bnd[(i64)e * (npass + 1) + pass];
                    dhi = e0 + bnd[(i64)e * (npass + 1) + pass + 1];
                }
                const i32 cs = valid ? (i32)(d0v - e0) : 0;
                const i32 cd = valid ? (i32)(dhi - dlo) : 0;
                const i32 incl = wave_incl_scan(cs + cd);
                const i32 excl = incl - cs - cd;
                const i32 T = __shfl(incl, kWave - 1, kWave);
                const int nb = __popcll(__ballot(valid));
                if (T >= kLongSegment * nb) {
                    // Long segments: h-edges G at a time, GU coalesced loads per
                    // h-edge and lane; more h-edges at once when they are short.
                    const i32 avg = T / max(nb, 1);
                    const i32 dsh = (i32)(dlo - e0) - cs;  // destination offset past the sources
                    if (avg <= 64)
                        propose_group<16, 1>(nb, lane, n, lo, hi, pins, e0, cs, cd, dsh, add, add_in, bins);
                    else if (avg <= 128)
                        propose_group<8, 2>(nb, lane, n, lo, hi, pins, e0, cs, cd, dsh, add, add_in, bins);
                    else
                        propose_group<4, 4>(nb, lane, n, lo, hi, pins, e0, cs, cd, dsh, add, add_in, bins);
                    continue;
                }
                sh.tab.start[wv][lane] = excl;
                sh.tab.src_end[wv][lane] = excl + cs;
                sh.tab.sbase[wv][lane] = e0 - excl;
                sh.tab.dbase[wv][lane] = dlo - cs - excl;
                sh.tab.add[wv][lane] = add;
                sh.tab.add_in[wv][lane] = add_in;
                wave_sync();
                int cur = 0;
                for (i32 j0 = 0; j0 < T; j0 += kProposeU * kWave) {
                    i32 mm[kProposeU];
                    BIN ad[kProposeU];
#pragma unroll
                    for (int u = 0; u < kProposeU; ++u) {
                        const i32 j = j0 + u * kWave + lane;
                        const int in = (int)(j < T);
                        while ((int)(cur + 1 < kWave) & in) {
                            if (sh.tab.start[wv][cur + 1] > j) break;
                            ++cur;
                        }
                        const int is_src = (int)(j < sh.tab.src_end[wv][cur]);
                        const i64 pos = in ? (is_src ? sh.tab.sbase[wv][cur] : sh.tab.dbase[wv][cur]) + j : 0;
                        ad[u] = is_src ? sh.tab.add[wv][cur] : sh.tab.add_in[wv][cur];
                        mm[u] = in ? (i32)pins[pos] : n;
                    }
#pragma unroll
                    for (int u = 0; u < kProposeU; ++u) {
                        const i32 m = mm[u];
                        if ((int)(m != n) & (int)(m >= lo) & (int)(m < hi)) atomicAdd(&bins[m - lo], ad[u]);
                    }
                }
                wave_sync();  // the table is rewritten by the next batch
            }
            __syncthreads();
            // Bin scan: every thread reads kScanVec 16-byte vectors of bins per
            // step and clears them; bins that can still reach the top PI are
            // queued and scored 64 at a time (top_select.h).
            const int nvec = (hi - lo + kBinsPerVec - 1) / kBinsPerVec;
            u32 qh = 0, qn = 0;
            for (int v0 = 0; v0 < nvec; v0 += kScanVec * (int)blockDim.x) {
                uint4 w[kScanVec];
#pragma unroll
                for (int j = 0; j < kScanVec; ++j) {
                    const int vi = v0 + j * (int)blockDim.x + (int)threadIdx.x;
                    w[j] = vi < nvec ? bins4[vi] : make_uint4(0u, 0u, 0u, 0u);
                    if (vi < nvec) bins4[vi] = make_uint4(0u, 0u, 0u, 0u);
                }
                const BIN vmin = sel_vmin<BIN, PI>(top, sn);
#pragma unroll
                for (int j = 0; j < kScanVec; ++j) {
                    const i32 mb = lo + (v0 + j * (int)blockDim.x + (int)threadIdx.x) * kBinsPerVec;
#pragma unroll
                    for (int i = 0; i < kBinsPerVec; ++i) {
                        const BIN v = vec_bin<BIN>(w[j], i);
                        sel_push(sh.q[wv], qh, qn, (int)(v >= vmin), mb + i, v, top, sn);
                    }
                }
            }
            sel_flush(sh.q[wv], qh, qn, top, sn);
            __syncthreads();
        }
        sel_merge(top, red_s, red_m, cand + (i64)n * PI, score + (i64)n * PI);
    }
}

// Sparse variant of the proposal for levels with many nodes and modest
// neighbourhoods: the histogram is an open-addressing table of C slots in
// shared memory (key, packed (eta << ib) | inter, and a list of used slots).
// Neighbours may be split into B passes by a hash of their id.  A node starts
// with the pass count its block's previous node needed; a pass that meets more
// than `cap` distinct keys is abandoned at once and the node restarts with
// twice as many passes.  The result is the same exact top-PI as the dense
// variant whatever B is.
//
// Pin sweep: h-edges G at a time, GU coalesced loads per h-edge and lane,
// software pipelined, as in the id-range variant (propose_group).
constexpr u32 kEmpty = 0xFFFFFFFFu;
constexpr u32 kNoSlot = 0xFFFFFFFFu;  // a ticket whose slot claim lost its race

__device__ __forceinline__ u32 slot_hash(u32 m) { return m * 0x9E3779B1u; }
__device__ __forceinline__ u32 pass_hash(u32 m) { return (m * 0x85EBCA77u) ^ (m >> 15); }

template <typename BIN>
struct HashTab {
    u32* keys;
    BIN* vals;
    u32* touched;   // ticket -> slot (kNoSlot when the claim lost)
    u32* nticket;   // tickets taken this pass
    int* overflow;  // set once a ticket reaches cap
    u32 cmask, cap;
};

// Adds v to key m's slot.  A new key first takes a ticket; tickets at or beyond
// cap abandon the pass, so fewer than cap slots are ever claimed and the probe
// always meets an empty slot or the key.
template <typename BIN>
__device__ __forceinline__ void hash_add(const HashTab<BIN>& T, u32 m, BIN v) {
    u32 sl = slot_hash(m) & T.cmask;
    for (;;) {
        const u32 kk = T.keys[sl];
        if (kk == m) {
            atomicAdd(&T.vals[sl], v);
            return;
        }
        if (kk == kEmpty) {
            const u32 t = atomicAdd(T.nticket, 1u);
            if (t >= T.cap) {
                *T.overflow = 1;
                return;
            }
            const u32 prev = atomicCAS(&T.keys[sl], kEmpty, m);
            T.touched[t] = prev == kEmpty ? sl : kNoSlot;
            if ((int)(prev == kEmpty) | (int)(prev == m)) {
                atomicAdd(&T.vals[sl], v);
                return;
            }
        }
        sl = (sl + 1) & T.cmask;
    }
}

// Entries that miss their home slot wait in a per-wave ring in shared memory
// and are inserted 64 at a time, one per lane, so the probing loop runs on
// full waves instead of once per entry with a few lanes.
template <typename BIN>
struct MissQueue {
    SelQueue<BIN>* q;  // the wave's ring (the selection's queue, idle during the sweep)
    u32 head, count;
};

template <typename BIN>
__device__ __forceinline__ void miss_drain(MissQueue<BIN>& Q, u32 cnt, const HashTab<BIN>& T) {
    wave_sync();  // the ring's writes are visible to every lane
    const int lane = lane_id();
    const int on = (int)((u32)lane < cnt);
    const u32 at = (Q.head + (u32)lane) & (u32)(kSelQ - 1);
    const i32 m = on ? Q.q->m[at] : 0;
    const BIN v = on ? Q.q->v[at] : (BIN)0;
    wave_sync();  // the slots may be refilled from here on
    Q.head += cnt;
    Q.count -= cnt;
    if (on) hash_add(T, (u32)m, v);
}

template <typename BIN>
__device__ __forceinline__ void miss_push(MissQueue<BIN>& Q, int miss, i32 m, BIN v, const HashTab<BIN>& T) {
    const u64 mask = __ballot(miss);
    if (mask == 0) return;
    if (miss) {
        const u32 below = __builtin_amdgcn_mbcnt_hi((u32)(mask >> 32), __builtin_amdgcn_mbcnt_lo((u32)mask, 0u));
        const u32 at = (Q.head + Q.count + below) & (u32)(kSelQ - 1);
        Q.q->m[at] = m;
        Q.q->v[at] = v;
    }
    Q.count += (u32)__popcll(mask);
    if (Q.count >= (u32)kWave) miss_drain(Q, (u32)kWave, T);
}

// The chunk's home slots are read together first; entries whose key already
// sits in its home slot (most of them once a node's neighbours are in the
// table) add without waiting, the rest go to the wave's miss ring.
template <int G, int GU, typename BIN>
__device__ __forceinline__ void group_apply_hash(const GroupChunk<G, GU, BIN>& c, i32 n, u32 bmask, u32 pass,
                                                 const HashTab<BIN>& T, MissQueue<BIN>& Q) {
    u32 home[G][GU], seen[G][GU];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int u = 0; u < GU; ++u) {
            const u32 m = (u32)c.m[g][u];
            home[g][u] = slot_hash(m) & T.cmask;
            seen[g][u] = T.keys[home[g][u]];
        }
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int u = 0; u < GU; ++u) {
            const i32 m = c.m[g][u];
            const int mine = (int)(m != n) & (int)((pass_hash((u32)m) & bmask) == pass);
            const int hit = mine & (int)(seen[g][u] == (u32)m);
            if (hit) atomicAdd(&T.vals[home[g][u]], c.ad[g][u]);
            miss_push(Q, mine & !hit, m, c.ad[g][u], T);
        }
}

// One wave batch: the grouped, pipelined sweep of propose_group with hashed
// updates; stops early once the pass has overflowed.
template <int G, int GU, typename BIN>
__device__ __forceinline__ void hash_group(int nb, int lane, i32 n, u32 bmask, u32 pass, const i32* __restrict__ pins,
                                           i64 e0, i32 cs, i32 cd, BIN add, BIN add_in, const HashTab<BIN>& T,
                                           MissQueue<BIN>& Q) {
    if (nb <= 0) return;
    GroupChunk<G, GU, BIN> c0, c1;
    int i0 = 0;
    i32 q0 = 0;
    auto next = [&](i32 mt) {
        q0 += GU * kWave;
        if (q0 >= mt) {
            i0 += G;
            q0 = 0;
        }
    };
    const volatile int* ovf = T.overflow;
    i32 mt = group_load<G, GU>(i0, q0, nb, lane, n, pins, e0, cs, cd, 0, add, add_in, c0);
    while (true) {
        next(mt);
        if (i0 < nb) mt = group_load<G, GU>(i0, q0, nb, lane, n, pins, e0, cs, cd, 0, add, add_in, c1);
        group_apply_hash(c0, n, bmask, pass, T, Q);
        if ((int)(i0 >= nb) | *ovf) break;
        next(mt);
        if (i0 < nb) mt = group_load<G, GU>(i0, q0, nb, lane, n, pins, e0, cs, cd, 0, add, add_in, c0);
        group_apply_hash(c1, n, bmask, pass, T, Q);
        if ((int)(i0 >= nb) | *ovf) break;
    }
}

// Short segments (averaging under kLongSegment pins, as at the coarser levels
// of the convolutional graph: ~200 h-edges of ~5 pins per node): the wave's
// batch is one flat index space [0, tot), lane l's h-edge at [start_l, start_l
// + len_l) with its sources first and its pins contiguous from e0_l, swept
// 64 * kHashFlatU entries at a time with every lane busy.  An entry's h-edge
// is found by a binary search over the lanes' starts with whole-wave
// shuffles; the updates are those of group_apply_hash.
constexpr int kHashFlatU = 4;

template <typename BIN>
__device__ __forceinline__ void hash_flat(int lane, i32 n, u32 bmask, u32 pass, const i32* __restrict__ pins, i64 e0,
                                          i32 cs, i32 len, BIN add, BIN add_in, const HashTab<BIN>& T,
                                          MissQueue<BIN>& Q) {
    const i32 incl = wave_incl_scan(len);
    const i32 start = incl - len;
    const i32 tot = __shfl(incl, kWave - 1, kWave);
    const volatile int* ovf = T.overflow;
    for (i32 j0 = 0; j0 < tot; j0 += kHashFlatU * kWave) {
        i32 mm[kHashFlatU];
        BIN ad[kHashFlatU];
        u32 live = 0;
#pragma unroll
        for (int u = 0; u < kHashFlatU; ++u) {
            const i32 j = j0 + u * kWave + lane;
            int o = 0;  // the last lane whose segment starts at or before j
#pragma unroll
            for (int step = kWave / 2; step >= 1; step >>= 1) {
                const int cand = o + step;
                const i32 sc = __shfl(start, cand, kWave);
                o = sc <= j ? cand : o;
            }
            const i32 st = __shfl(start, o, kWave), ns = __shfl(cs, o, kWave);
            const i64 base = __shfl(e0, o, kWave);
            const BIN a1 = __shfl(add, o, kWave), a2 = __shfl(add_in, o, kWave);
            const int in = (int)(j < tot);
            live |= (u32)in << u;
            mm[u] = pins[in ? base + (j - st) : 0];  // past the end: the first pin slot, dropped below
            ad[u] = j - st < ns ? a1 : a2;
        }
        u32 home[kHashFlatU], seen[kHashFlatU];
#pragma unroll
        for (int u = 0; u < kHashFlatU; ++u) {
            const u32 m = ((live >> u) & 1u) ? (u32)mm[u] : (u32)n;
            home[u] = slot_hash(m) & T.cmask;
            seen[u] = T.keys[home[u]];
        }
#pragma unroll
        for (int u = 0; u < kHashFlatU; ++u) {
            const i32 m = ((live >> u) & 1u) ? mm[u] : n;
            const int mine = (int)(m != n) & (int)((pass_hash((u32)m) & bmask) == pass);
            const int hit = mine & (int)(seen[u] == (u32)m);
            if (hit) atomicAdd(&T.vals[home[u]], ad[u]);
            miss_push(Q, mine & !hit, m, ad[u], T);
        }
        if (*ovf) break;
    }
}

template <typename BIN, int PI>
__device__ __forceinline__ void propose_hash_body(
    i32 N, const i64* __restrict__ inc_off, const i32* __restrict__ inc_nin, const i32* __restrict__ inc,
    const i64* __restrict__ he_off, const i32* __restrict__ he_nsrc, const i32* __restrict__ pins,
    const i32* __restrict__ hw, const i32* __restrict__ nw, i64 omega, i64 delta, u64 seed,
    const unsigned long long* __restrict__ stats, int ib, i32* cand, u64* score, int C) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    BIN* vals = (BIN*)smem_raw;
    u32* keys = (u32*)(vals + C);
    u32* touched = keys + C;
    __shared__ u32 nticket;
    __shared__ int overflow;
    __shared__ u64 red_s[16];
    __shared__ i32 red_m[16];
    __shared__ SelQueue<BIN> selq[4];
    __shared__ unsigned long long s_floor;
    SelNode sn;
    sn.seed = seed;
    sn.cap = stats[4];
    sn.ndiv = noise_div(stats);
    sn.ib = ib;
    sn.omega = omega;
    sn.delta = delta;
    sn.nw = nw;
    sn.inc_nin = inc_nin;
    sn.floor = &s_floor;
    sn.union_floor = 1;
    HashTab<BIN> T;
    T.keys = keys;
    T.vals = vals;
    T.touched = touched;
    T.nticket = &nticket;
    T.overflow = &overflow;
    T.cmask = (u32)C - 1;
    T.cap = (u32)C - (u32)C / 4;  // load factor at most 3/4
    const int lane = lane_id(), wv = wave_id(), nwv = blockDim.x / kWave;
    for (int i = threadIdx.x; i < C; i += blockDim.x) {
        vals[i] = 0;
        keys[i] = kEmpty;
    }
    if (threadIdx.x == 0) {
        nticket = 0;
        overflow = 0;
    }
    __syncthreads();
    u64 Bhint = 1;  // passes the block's previous node needed
    for (i64 r = 0;; ++r) {
        const i64 nx = xcd_item(r, blockIdx.x, gridDim.x);  // neighbouring nodes on one XCD
        if (nx >= N) break;
        const i32 n = (i32)nx;
        const i64 a = inc_off[n], b = inc_off[n + 1];
        const i32 nin_n = inc_nin[n];
        const i64 nw_n = nw[n];
        // Passes split the neighbours by a hash of their id; any split gives the
        // same result, so the count is a power of two (a mask, not a division).
        u64 B = Bhint;
        sn.n = n;
        sn.nin_n = nin_n;
        sn.nw_n = nw_n;
        sn.all_valid = (int)(nw_n + (i64)stats[11] <= omega) & (int)((i64)nin_n + (i64)stats[1] <= delta);
        // h-edges per wave batch: spread the node's h-edges evenly over the waves.
        const i64 deg = b - a;
        const bool one_batch = deg <= (i64)nwv * kWave;
        const i64 chunk = one_batch ? (deg + nwv - 1) / nwv : (i64)kWave;
        TopList<PI> top;
        u32 most = 0;  // most keys any pass of the node held
        for (;;) {     // restarts with more passes if a pass overflows the table
            top.clear();
            most = 0;
            if (threadIdx.x == 0) s_floor = 0;  // read after the first pass's barrier
            bool again = false;
            for (u64 pass = 0; pass < B && a < b; ++pass) {
                MissQueue<BIN> Q{&selq[wv], 0u, 0u};
                for (i64 kb = a + (i64)wv * chunk; kb < b; kb += (i64)nwv * chunk) {
                    const i64 k = kb + lane;
                    const int valid = (int)(lane < chunk) & (int)(k < b);
                    const i32 e = inc[valid ? k : kb];
                    const i64 e0 = he_off[e], e1 = he_off[e + 1];
                    const i32 ns = he_nsrc[e];
                    const BIN add = ((BIN)norm_weight(hw[e], e1 - e0)) << ib;
                    const BIN add_in = add + (((k - a) < nin_n) ? (BIN)1 : (BIN)0);  // dsts of e lie in in(n)
                    const i32 cs = valid ? ns : 0;
                    const i32 cd = valid ? (i32)(e1 - e0) - ns : 0;
                    const i32 tot = wave_sum(cs + cd);
                    const int nb = __popcll(__ballot(valid));
                    const i32 avg = tot / max(nb, 1);
                    const u32 bm = (u32)(B - 1), ps = (u32)pass;
                    if (tot < kLongSegment * nb)
                        hash_flat(lane, n, bm, ps, pins, e0, cs, cs + cd, add, add_in, T, Q);
                    else if (avg <= 64)
                        hash_group<8, 1>(nb, lane, n, bm, ps, pins, e0, cs, cd, add, add_in, T, Q);
                    else if (avg <= 128)
                        hash_group<4, 2>(nb, lane, n, bm, ps, pins, e0, cs, cd, add, add_in, T, Q);
                    else
                        hash_group<2, 4>(nb, lane, n, bm, ps, pins, e0, cs, cd, add, add_in, T, Q);
                }
                if (Q.count > 0) miss_drain(Q, Q.count, T);  // the rest of the wave's misses
                __syncthreads();
                const u32 nt = min(nticket, T.cap);
                const int ov = overflow;
                most = max(most, nt);
                u32 qh = 0, qn = 0;
                for (u32 t0 = 0; t0 < nt; t0 += blockDim.x) {
                    const u32 t = t0 + threadIdx.x;
                    const u32 sl = t < nt ? touched[t] : kNoSlot;
                    const int in = (int)(sl != kNoSlot);
                    const i32 m = in ? (i32)keys[sl] : 0;
                    const BIN v = in ? vals[sl] : (BIN)0;
                    if (in) {
                        keys[sl] = kEmpty;
                        vals[sl] = 0;
                    }
                    const BIN vmin = sel_vmin<BIN, PI>(top, sn);
                    sel_push(selq[wv], qh, qn, in & !ov & (int)(v >= vmin), m, v, top, sn);
                }
                sel_flush(selq[wv], qh, qn, top, sn);
                __syncthreads();
                if (threadIdx.x == 0) {
                    nticket = 0;
                    overflow = 0;
                }
                __syncthreads();
                if (ov) {
                    again = true;
                    break;
                }
            }
            if (!again) break;
            B *= 2;
        }
        // the next node starts from this node's pass count, one fewer halving
        // step when the table stayed at most a quarter full
        Bhint = (most <= (u32)C / 4 && B > 1) ? B / 2 : B;
        sel_merge(top, red_s, red_m, cand + (i64)n * PI, score + (i64)n * PI);
    }
}

// The kernel for 32-bit bins asks for five waves per SIMD (at most 102 VGPRs;
// the register allocator spills a handful of cold values to scratch): a fifth
// more waves to hide the pin loads' latency measured 857 -> 809 ms per
// partitioning of the 6.9 M-node convolutional graph.  With 64-bit bins the
// same request spilled 30-99 registers, so that kernel keeps the compiler's
// choice.
template <typename BIN, int PI>
__global__ __launch_bounds__(256) void k_propose_hash(
    i32 N, const i64* __restrict__ inc_off, const i32* __restrict__ inc_nin, const i32* __restrict__ inc,
    const i64* __restrict__ he_off, const i32* __restrict__ he_nsrc, const i32* __restrict__ pins,
    const i32* __restrict__ hw, const i32* __restrict__ nw, i64 omega, i64 delta, u64 seed,
    const unsigned long long* __restrict__ stats, int ib, i32* cand, u64* score, int C) {
    propose_hash_body<BIN, PI>(N, inc_off, inc_nin, inc, he_off, he_nsrc, pins, hw, nw, omega, delta, seed, stats,
                               ib, cand, score, C);
}

template <int PI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_propose_hash32(
    i32 N, const i64* __restrict__ inc_off, const i32* __restrict__ inc_nin, const i32* __restrict__ inc,
    const i64* __restrict__ he_off, const i32* __restrict__ he_nsrc, const i32* __restrict__ pins,
    const i32* __restrict__ hw, const i32* __restrict__ nw, i64 omega, i64 delta, u64 seed,
    const unsigned long long* __restrict__ stats, int ib, i32* cand, u64* score, int C) {
    propose_hash_body<u32, PI>(N, inc_off, inc_nin, inc, he_off, he_nsrc, pins, hw, nw, omega, delta, seed, stats,
                               ib, cand, score, C);
}

// For each h-edge: offsets (from the h-edge start) where the destination
// block crosses the pass boundaries 0, R, 2R, ..., npass*R; the destination
// block is sorted, so each is a lower bound.
__global__ void k_pass_bounds(i32 E, const i64* __restrict__ he_off, const i32* __restrict__ he_nsrc,
                              const i32* __restrict__ pins, int R, int npass, i32* bnd) {
    for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += (i64)gridDim.x * blockDim.x) {
        const i64 e0 = he_off[e], e1 = he_off[e + 1], d0 = e0 + he_nsrc[e];
        i64 lo = d0;
        for (int p = 0; p <= npass; ++p) {
            const i64 key = (i64)p * R;
            i64 l = lo, h = e1;
            while (l < h) {
                const i64 mid = (l + h) >> 1;
                const i32 v = pins[mid];
                const int lt = (int)((i64)v < key);
                l = lt ? mid + 1 : l;
                h = lt ? h : mid;
            }
            bnd[e * (npass + 1) + p] = (i32)(l - e0);
            lo = l;
        }
    }
}

// ---- matching rounds (Sec. V-D) -------------------------------------------
// Round r's target: the r-th candidate if both ends are still unmatched
// (t = -2 marks nodes matched in an earlier round, -1 an undefined target).
__device__ __forceinline__ void round_targets_elem(i64 n, int Pi, int r, const i32* __restrict__ cand,
                                                   const u64* __restrict__ score, const i32* __restrict__ match,
                                                   i32* t, u64* s) {
    if (match[n] >= 0) {
        t[n] = -2;
        return;
    }
    const i32 c = cand[n * Pi + r];
    const i32 mc = match[c >= 0 ? c : 0];  // in bounds either way; used only when c >= 0
    t[n] = ((int)(c >= 0) & (int)(mc < 0)) ? c : -1;
    s[n] = score[n * Pi + r];
}

// Parent in the pseudo-forest: the target, except inside a two-cycle (the set
// R of the paper) and for undefined targets, whose nodes are tree roots.
__device__ __forceinline__ void round_parent_elem(i64 n, const i32* __restrict__ t, i32* parent, i32* jump,
                                                  i32* depth, i64* accA, u64* accBV, i32* accBC) {
    accA[n] = 0;
    accBV[n] = 0;
    accBC[n] = -1;
    const i32 tn = t[n];
    if (tn == -2) {
        parent[n] = -2;
        jump[n] = -1;
        depth[n] = -1;
        return;
    }
    const i32 tp = t[tn >= 0 ? tn : 0];
    const i32 p = ((int)(tn >= 0) & (int)(tp == (i32)n)) ? -1 : tn;
    parent[n] = p;
    jump[n] = p;
    depth[n] = p >= 0 ? 1 : 0;
}

// Pointer jumping towards the roots: depth = number of hops to the root.
// Returns 1 while n's pointer has not reached a root.
__device__ __forceinline__ int jump_elem(i64 n, const i32* __restrict__ jin, const i32* __restrict__ din,
                                         i32* jout, i32* dout) {
    const i32 j = jin[n];
    const i32 jj = j >= 0 ? j : (i32)n;
    const i32 dj = din[jj], nj = jin[jj];
    const i32 dn = din[n];
    dout[n] = j >= 0 ? dn + dj : dn;
    const i32 nxt = j >= 0 ? nj : j;
    jout[n] = nxt;
    return nxt >= 0 ? 1 : 0;
}

// Bottom-up at depth d: ss0 from the children's sums (Eq. ss0), the return of
// matching with the parent ss1 - ss0, and the push of both to the parent.
__device__ __forceinline__ void up_a_elem(i64 n, int d, const i32* __restrict__ depth,
                                          const i32* __restrict__ parent, const u64* __restrict__ s, i64* accA,
                                          u64* accBV, const i32* __restrict__ accBC, i64* ss0, i64* ss10) {
    if (depth[n] != d) return;
    const i32 bc = load_l2(&accBC[n]);
    const i64 bvr = dec_i64(load_l2(&accBV[n]));
    const i64 take = ((int)(bc >= 0) & (int)(bvr > 0)) ? bvr : 0;
    const i64 v0 = load_l2(&accA[n]) + take;
    ss0[n] = v0;
    const i32 p = parent[n];
    if (p >= 0) {
        const i64 x = (i64)s[n] - take;
        ss10[n] = x;
        atomicAdd((unsigned long long*)&accA[p], (unsigned long long)v0);
        atomicMax((unsigned long long*)&accBV[p], (unsigned long long)enc_i64(x));
    }
}

// Second half of the lexicographic (ss1 - ss0, id) maximum over children.
__device__ __forceinline__ void up_b_elem(i64 n, int d, const i32* __restrict__ depth,
                                          const i32* __restrict__ parent, const i64* __restrict__ ss10,
                                          const u64* __restrict__ accBV, i32* accBC) {
    if (depth[n] != d) return;
    const i32 p = parent[n];
    const u64 bvp = load_l2(&accBV[p >= 0 ? p : 0]);
    if ((int)(p >= 0) & (int)(enc_i64(ss10[n]) == bvp)) atomicMax(&accBC[p], (i32)n);
}

// Two-cycle roots (Eq. ss1_roots, Eq. match_root): the pair matches iff
// ss1 > ss0(n) + ss0(target(n)).
__device__ __forceinline__ void pairs_elem(i64 n, const i32* __restrict__ t, const u64* __restrict__ s,
                                           const i64* __restrict__ accA, const i64* __restrict__ ss0, i32* match) {
    const i32 m = t[n];
    const i32 tm = t[m >= 0 ? m : 0];
    if (!((int)(m >= 0) & (int)(tm == (i32)n) & (int)((i32)n < m))) return;
    const i64 ss1 = (i64)s[n] + load_l2(&accA[n]) + load_l2(&accA[m]);
    if (ss1 > ss0[n] + ss0[m]) {
        match[n] = m;
        match[m] = (i32)n;
    }
}

// Top-down at depth d (Eq. match): a node its parent did not take picks its
// best child when that child's return is positive.
__device__ __forceinline__ void down_elem(i64 n, int d, const i32* __restrict__ depth,
                                          const u64* __restrict__ accBV, const i32* __restrict__ accBC,
                                          i32* match) {
    const i32 dn = depth[n], mn = match[n];
    if ((int)(dn != d) | (int)(mn >= 0)) return;
    const i32 bc = load_l2(&accBC[n]);
    const i64 bv = dec_i64(load_l2(&accBV[n]));
    if ((int)(bc >= 0) & (int)(bv > 0)) {
        match[n] = bc;
        match[bc] = (i32)n;
    }
}

// The prototype's greedy matching (the ablation of Sec. VII-D, Reading R28):
// every node's best child by (score, id), the lexicographic maximum taken in
// two phases (scores, then the ids holding the maximum score); two-cycles
// always matched; then, from the roots down, a node left unmatched takes its
// best child.
__device__ __forceinline__ void greedy_best_a_elem(i64 n, const i32* __restrict__ parent, const u64* __restrict__ s,
                                                   u64* accBV) {
    const i32 p = parent[n];
    if (p >= 0) atomicMax((unsigned long long*)&accBV[p], (unsigned long long)s[n]);
}

__device__ __forceinline__ void greedy_best_b_elem(i64 n, const i32* __restrict__ parent, const u64* __restrict__ s,
                                                   const u64* __restrict__ accBV, i32* accBC) {
    const i32 p = parent[n];
    const u64 bv = load_l2(&accBV[p >= 0 ? p : 0]);
    if ((int)(p >= 0) & (int)(s[n] == bv)) atomicMax(&accBC[p], (i32)n);
}

__device__ __forceinline__ void greedy_pairs_elem(i64 n, const i32* __restrict__ t, i32* match) {
    const i32 m = t[n];
    const i32 tm = t[m >= 0 ? m : 0];
    if ((int)(m >= 0) & (int)(tm == (i32)n)) match[n] = m;
}

__device__ __forceinline__ void greedy_down_elem(i64 n, int d, const i32* __restrict__ depth,
                                                 const i32* __restrict__ accBC, i32* match) {
    const i32 dn = depth[n], mn = match[n];
    if ((int)(dn != d) | (int)(mn >= 0)) return;
    const i32 bc = load_l2(&accBC[n]);
    if (bc >= 0) {
        match[n] = bc;
        match[bc] = (i32)n;
    }
}

#define HGP_GRID_LOOP(i, n) for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (i64)gridDim.x * blockDim.x)

__global__ void k_greedy_best_a(i32 N, const i32* __restrict__ parent, const u64* __restrict__ s, u64* accBV) {
    HGP_GRID_LOOP(n, N) greedy_best_a_elem(n, parent, s, accBV);
}

__global__ void k_greedy_best_b(i32 N, const i32* __restrict__ parent, const u64* __restrict__ s,
                                const u64* __restrict__ accBV, i32* accBC) {
    HGP_GRID_LOOP(n, N) greedy_best_b_elem(n, parent, s, accBV, accBC);
}

__global__ void k_greedy_pairs(i32 N, const i32* __restrict__ t, i32* match) {
    HGP_GRID_LOOP(n, N) greedy_pairs_elem(n, t, match);
}

__global__ void k_greedy_down(i32 N, int d, const i32* __restrict__ depth, const i32* __restrict__ accBC,
                              i32* match) {
    HGP_GRID_LOOP(n, N) greedy_down_elem(n, d, depth, accBC, match);
}

__global__ void k_round_targets(i32 N, int Pi, int r, const i32* __restrict__ cand, const u64* __restrict__ score,
                                const i32* __restrict__ match, i32* t, u64* s) {
    HGP_GRID_LOOP(n, N) round_targets_elem(n, Pi, r, cand, score, match, t, s);
}

__global__ void k_round_parent(i32 N, const i32* __restrict__ t, i32* parent, i32* jump, i32* depth, i64* accA,
                               u64* accBV, i32* accBC) {
    HGP_GRID_LOOP(n, N) round_parent_elem(n, t, parent, jump, depth, accA, accBV, accBC);
}

// *pending counts nodes whose pointer has not reached a root yet.
__global__ void k_jump(i32 N, const i32* __restrict__ jin, const i32* __restrict__ din, i32* jout, i32* dout,
                       unsigned long long* pending) {
    unsigned long long c = 0;
    HGP_GRID_LOOP(n, N) c += (unsigned long long)jump_elem(n, jin, din, jout, dout);
    c = wave_sum(c);
    if (lane_id() == 0 && c) atomicAdd(pending, c);
}

__global__ void k_max_i32(i32 N, const i32* __restrict__ v, unsigned long long* out) {
    i32 m = -1;
    HGP_GRID_LOOP(n, N) m = max(m, v[n]);
    m = wave_max(m);
    if (lane_id() == 0 && m >= 0) atomicMax(out, (unsigned long long)m);
}

__global__ void k_up_a(i32 N, int d, const i32* __restrict__ depth, const i32* __restrict__ parent,
                       const u64* __restrict__ s, i64* accA, u64* accBV, const i32* __restrict__ accBC, i64* ss0,
                       i64* ss10) {
    HGP_GRID_LOOP(n, N) up_a_elem(n, d, depth, parent, s, accA, accBV, accBC, ss0, ss10);
}

__global__ void k_up_b(i32 N, int d, const i32* __restrict__ depth, const i32* __restrict__ parent,
                       const i64* __restrict__ ss10, const u64* __restrict__ accBV, i32* accBC) {
    HGP_GRID_LOOP(n, N) up_b_elem(n, d, depth, parent, ss10, accBV, accBC);
}

__global__ void k_pairs(i32 N, const i32* __restrict__ t, const u64* __restrict__ s, const i64* __restrict__ accA,
                        const i64* __restrict__ ss0, i32* match) {
    HGP_GRID_LOOP(n, N) pairs_elem(n, t, s, accA, ss0, match);
}

__global__ void k_down(i32 N, int d, const i32* __restrict__ depth, const u64* __restrict__ accBV,
                       const i32* __restrict__ accBC, i32* match) {
    HGP_GRID_LOOP(n, N) down_elem(n, d, depth, accBV, accBC, match);
}

// All Pi matching rounds in one workgroup, for levels where the per-depth
// launches and host checks would dominate.  Same steps as the kernels above,
// separated by block barriers; pointer buffers alternate as on the host.
constexpr int kMatchSingleMax = 16384;

__global__ __launch_bounds__(1024) void k_match_rounds(i32 N, int Pi, int jump_iters, const i32* __restrict__ cand,
                                                       const u64* __restrict__ score, i32* match, i32* t, u64* s,
                                                       i32* parent, i32* j0, i32* j1, i32* d0, i32* d1, i64* accA,
                                                       u64* accBV, i32* accBC, i64* ss0, i64* ss10, int greedy) {
    __shared__ unsigned long long red[16];
    __shared__ i32 redi[16];
    for (int r = 0; r < Pi; ++r) {
        for (i64 n = threadIdx.x; n < N; n += blockDim.x) round_targets_elem(n, Pi, r, cand, score, match, t, s);
        __syncthreads();
        for (i64 n = threadIdx.x; n < N; n += blockDim.x)
            round_parent_elem(n, t, parent, j0, d0, accA, accBV, accBC);
        __syncthreads();
        i32 *ja = j0, *jb = j1, *da = d0, *db = d1;
        for (int it = 0; it < jump_iters; ++it) {
            unsigned long long c = 0;
            for (i64 n = threadIdx.x; n < N; n += blockDim.x) c += (unsigned long long)jump_elem(n, ja, da, jb, db);
            c = block_sum(c, red);  // ends with a barrier
            i32* tp = ja;
            ja = jb;
            jb = tp;
            tp = da;
            da = db;
            db = tp;
            if (c == 0) break;
        }
        i32 m = -1;
        for (i64 n = threadIdx.x; n < N; n += blockDim.x) m = max(m, da[n]);
        m = wave_max(m);
        if (lane_id() == 0) redi[wave_id()] = m;
        __syncthreads();
        i32 maxd = -1;
        for (int w = 0; w < (int)(blockDim.x / kWave); ++w) maxd = max(maxd, redi[w]);
        __syncthreads();
        const i32* depth = da;
        if (greedy) {
            for (i64 n = threadIdx.x; n < N; n += blockDim.x) greedy_best_a_elem(n, parent, s, accBV);
            __syncthreads();
            for (i64 n = threadIdx.x; n < N; n += blockDim.x) greedy_best_b_elem(n, parent, s, accBV, accBC);
            for (i64 n = threadIdx.x; n < N; n += blockDim.x) greedy_pairs_elem(n, t, match);
            __syncthreads();
            for (int d = 0; d <= maxd; ++d) {
                for (i64 n = threadIdx.x; n < N; n += blockDim.x) greedy_down_elem(n, d, depth, accBC, match);
                __syncthreads();
            }
            continue;
        }
        for (int d = maxd; d >= 0; --d) {
            for (i64 n = threadIdx.x; n < N; n += blockDim.x)
                up_a_elem(n, d, depth, parent, s, accA, accBV, accBC, ss0, ss10);
            __syncthreads();
            for (i64 n = threadIdx.x; n < N; n += blockDim.x) up_b_elem(n, d, depth, parent, ss10, accBV, accBC);
            __syncthreads();
        }
        for (i64 n = threadIdx.x; n < N; n += blockDim.x) pairs_elem(n, t, s, accA, ss0, match);
        __syncthreads();
        for (int d = 0; d <= maxd; ++d) {
            for (i64 n = threadIdx.x; n < N; n += blockDim.x) down_elem(n, d, depth, accBV, accBC, match);
            __syncthreads();
        }
    }
}

// ---- isolated pairing (Sec. V-C) --------------------------------------------
__global__ void k_iso_flags(i32 N, int Pi, const i32* __restrict__ cand, i32* flag) {
    for (i64 n = (i64)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (i64)gridDim.x * blockDim.x)
        flag[n] = cand[n * Pi] < 0 ? 1 : 0;
}

__global__ void k_iso_keys(i32 N, const i32* __restrict__ flag, const i32* __restrict__ pos,
                           const i32* __restrict__ nw, u64* keys, i32* vals) {
    for (i64 n = (i64)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (i64)gridDim.x * blockDim.x)
        if (flag[n]) {
            keys[pos[n]] = ((u64)(u32)nw[n] << 32) | (u64)(u32)n;
            vals[pos[n]] = (i32)n;
        }
}

// Nodes sorted by (size, id): the smallest left pairs with the largest that
// fits both caps, with |in| + |in| standing in for the union.  The walk is
// serial (each pairing moves both ends), but the search for the largest
// fitting partner of the current smallest node is done by one wave over 64
// candidates at a time: the serial walk would step down one candidate per
// iteration to the same partner.
__global__ __launch_bounds__(1024) void k_iso_pair(i32 cnt, const i32* __restrict__ order,
                                                   const i32* __restrict__ nw, const i32* __restrict__ nin,
                                                   i64 omega, i64 delta, i32* match, int staged) {
    // With `staged`, the block first gathers sizes and |in| of the sorted nodes
    // into shared memory so that the walk reads only LDS.
    extern __shared__ i32 st[];
    i32* sw = st;
    i32* si = st + (staged ? cnt : 0);
    if (staged) {
        for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
            const i32 v = order[t];
            sw[t] = nw[v];
            si[t] = nin[v];
        }
        __syncthreads();
    }
    if (wave_id() != 0) return;
    const int lane = lane_id();
    i32 i = 0, j = cnt - 1;
    while (i < j) {
        const i64 wa = staged ? sw[i] : nw[order[i]];
        const i64 ia = staged ? si[i] : nin[order[i]];
        const i32 jl = j - lane;
        const i32 q = jl > i ? jl : i;  // in range; lanes at or below i never fit
        const i64 wb = staged ? sw[q] : nw[order[q]];
        const i64 ib = staged ? si[q] : nin[order[q]];
        const int ok = (int)(jl > i) & (int)(wa + wb <= omega) & (int)(ia + ib <= delta);
        const u64 mask = __ballot(ok);
        if (mask == 0) {
            j -= kWave;
            continue;
        }
        const i32 jp = j - (__ffsll((long long)mask) - 1);  // lowest lane: the largest fitting partner
        if (lane == 0) {
            const i32 a = order[i], b = order[jp];
            match[a] = b;
            match[b] = a;
        }
        ++i;
        j = jp - 1;
    }
}

// ---- cluster map (Sec. V-E) ------------------------------------------------
__global__ void k_rep_flags(i32 N, const i32* __restrict__ match, i32* rep, unsigned long long* pairs) {
    unsigned long long c = 0;
    for (i64 n = (i64)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (i64)gridDim.x * blockDim.x) {
        const i32 m = match[n];
        rep[n] = ((int)(m < 0) | (int)(m > (i32)n)) ? 1 : 0;
        c += (m > (i32)n) ? 1 : 0;
    }
    c = wave_sum(c);
    if (lane_id() == 0 && c) atomicAdd(pairs, c);
}

// gamma(n) = rank of the cluster's smallest member; sizes add up.
__global__ void k_gamma(i32 N, const i32* __restrict__ match, const i32* __restrict__ cid,
                        const i32* __restrict__ nw, i32* gamma, i32* nw2) {
    for (i64 n = (i64)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (i64)gridDim.x * blockDim.x) {
        const i32 m = match[n];
        const int is_rep = (int)(m < 0) | (int)(m > (i32)n);
        const i32 r = is_rep ? (i32)n : m;
        gamma[n] = cid[r];
        const i32 wm = nw[m >= 0 ? m : (i32)n];
        if (is_rep) nw2[cid[n]] = nw[n] + (m >= 0 ? wm : 0);
    }
}

int bits_for(u64 v) {
    int b = 0;
    while (b < 64 && (v >> b) != 0) ++b;
    return b;
}

template <typename BIN>
void launch_propose_hash(Ctx* c, const Level& L, int Pi, const unsigned long long* stats, int ib, i32* cand,
                         u64* score) {
    const int C = 1 << (c->opt.tune[0] ? c->opt.tune[0] : 12);  // slots; shared memory = C * (8 + sizeof(BIN)) B
    const size_t lds = (size_t)C * (8 + sizeof(BIN));
    // as many blocks as are resident at once (registers and shared memory, as
    // the runtime's occupancy query gives them): a second, partial round of
    // blocks would leave most of the chip idle while it runs
    int per_cu = 0;
#define HGP_PROPH_OCC(PIV)                                                                                         \
    case PIV:                                                                                                      \
        if constexpr (std::is_same<BIN, u32>::value) {                                                             \
            HIPC(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_propose_hash32<PIV>, 256, lds));         \
        } else {                                                                                                   \
            HIPC(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_propose_hash<BIN, PIV>, 256, lds));      \
        }                                                                                                          \
        break;
    switch (Pi) {
        HGP_PROPH_OCC(1) HGP_PROPH_OCC(2) HGP_PROPH_OCC(3) HGP_PROPH_OCC(4) HGP_PROPH_OCC(5) HGP_PROPH_OCC(6)
        HGP_PROPH_OCC(7) HGP_PROPH_OCC(8)
        default: fail(HGP_E_INVALID, "pi must be in 1..8");
    }
#undef HGP_PROPH_OCC
    const int grid = std::min<i64>(L.N, (i64)c->num_cu * std::max(1, per_cu));
#define HGP_PROPH(PIV)                                                                                             \
    case PIV:                                                                                                      \
        if constexpr (std::is_same<BIN, u32>::value) {                                                             \
            LAUNCH(c, KF_PROPOSE, (k_propose_hash32<PIV>), grid, 256, lds, L.N, L.inc_off(), L.inc_nin(),          \
                   L.inc(), L.he_off(), L.he_nsrc(), L.pins(), c->hw(), L.nw(), c->omega, c->delta, c->opt.seed,   \
                   stats, ib, cand, score, C);                                                                     \
        } else {                                                                                                   \
            LAUNCH(c, KF_PROPOSE, (k_propose_hash<BIN, PIV>), grid, 256, lds, L.N, L.inc_off(), L.inc_nin(),      \
                   L.inc(), L.he_off(), L.he_nsrc(), L.pins(), c->hw(), L.nw(), c->omega, c->delta, c->opt.seed,   \
                   stats, ib, cand, score, C);                                                                     \
        }                                                                                                          \
        break;
    switch (Pi) {
        HGP_PROPH(1) HGP_PROPH(2) HGP_PROPH(3) HGP_PROPH(4) HGP_PROPH(5) HGP_PROPH(6) HGP_PROPH(7) HGP_PROPH(8)
        default: fail(HGP_E_INVALID, "pi must be in 1..8");
    }
#undef HGP_PROPH
}

template <typename BIN>
void launch_propose(Ctx* c, const Level& L, int Pi, const unsigned long long* stats, int ib, i32* cand,
                    u64* score) {
    // Dense id-range histogram while the node ids fit in a few passes over
    // 64 KiB of bins.  Beyond, the hashed table when a node's neighbourhood
    // typically fits it in a few passes (each pass re-reads all of a node's
    // pins; the table adapts its pass count per node), else dense passes,
    // which read each destination pin once.  The typical neighbourhood is
    // bounded by the mean of sum_{e in I(n)} (|e| - 1) over the nodes,
    // (sum_e |e|^2 - P) / N.
    const i64 dense_passes = ceil_div((i64)L.N, (i64)(65536 / (int)sizeof(BIN)));
    const i64 mean_bound = ((i64)c->sum_card_sq - L.P) / std::max<i64>(1, L.N);
    i64 hash_passes = 1;
    while (hash_passes * 2048 < mean_bound) hash_passes <<= 1;
    const bool hashed = dense_passes > 4 && (hash_passes <= std::max<i64>(4, dense_passes / 4) || dense_passes > 256);
    if (hashed || c->force_hash_propose) {
        launch_propose_hash<BIN>(c, L, Pi, stats, ib, cand, score);
        return;
    }
    // Bins per pass: all neighbour ids at once when they fit 64 KiB of LDS,
    // otherwise 128 KiB worth per pass in one 8-wave block per CU (half the
    // passes: each pass re-reads the sources and the pass bounds); smaller
    // histograms let more blocks share a CU.
    const int r64 = 65536 / (int)sizeof(BIN);
    const bool big = L.N > r64;
    const int rmax = big ? 2 * r64 : r64;
    const int waves = big ? kProposeWavesBig : kProposeWaves;
    const int R = (int)std::min<i64>(rmax, std::max<i64>(64, L.N));
    const size_t lds = sizeof(BIN) * (size_t)propose_bins_alloc(R);
    const size_t lds_all =
        lds + (big ? sizeof(ProposeShared<BIN, kProposeWavesBig>) : sizeof(ProposeShared<BIN, kProposeWaves>)) + 256;
    const int per_cu = std::max(1, std::min(8, (int)(160 * 1024 / lds_all)));
    const int grid = std::min<i64>(L.N, (i64)c->num_cu * per_cu * 2);
    const int npass = (int)ceil_div(L.N, R);
    i32* bnd = nullptr;
    if (npass > 1 && L.E > 0) {
        bnd = wsp<i32>(c, WS_BND, (size_t)L.E * (npass + 1));
        LAUNCH(c, KF_LEVEL_STATS, k_pass_bounds, grid_for(L.E, 256, c->num_cu * 8), 256, 0, L.E, L.he_off(),
               L.he_nsrc(), L.pins(), R, npass, bnd);
    }
    // Ids of at most 65,536 nodes are read from the level's 16-bit pin
    // mirror: half the bytes per pin visit.
    const unsigned short* pins16 = (const unsigned short*)L.b_pins16.p;
#define HGP_PROPW(PIV, PINT, PINS, WV)                                                                             \
    LAUNCH(c, KF_PROPOSE, (k_propose<BIN, PIV, PINT, WV>), grid, WV * kWave, lds, L.N, L.inc_off(), L.inc_nin(),  \
           L.inc(), L.he_off(), L.he_nsrc(), PINS, c->hw(), L.nw(), c->omega, c->delta, c->opt.seed, stats, ib,  \
           cand, score, R, bnd)
#define HGP_PROP(PIV)                                                                                              \
    case PIV:                                                                                                      \
        if (pins16 && waves == kProposeWavesBig)                                                                   \
            HGP_PROPW(PIV, unsigned short, pins16, kProposeWavesBig);                                              \
        else if (pins16)                                                                                           \
            HGP_PROPW(PIV, unsigned short, pins16, kProposeWaves);                                                 \
        else if (waves == kProposeWavesBig)                                                                        \
            HGP_PROPW(PIV, i32, L.pins(), kProposeWavesBig);                                                       \
        else                                                                                                       \
            HGP_PROPW(PIV, i32, L.pins(), kProposeWaves);                                                          \
        break;
    switch (Pi) {
        HGP_PROP(1) HGP_PROP(2) HGP_PROP(3) HGP_PROP(4) HGP_PROP(5) HGP_PROP(6) HGP_PROP(7) HGP_PROP(8)
        default: fail(HGP_E_INVALID, "pi must be in 1..8");
    }
#undef HGP_PROP
#undef HGP_PROPW
}

}  // namespace

void coarsen_level(Ctx* c, int lv) {
    const Level& L = c->levels[lv];
    const i32 N = L.N;
    const int Pi = c->opt.pi;
    const int nb = grid_for(N, 256, c->num_cu * 8);
    unsigned long long* stats = wsp<unsigned long long>(c, WS_STATS, 16);
    HIPC(hipMemsetAsync(stats, 0, 16 * sizeof(u64), c->stream));
    u64* te = wsp<u64>(c, WS_TE, (size_t)(L.E > 0 ? L.E : 1));
    i32* cm1 = wsp<i32>(c, WS_CM1, (size_t)(L.E > 0 ? L.E : 1));
    if (L.E > 0)
        LAUNCH(c, KF_LEVEL_STATS, k_edge_tsum, grid_for(L.E, 256, c->num_cu * 4), 256, 0, L.E, L.he_off(), c->hw(),
               stats, te, cm1);
    LAUNCH(c, KF_LEVEL_STATS, k_node_tsum, grid_for(N, 4, c->num_cu * 16), 256, 0, N, L.inc_off(), L.inc_nin(),
           L.inc(), (const u64*)te, (const i32*)cm1, L.nw(), stats);
    LAUNCH(c, KF_LEVEL_STATS, k_noise_cap, 1, 1, 0, stats);
    i64 st[16];
    read_back(c, stats, st, 16, 8);
    const u64 max_tsum = (u64)st[0], max_nin = (u64)st[1];
    c->max_nbound = (i64)st[12];
    c->sum_card_sq = (u64)st[13];

    Level& Lm = c->levels[lv];
    Lm.b_cand = c->alloc(sizeof(i32) * (size_t)N * Pi);
    Lm.b_score = c->alloc(sizeof(u64) * (size_t)N * Pi);
    Lm.b_match = c->alloc(sizeof(i32) * (size_t)N);
    i32* cand = (i32*)Lm.b_cand.p;
    u64* score = (u64*)Lm.b_score.p;
    i32* match = (i32*)Lm.b_match.p;

    // Histogram bins pack (eta << ib) | inter; pick the narrowest that holds both.
    const int ib = std::max(1, bits_for(max_nin));
    const u64 max_t = (u64)st[14], sum_card_sq = (u64)st[13];
    const bool dense_ok = bits_for(max_tsum) <= 64 - ib && !c->force_hash_propose && !(c->opt.flags & 4) &&
                          dense_proposal_fits(N, L.E, max_t);
    if (dense_ok && ((c->opt.flags & 2) || prefer_dense_proposal(c, N, L.E, max_t, sum_card_sq)))
        propose_dense(c, L, Pi, stats, ib, max_t, cand, score);
    else if (ib < 32 && bits_for(max_tsum) <= 32 - ib)
        launch_propose<u32>(c, L, Pi, stats, ib, cand, score);
    else if (bits_for(max_tsum) <= 64 - ib)
        launch_propose<unsigned long long>(c, L, Pi, stats, ib, cand, (u64*)score);
    else
        fail(HGP_E_UNSUPPORTED, "histogram values exceed 64 bits");

    // Pi matching rounds.
    i32* t = wsp<i32>(c, WS_T, N);
    u64* s = wsp<u64>(c, WS_S, N);
    i32* parent = wsp<i32>(c, WS_PARENT, N);
    i32* j0 = wsp<i32>(c, WS_J0, N);
    i32* j1 = wsp<i32>(c, WS_J1, N);
    i32* d0 = wsp<i32>(c, WS_D0, N);
    i32* d1 = wsp<i32>(c, WS_D1, N);
    i64* accA = wsp<i64>(c, WS_ACC_A, N);
    u64* accBV = wsp<u64>(c, WS_ACC_BV, N);
    i32* accBC = wsp<i32>(c, WS_ACC_BC, N);
    i64* ss0 = wsp<i64>(c, WS_SS0, N);
    i64* ss10 = wsp<i64>(c, WS_SS10, N);
    fill_i32(c, match, -1, N);
    const int jump_iters = bits_for((u64)N) + 1;
    const int greedy = (c->opt.flags & 64) ? 1 : 0;  // the prototype's greedy matching (ablation)
    if (N <= kMatchSingleMax)
        LAUNCH(c, KF_MATCH, k_match_rounds, 1, 1024, 0, N, Pi, jump_iters, cand, (const u64*)score, match, t, s,
               parent, j0, j1, d0, d1, accA, accBV, accBC, ss0, ss10, greedy);
    for (int r = 0; r < Pi && N > kMatchSingleMax; ++r) {
        LAUNCH(c, KF_MATCH, k_round_targets, nb, 256, 0, N, Pi, r, cand, score, match, t, s);
        LAUNCH(c, KF_MATCH, k_round_parent, nb, 256, 0, N, t, parent, j0, d0, accA, accBV, accBC);
        i32 *ja = j0, *jb = j1, *da = d0, *db = d1;
        for (int it = 0; it < jump_iters; ++it) {
            HIPC(hipMemsetAsync(stats + 7, 0, sizeof(u64), c->stream));
            LAUNCH(c, KF_MATCH, k_jump, nb, 256, 0, N, ja, da, jb, db, stats + 7);
            std::swap(ja, jb);
            std::swap(da, db);
            if (it % 3 == 2) {  // every pointer at a root: depths are final
                i64 pend = 0;
                read_back(c, stats + 7, &pend, 1, 8);
                if (pend == 0) break;
            }
        }
        HIPC(hipMemsetAsync(stats + 5, 0, sizeof(u64), c->stream));
        LAUNCH(c, KF_MATCH, k_max_i32, nb, 256, 0, N, da, stats + 5);
        i64 maxd = 0;
        read_back(c, stats + 5, &maxd, 1, 8);
        const i32* depth = da;
        if (greedy) {
            LAUNCH(c, KF_MATCH, k_greedy_best_a, nb, 256, 0, N, parent, s, accBV);
            LAUNCH(c, KF_MATCH, k_greedy_best_b, nb, 256, 0, N, parent, s, accBV, accBC);
            LAUNCH(c, KF_MATCH, k_greedy_pairs, nb, 256, 0, N, t, match);
            for (int d = 0; d <= (int)maxd; ++d)
                LAUNCH(c, KF_MATCH, k_greedy_down, nb, 256, 0, N, d, depth, accBC, match);
            continue;
        }
        for (int d = (int)maxd; d >= 0; --d) {
            LAUNCH(c, KF_MATCH, k_up_a, nb, 256, 0, N, d, depth, parent, s, accA, accBV, accBC, ss0, ss10);
            LAUNCH(c, KF_MATCH, k_up_b, nb, 256, 0, N, d, depth, parent, ss10, accBV, accBC);
        }
        LAUNCH(c, KF_MATCH, k_pairs, nb, 256, 0, N, t, s, accA, ss0, match);
        for (int d = 0; d <= (int)maxd; ++d)
            LAUNCH(c, KF_MATCH, k_down, nb, 256, 0, N, d, depth, accBV, accBC, match);
    }

    // Isolated nodes.
    i32* flag = wsp<i32>(c, WS_ISO_FLAG, N);
    i32* pos = wsp<i32>(c, WS_ISO_POS, (size_t)N + 1);
    LAUNCH(c, KF_ISOLATED, k_iso_flags, nb, 256, 0, N, Pi, cand, flag);
    scan_excl_i32(c, flag, pos, N);
    i64 niso = 0;
    read_back(c, pos + N, &niso, 1, 4);
    if (niso >= 2) {
        u64* keys = wsp<u64>(c, WS_ISO_KEYS, niso);
        u64* keys2 = wsp<u64>(c, WS_ISO_KEYS2, niso);
        i32* vals = wsp<i32>(c, WS_ISO_VALS, niso);
        i32* vals2 = wsp<i32>(c, WS_ISO_VALS2, niso);
        LAUNCH(c, KF_ISOLATED, k_iso_keys, nb, 256, 0, N, flag, pos, L.nw(), keys, vals);
        sort_pairs_u64(c, keys, keys2, vals, vals2, niso, 64);
        const int staged = niso <= 8192 ? 1 : 0;  // 64 KiB of shared memory at most
        LAUNCH(c, KF_ISOLATED, k_iso_pair, 1, 1024, staged ? sizeof(i32) * 2 * niso : 0, (i32)niso, vals2, L.nw(),
               L.inc_nin(), c->omega, c->delta, match, staged);
    }

    // Cluster map.
    i32* rep = wsp<i32>(c, WS_REP, N);
    i32* cid = wsp<i32>(c, WS_CID, (size_t)N + 1);
    HIPC(hipMemsetAsync(stats + 6, 0, sizeof(u64), c->stream));
    LAUNCH(c, KF_GAMMA, k_rep_flags, nb, 256, 0, N, match, rep, stats + 6);
    scan_excl_i32(c, rep, cid, N);
    i64 pairs = 0;
    read_back(c, stats + 6, &pairs, 1, 8);
    c->levels[lv].pairs = pairs;
    if (pairs == 0) return;

    Level nl;
    nl.N = N - (i32)pairs;
    c->levels[lv].b_gamma = c->alloc(sizeof(i32) * (size_t)N);
    nl.b_nw = c->alloc(sizeof(i32) * (size_t)nl.N);
    LAUNCH(c, KF_GAMMA, k_gamma, nb, 256, 0, N, match, cid, L.nw(), c->levels[lv].gamma(), nl.nw());
    contract_edges(c, c->levels[lv], c->levels[lv].gamma(), nl);
    build_incidence(c, nl);
    c->levels.push_back(nl);
}

}  // namespace hgp
