// Exact top-PI candidate selection from a node's histogram (Sec. V-C), shared
// by the id-range, hashed and dense proposal kernels.
//
// Every lane keeps the PI best valid (score, id) pairs it has been given, in
// descending lexicographic order (score = eta + symmetric noise, ties to the
// larger id); the block merges the lane lists at the end.  A bin can enter the
// block's top PI only if its largest possible score, eta plus the noise cap,
// reaches both the lane's PI-th best (once the lane holds PI) and the block
// floor (the largest PI-th best of any full lane list): PI valid candidates
// already beat anything below either.  That bound is one compare on the packed
// bin.  After each scoring round the wave can also raise the floor to the best
// score that PI of its lanes all reach with their best entries.  Bins that
// pass are compacted through a per-wave ring in shared memory
// and scored 64 at a time (noise hash, validity operands, insertion), so the
// costly part runs on full waves however sparse the survivors are.  Which lane
// scores a bin does not matter: every bin reaches exactly one lane list or is
// provably outside the top PI, so the merged result is the exact top PI.
#pragma once

#include "dev_util.h"

namespace hgp {

constexpr int kSelQ = 128;  // ring slots per wave: fewer than 64 wait, at most 64 arrive per push

template <typename BIN>
struct SelQueue {
    i32 m[kSelQ];
    BIN v[kSelQ];
};

template <int PI>
struct TopList {
    u64 s[PI];
    i32 m[PI];

    __device__ __forceinline__ void clear() {
#pragma unroll
        for (int r = 0; r < PI; ++r) {
            s[r] = 0;
            m[r] = -1;
        }
    }
    __device__ __forceinline__ bool full() const { return m[PI - 1] >= 0; }
    // Branch-free sorted insertion; the entry falls off the end if it is worse
    // than all PI.
    __device__ __forceinline__ void insert(u64 cs, i32 cm) {
#pragma unroll
        for (int r = 0; r < PI; ++r) {
            const bool better = lex_better(cs, cm, s[r], m[r]);
            const u64 ts = s[r];
            const i32 tm = m[r];
            s[r] = better ? cs : ts;
            m[r] = better ? cm : tm;
            cs = better ? ts : cs;
            cm = better ? tm : cm;
        }
    }
};

// What the scoring of one node's bins needs.
struct SelNode {
    u64 seed, cap;
    DivU64 ndiv;
    int ib;
    i32 n, nin_n;
    i64 nw_n, omega, delta;
    int all_valid;  // every pair (n, m) is valid: no per-candidate loads
    int union_floor;  // raise the floor by the wave-wide union bound after each scoring round
    const i32* nw;
    const i32* inc_nin;
    unsigned long long* floor;  // block floor, in shared memory
};

__device__ __forceinline__ u64 sel_floor(const SelNode& c) {
    return __hip_atomic_load(c.floor, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Smallest packed bin worth scoring for this lane now: eta + cap must reach
// max(floor, PI-th best when full), and eta >= 1 for any touched bin.  Scores
// are at most eta_max + cap, so the bound never exceeds the packed maximum.
template <typename BIN, int PI>
__device__ __forceinline__ BIN sel_vmin(const TopList<PI>& L, const SelNode& c) {
    const u64 fl = sel_floor(c);
    const u64 own = L.full() ? L.s[PI - 1] : 0ull;
    const u64 thr = fl > own ? fl : own;
    u64 lim = thr > c.cap ? thr - c.cap : 0ull;
    lim = lim > 1ull ? lim : 1ull;
    return (BIN)(lim << c.ib);
}

// Scores cnt (<= 64) queued bins, one per lane, and inserts the valid ones
// that can still matter into the scoring lane's list.
template <typename BIN, int PI>
__device__ __forceinline__ void sel_drain(SelQueue<BIN>& q, u32& qh, u32& qn, u32 cnt, TopList<PI>& L,
                                          const SelNode& c) {
    wave_sync();  // the wave's queue writes are visible to every lane
    const int lane = lane_id();
    const int on = (int)((u32)lane < cnt);
    const u32 pos = (qh + (u32)lane) & (u32)(kSelQ - 1);
    const i32 m = on ? q.m[pos] : 0;
    const BIN v = on ? q.v[pos] : (BIN)0;
    wave_sync();  // slots may be refilled from here on
    qh += cnt;
    qn -= cnt;
    const u64 fl = sel_floor(c);
    const u64 eta = (u64)(v >> c.ib);
    const i64 itr = (i64)(v & ((((BIN)1) << c.ib) - 1));
    const u64 sc = eta + pair_noise(c.seed, c.n, m, c.ndiv);
    const int pick = on & ((int)!L.full() | (int)lex_gt(sc, m, L.s[PI - 1], L.m[PI - 1])) & (int)(sc >= fl);
    const int ld = pick & !c.all_valid;
    const i64 nwm = ld ? (i64)c.nw[m] : 0;
    const i64 ninm = ld ? (i64)c.inc_nin[m] : 0;
    const int ok = pick & (int)(c.nw_n + nwm <= c.omega) & (int)((i64)c.nin_n + ninm - itr <= c.delta);
    if (ok) L.insert(sc, m);  // ok is computed bitwise; the insertion is branch-free
    if ((int)L.full() & (int)(L.s[PI - 1] > fl)) atomicMax(c.floor, (unsigned long long)L.s[PI - 1]);
    // Union bound across the wave: if G lanes (G the smallest power of two
    // >= PI) all hold a best entry scoring at least x, the block already has
    // PI distinct valid candidates scoring >= x, so x is a floor too.  It
    // rises long before any single lane list fills with high scores.
    if (!c.union_floor) return;
    constexpr int G = PI <= 1 ? 1 : PI <= 2 ? 2 : PI <= 4 ? 4 : 8;
    u64 gb = L.m[0] >= 0 ? L.s[0] : 0ull;
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
        const u64 t = __shfl_xor(gb, o, kWave);
        gb = t < gb ? t : gb;
    }
#pragma unroll
    for (int o = G; o < kWave; o <<= 1) {
        const u64 t = __shfl_xor(gb, o, kWave);
        gb = t > gb ? t : gb;
    }
    if ((int)(lane == 0) & (int)(gb > fl)) atomicMax(c.floor, (unsigned long long)gb);
}

// Wave-collective: every lane of the wave calls it, keep says whether the
// lane's bin (m, v) is queued.  Scores a full wave's worth once 64 wait.
template <typename BIN, int PI>
__device__ __forceinline__ void sel_push(SelQueue<BIN>& q, u32& qh, u32& qn, int keep, i32 m, BIN v,
                                         TopList<PI>& L, const SelNode& c) {
    const u64 mask = __ballot(keep);
    if (keep) {
        const u32 below = __builtin_amdgcn_mbcnt_hi((u32)(mask >> 32), __builtin_amdgcn_mbcnt_lo((u32)mask, 0u));
        const u32 pos = (qh + qn + below) & (u32)(kSelQ - 1);
        q.m[pos] = m;
        q.v[pos] = v;
    }
    qn += (u32)__popcll(mask);
    if (qn >= (u32)kWave) sel_drain(q, qh, qn, (u32)kWave, L, c);
}

// Scores whatever is left in the queue.
template <typename BIN, int PI>
__device__ __forceinline__ void sel_flush(SelQueue<BIN>& q, u32& qh, u32& qn, TopList<PI>& L, const SelNode& c) {
    if (qn > 0) sel_drain(q, qh, qn, qn, L, c);
}

// Block merge of the lane lists into the node's PI candidates (id -1 and
// score 0 where fewer than PI exist).  red_s / red_m hold one entry per wave.
template <int PI>
__device__ __forceinline__ void sel_merge(TopList<PI>& L, u64* red_s, i32* red_m, i32* cand_n, u64* score_n) {
    const int lane = lane_id(), wv = wave_id(), nwv = blockDim.x / kWave;
    for (int r = 0; r < PI; ++r) {
        u64 hs = L.s[0];
        i32 hm = L.m[0];
        wave_lexmax(hs, hm);
        if (lane == 0) {
            red_s[wv] = hs;
            red_m[wv] = hm;
        }
        __syncthreads();
        u64 ws = red_s[0];
        i32 wm = red_m[0];
        for (int w = 1; w < nwv; ++w) {
            const u64 s2 = red_s[w];
            const i32 m2 = red_m[w];
            const bool t = lex_gt(s2, m2, ws, wm);
            ws = t ? s2 : ws;
            wm = t ? m2 : wm;
        }
        __syncthreads();
        if ((int)(wm >= 0) & (int)(L.m[0] == wm)) {
#pragma unroll
            for (int k = 0; k + 1 < PI; ++k) {
                L.s[k] = L.s[k + 1];
                L.m[k] = L.m[k + 1];
            }
            L.s[PI - 1] = 0;
            L.m[PI - 1] = -1;
        }
        if (threadIdx.x == 0) {
            cand_n[r] = wm;
            score_n[r] = wm >= 0 ? ws : 0;
        }
    }
}

}  // namespace hgp
