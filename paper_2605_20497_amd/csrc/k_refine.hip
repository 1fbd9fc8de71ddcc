// One refinement repetition (Sec. VI): pins(p,e) rows, in-isolation moves and
// gains, the moves sequence of ranked chains, in-sequence gains, event-based
// validity of every prefix, and the application of the best valid prefix.
#include <algorithm>
#include <map>
#include <mutex>

#include "dev_util.h"
#include "scan_lb.h"

// Workspace of hgp_evaluate_noalloc, for callers that cannot allocate device
// memory.  Every device the library runs on holds its own copy until the
// process ends.  Host code never passes this name to a kernel or a copy: it
// uses the device address looked up by noalloc_scratch_init.
static __device__ __align__(256) unsigned char scratch[hgp::kNoAllocScratchBytes];

namespace hgp {

namespace {

enum {
    WS_PHI_PART = 60, WS_PHI_CNT = 61, WS_PHI_CIN = 62, WS_PHI_LEN = 63, WS_PSIZE = 64, WS_PD = 65, WS_MDST = 66,
    WS_MGAIN = 67, WS_MFLAG = 68, WS_MPOS = 69, WS_MKEY = 70, WS_MKEY2 = 71, WS_MVAL = 72, WS_SNODE = 73,
    WS_SPS = 74, WS_SPD = 75, WS_SG = 76, WS_SNW = 77, WS_SNIN = 78, WS_SEGB = 79, WS_SEGE = 80, WS_PRED = 81,
    WS_SUCC = 82, WS_PL = 83, WS_PLS = 84, WS_CL = 85, WS_PROP = 86, WS_PROPG = 87, WS_ACCG = 88, WS_ACCN = 89,
    WS_FLAGS = 90, WS_J0 = 91, WS_J1 = 92, WS_MN0 = 93, WS_MN1 = 94, WS_P0 = 95, WS_P1 = 96, WS_R0 = 97,
    WS_R1 = 98, WS_H0 = 99, WS_H1 = 100, WS_HEAD = 101, WS_CG = 102, WS_CLEN = 103, WS_SIDX = 104,
    WS_HF = 105, WS_HPOS = 106, WS_HKEY = 107, WS_HKEY2 = 108, WS_HVAL = 109, WS_HVAL2 = 110, WS_LR = 111,
    WS_LRS = 112, WS_CSTART = 113, WS_SEQN = 114, WS_SEQS = 115, WS_SEQD = 116, WS_POSN = 117, WS_GSEQ = 118,
    WS_EVK = 119, WS_EVK2 = 120, WS_EVI = 121, WS_EVI2 = 122, WS_EVDS = 123, WS_EVDD = 124, WS_ES = 125,
    WS_ED = 126, WS_SEX = 127, WS_DEX = 128, WS_SEGST = 129, WS_DVQ = 130, WS_CEX = 131, WS_VEX = 132,
    WS_RSTATS = 133, WS_DDS = 134, WS_DDD = 135, WS_MDST_SA = 136, WS_MGAIN_SA = 137, WS_CODE = 138, WS_PHI_PART16 = 139,
    WS_SINGLE = 140, WS_EMARK = 141, WS_ELIST = 142, WS_ECOUNT = 143, WS_ELIST2 = 144
};

// rstats: [0] active chain rounds flag, [1] links this round, [2] total links,
// [3] kstar, [4] applied gain, [5] initial violations, [6] chains, [7] spare
constexpr i64 kGradeScale = 10000000;  // 10^7 x the paper's grade with alpha=1e-6, beta=1e-7
constexpr int kWindow = 256;
constexpr int kChainRounds = 16;

// Row lookup: pins(p,e) and pins_in(p,e), zero if p holds no pin of e.
__device__ __forceinline__ void row_find(const i32* __restrict__ part, const i32* __restrict__ cnt,
                                         const i32* __restrict__ cin, i64 r0, i32 L, i32 p, i32& c, i32& ci) {
    i32 lo = 0, hi = L;
    while (lo < hi) {
        const i32 mid = (lo + hi) >> 1;
        if (part[r0 + mid] < p) lo = mid + 1;
        else hi = mid;
    }
    const i32 at = lo < L ? lo : L - 1;  // rows are never empty
    const int hit = (int)(lo < L) & (int)(part[r0 + at] == p);
    const i32 cv = cnt[r0 + at], civ = cin[r0 + at];
    c = hit ? cv : 0;
    ci = hit ? civ : 0;
}

// size(p) = sum of node weights in p (Sec. II-B).  With nbins > 0 (all
// partition ids fit) each block sums in shared memory and adds its nonzero
// totals once at the end, so the device atomics per partition are one per
// block rather than one per node.
__global__ __launch_bounds__(256) void k_part_sizes(i32 N, const i32* __restrict__ rho, const i32* __restrict__ nw,
                                                    i64* psize, int nbins, unsigned long long* bytes) {
    extern __shared__ u32 hist[];
    for (int i = threadIdx.x; i < nbins; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    u64 nodes = 0;
    for (i64 n = (i64)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (i64)gridDim.x * blockDim.x) {
        const i32 p = rho[n], w = nw[n];
        if (nbins > 0) atomicAdd(&hist[p], (u32)w);
        else atomicAdd((unsigned long long*)&psize[p], (unsigned long long)w);
        nodes += 1;
    }
    __syncthreads();
    u64 parts = 0;
    for (int i = threadIdx.x; i < nbins; i += blockDim.x)
        if (hist[i]) {
            atomicAdd((unsigned long long*)&psize[i], (unsigned long long)hist[i]);
            parts += 1;
        }
    // per node its partition and weight (8); per partition total added (8)
    const u64 acc = wave_sum(8 * nodes + 8 * parts);
    if ((bytes != nullptr) & (lane_id() == 0) & (acc != 0)) atomicAdd(bytes, (unsigned long long)acc);
}

// Partition sizes after the previous repetition applied the first k moves of
// its sequence: each applied move takes its node's weight from p_s to p_d.
// Signed counts per block in shared memory when the partition ids fit.
__global__ __launch_bounds__(256) void k_sizes_moved(i64 k, const i32* __restrict__ seqn,
                                                     const i32* __restrict__ seqs, const i32* __restrict__ seqd,
                                                     const i32* __restrict__ nw, i64* psize, int nbins) {
    extern __shared__ i32 shist[];
    for (int i = threadIdx.x; i < nbins; i += blockDim.x) shist[i] = 0;
    __syncthreads();
    for (i64 q = (i64)blockIdx.x * blockDim.x + threadIdx.x; q < k; q += (i64)gridDim.x * blockDim.x) {
        const i32 w = nw[seqn[q]], ps = seqs[q], pd = seqd[q];
        if (nbins > 0) {
            atomicAdd(&shist[ps], -w);
            atomicAdd(&shist[pd], w);
        } else {
            atomicAdd((unsigned long long*)&psize[ps], (unsigned long long)(-(i64)w));
            atomicAdd((unsigned long long*)&psize[pd], (unsigned long long)(i64)w);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nbins; i += blockDim.x)
        if (shist[i]) atomicAdd((unsigned long long*)&psize[i], (unsigned long long)(i64)shist[i]);
}

// sign * |{listed e : pins_in(p,e) > 0}| added to D(p): with the listed
// h-edges' old rows before they are rebuilt (sign -1) and their new rows after
// (sign +1), D follows the rebuild without a pass over every row.
__global__ __launch_bounds__(256) void k_inbound_listed(const i32* __restrict__ elist, const u32* __restrict__ ecount,
                                                        const i64* __restrict__ he_off, const i32* __restrict__ part,
                                                        const i32* __restrict__ cin, const i32* __restrict__ len,
                                                        i64* pD, int nbins, int sign) {
    extern __shared__ i32 shist[];
    for (int i = threadIdx.x; i < nbins; i += blockDim.x) shist[i] = 0;
    __syncthreads();
    const i64 ne = (i64)*ecount;
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < ne; i += (i64)gridDim.x * blockDim.x) {
        const i64 e = elist[i];
        const i64 a = he_off[e];
        const i32 L = len[e];
        for (i32 r = 0; r < L; ++r) {
            if (cin[a + r] > 0) {
                const i32 p = part[a + r];
                if (nbins > 0) atomicAdd(&shist[p], sign);
                else atomicAdd((unsigned long long*)&pD[p], (unsigned long long)(i64)sign);
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nbins; i += blockDim.x)
        if (shist[i]) atomicAdd((unsigned long long*)&pD[i], (unsigned long long)(i64)shist[i]);
}

// D(p) = |{e : pins_in(p,e) > 0}| from the rows.  Each wave takes 64 h-edges,
// one per lane, and walks the concatenation of their rows 64 entries at a
// time (kRowU loads per lane in flight), so every lane is busy whatever the
// row lengths.  With nbins > 0 (all partition ids fit) each block counts in
// shared memory and adds its nonzero counts once at the end.
constexpr int kRowU = 4;

__global__ __launch_bounds__(256) void k_part_inbound(i32 E, const i64* __restrict__ he_off,
                                                      const i32* __restrict__ part, const i32* __restrict__ cin,
                                                      const i32* __restrict__ len, i64* pD, int nbins,
                                                      unsigned long long* bytes) {
    extern __shared__ u32 hist[];
    __shared__ i32 s_start[4][kWave];
    __shared__ i64 s_base[4][kWave];
    const int lane = lane_id(), wv = wave_id();
    const int wpb = blockDim.x / kWave;
    u64 acc = 0;
    for (int i = threadIdx.x; i < nbins; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    for (i64 e0 = ((i64)blockIdx.x * wpb + wv) * kWave; e0 < E; e0 += (i64)gridDim.x * wpb * kWave) {
        const i64 e = e0 + lane;
        const int in_e = (int)(e < E);
        const i32 L = in_e ? len[e] : 0;
        const i64 base = in_e ? he_off[e] : 0;
        const i32 incl = wave_incl_scan(L);
        const i32 excl = incl - L;
        const i32 T = __shfl(incl, kWave - 1, kWave);
        s_start[wv][lane] = excl;
        s_base[wv][lane] = base - excl;  // row entry j of this segment is at s_base + j
        wave_sync();
        int cur = 0;
        for (i32 j0 = 0; j0 < T; j0 += kRowU * kWave) {
            i32 pp[kRowU], cc[kRowU];
#pragma unroll
            for (int u = 0; u < kRowU; ++u) {
                const i32 j = j0 + u * kWave + lane;
                const int in = (int)(j < T);
                while ((int)(cur + 1 < kWave) & in) {
                    if (s_start[wv][cur + 1] > j) break;
                    ++cur;
                }
                const i64 pos = in ? s_base[wv][cur] + j : 0;
                pp[u] = in ? part[pos] : 0;
                cc[u] = in ? cin[pos] : 0;
            }
#pragma unroll
            for (int u = 0; u < kRowU; ++u)
                if (cc[u] > 0) {
                    if (nbins > 0) atomicAdd(&hist[pp[u]], 1u);
                    else atomicAdd((unsigned long long*)&pD[pp[u]], 1ull);
                }
        }
        wave_sync();  // the table is rewritten by the next batch
        // per h-edge its offset and lambda (12), per row entry part and cnt_in (8)
        acc += 12 * (u64)__popcll(__ballot(in_e)) + 8 * (u64)T;
    }
    __syncthreads();
    u64 parts = 0;
    for (int i = threadIdx.x; i < nbins; i += blockDim.x)
        if (hist[i]) {
            atomicAdd((unsigned long long*)&pD[i], (unsigned long long)hist[i]);
            parts += 1;
        }
    acc += wave_sum(8 * parts);
    if ((bytes != nullptr) & (lane == 0) & (acc != 0)) atomicAdd(bytes, (unsigned long long)acc);
}

// Violated partitions before any move.
__global__ void k_initial_violations(i32 nparts, const i64* __restrict__ psize, const i64* __restrict__ pD,
                                     i64 omega, i64 delta, unsigned long long* out) {
    unsigned long long c = 0;
    for (i64 p = (i64)blockIdx.x * blockDim.x + threadIdx.x; p < nparts; p += (i64)gridDim.x * blockDim.x) {
        const i64 sz = psize[p], dd = pD[p];
        c += ((int)(sz > omega) | (int)(dd > delta)) ? 1 : 0;
    }
    c = wave_sum(c);
    if (lane_id() == 0 && c) atomicAdd(out, c);
}

// In-isolation move of each node (Eq. refinement_move_selection), one block per
// node: conn(n,p) = sum of omega(e) over e in I(n) with pins(p,e) > 0,
// accumulated per partition in shared memory; gain(n,p) = saving(n) -
// (W_I(n) - conn(n,p)).  Only partitions adjacent through some h-edge can have
// a positive gain, so only those are visited.  Partition ids are split into
// ranges of R bins, one pass each.
//
// Row sweep: each wave owns a batch of up to 64 incident h-edges (metadata one
// per lane) and walks their pins(p,e) rows kGainsG h-edges at a time, kGainsU
// coalesced loads per h-edge and lane, so kGainsG * kGainsU loads are in flight.
// The row of n's own partition is noted during the first pass's sweep (shared
// memory, one entry per h-edge), and its count, which decides the saving, is
// read once per h-edge after the batch.
constexpr int kGainsG = 4;
constexpr int kGainsU = 4;
constexpr int kGainsWaves = 4;

template <typename PART>
__global__ __launch_bounds__(kGainsWaves * kWave) void k_gains(
    i32 N, i32 nparts, const i64* __restrict__ inc_off, const i32* __restrict__ inc, const i64* __restrict__ he_off,
    const PART* __restrict__ part, const i32* __restrict__ cnt, const i32* __restrict__ len,
    const i32* __restrict__ hw, const i32* __restrict__ nw, const i32* __restrict__ rho,
    const i64* __restrict__ psize, i64 omega, i32* move_dst, i64* move_gain, i32* move_dst_sa,
    i64* move_gain_sa, int R) {
    extern __shared__ u32 bins[];  // R bins: one pass covers R consecutive partition ids
    __shared__ i64 red[16];
    __shared__ i64 red_g[16], red_g2[16];
    __shared__ i32 red_p[16], red_p2[16];
    __shared__ i64 own[kGainsWaves][kWave];  // row of p_s in each h-edge of the batch
    const int lane = lane_id(), wv = wave_id(), nwv = blockDim.x / kWave;
    const int npass = (int)((nparts + R - 1) / R);
    for (int i = threadIdx.x; i < R; i += blockDim.x) bins[i] = 0;
    __syncthreads();
    for (i64 r = 0;; ++r) {
        const i64 nx = xcd_item(r, blockIdx.x, gridDim.x);  // neighbouring nodes on one XCD
        if (nx >= N) break;
        const i32 n = (i32)nx;
        const i32 ps = rho[n];
        const i64 a = inc_off[n], b = inc_off[n + 1];
        const i64 deg = b - a;
        const bool one_batch = deg <= (i64)nwv * kWave;
        const i64 chunk = one_batch ? (deg + nwv - 1) / nwv : (i64)kWave;
        i64 saving = 0, wi = 0;
        i64 bg = 0, bg2 = 0;  // best move, and best move that keeps size(p) + size(n) <= Omega
        i32 bp = -1, bp2 = -1;
        i64 r0 = 0;
        i32 L = 0, w = 0;
        for (int pass = 0; pass < npass; ++pass) {
            const i32 lo = pass * R;
            const i32 hi = min(nparts, lo + R);
            for (i64 kb = a + (i64)wv * chunk; kb < b; kb += (i64)nwv * chunk) {
                const int nb = (int)min((i64)chunk, b - kb);
                if ((pass == 0) | !one_batch) {
                    const i64 k = kb + lane;
                    const int valid = (int)(lane < nb);
                    const i32 e = inc[valid ? k : kb];
                    r0 = he_off[e];
                    const i32 Le = len[e], we = hw[e];
                    L = valid ? Le : 0;
                    w = valid ? we : 0;
                }
                if (pass == 0) own[wv][lane] = r0;
                wave_sync();
                for (int i0 = 0; i0 < nb; i0 += kGainsG) {
                    i64 sb[kGainsG];
                    i32 sl[kGainsG];
                    u32 sw[kGainsG];
                    i32 maxl = 0;
#pragma unroll
                    for (int g = 0; g < kGainsG; ++g) {
                        const int src = min(i0 + g, kWave - 1);
                        sb[g] = bcast(r0, src);
                        const i32 l = bcast(L, src);
                        sl[g] = i0 + g < nb ? l : 0;
                        sw[g] = (u32)bcast(w, src);
                        maxl = max(maxl, sl[g]);
                    }
                    for (i32 q0 = 0; q0 < maxl; q0 += kGainsU * kWave) {
                        i32 pp[kGainsG][kGainsU];
#pragma unroll
                        for (int g = 0; g < kGainsG; ++g)
#pragma unroll
                            for (int u = 0; u < kGainsU; ++u) {
                                const i32 q = q0 + u * kWave + lane;
                                pp[g][u] = q < sl[g] ? (i32)part[sb[g] + q] : -1;
                            }
#pragma unroll
                        for (int g = 0; g < kGainsG; ++g)
#pragma unroll
                            for (int u = 0; u < kGainsU; ++u) {
                                const i32 p = pp[g][u];
                                if ((int)(p != ps) & (int)(p >= lo) & (int)(p < hi)) atomicAdd(&bins[p - lo], sw[g]);
                                // every h-edge of n has exactly one row of p_s: one writer per entry
                                if ((int)(pass == 0) & (int)(p == ps))
                                    own[wv][i0 + g] = sb[g] + q0 + u * kWave + lane;
                            }
                    }
                }
                wave_sync();
                if (pass == 0) {
                    const i32 c_own = L > 0 ? cnt[own[wv][lane]] : 0;  // pins(p_s, e) >= 1
                    wi += w;
                    saving += (int)(c_own == 1) ? w : 0;
                }
                wave_sync();  // the table is rewritten by the next batch
            }
            if (pass == 0) {
                saving = block_sum(saving, red);
                wi = block_sum(wi, red);
            } else {
                __syncthreads();
            }
            const int used = hi - lo;
            for (int sidx = threadIdx.x; sidx < used; sidx += blockDim.x) {
                const u32 v = bins[sidx];
                if (v == 0) continue;
                bins[sidx] = 0;
                const i32 p = lo + sidx;
                const i64 g = saving - (wi - (i64)v);
                const i64 szp = psize[p];
                const int pos = (int)(g > 0);
                const int fits = (int)((i64)nw[n] + szp <= omega);
                const bool t = (pos & (int)lex_better(g, p, bg, bp)) != 0;
                bg = t ? g : bg;
                bp = t ? p : bp;
                const bool t2 = (pos & fits & (int)lex_better(g, p, bg2, bp2)) != 0;
                bg2 = t2 ? g : bg2;
                bp2 = t2 ? p : bp2;
            }
            __syncthreads();
        }
        wave_lexmax_i64(bg, bp);
        wave_lexmax_i64(bg2, bp2);
        if (lane == 0) {
            red_g[wv] = bg;
            red_p[wv] = bp;
            red_g2[wv] = bg2;
            red_p2[wv] = bp2;
        }
        __syncthreads();
        if (threadIdx.x < 2) {
            const i64* rg = threadIdx.x == 0 ? red_g : red_g2;
            const i32* rp = threadIdx.x == 0 ? red_p : red_p2;
            i64 G = rg[0];
            i32 Pp = rp[0];
            for (int w = 1; w < nwv; ++w) {
                const i64 g2 = rg[w];
                const i32 p2 = rp[w];
                const bool t = lex_better(g2, p2, G, Pp);
                G = t ? g2 : G;
                Pp = t ? p2 : Pp;
            }
            i32* md = threadIdx.x == 0 ? move_dst : move_dst_sa;
            i64* mg = threadIdx.x == 0 ? move_gain : move_gain_sa;
            md[n] = Pp;
            mg[n] = Pp >= 0 ? G : 0;
        }
        __syncthreads();
    }
}

// Same moves for at most kGainsFlagParts partitions, from a 16-bit row copy
// whose top bit flags pins(p,e) = 1.  The saving of n is then summed while
// sweeping (the row of p_s in e carries the flag), so no own-row table and no
// per-h-edge count load; with a single pass the bins need no range test.
constexpr i32 kGainsFlagParts = 32767;

// Batches whose rows all have at most kLaneRow entries are swept one row per
// lane: every lane loads its own row whole (kLaneRow loads in flight), one
// dependent round for the batch instead of one per G rows.
constexpr int kLaneRow = 8;

// Partitions a wave's node touched, as a bitmap beside its bins (one bit per
// partition, set with a no-return atomic OR, so the bin updates never wait on
// a returned value); the scan after the sweep visits the set bits only.
struct Touched {
    u32* bits;
};

// One row entry of the 16-bit copy: the bin update of its partition, or for
// the row of p_s the saving (e counts when p_s holds one pin of it).
template <bool ONE_PASS, bool TRACK = false>
__device__ __forceinline__ void gains_entry(u32 raw, u32 w, int pass, i32 ps, i32 lo, i32 hi, i64& saving,
                                            u32* bins, Touched tt = Touched{nullptr}) {
    const i32 p = (i32)(raw & 0x7FFFu);
    const int in = (int)(raw != 0xFFFFFFFFu);
    if ((pass == 0) & in & (int)(p == ps)) saving += (raw >> 15) ? (i64)w : 0;
    const int range = ONE_PASS ? 1 : (int)((u32)(p - lo) < (u32)(hi - lo));
    if (in & (int)(p != ps) & range) {
        atomicAdd(&bins[p - lo], w);
        if (TRACK) atomicOr(&tt.bits[(p - lo) >> 5], 1u << ((p - lo) & 31));
    }
}

// Row sweep of one wave batch for k_gains16: rows G at a time, GU coalesced
// loads per row and lane, so G * GU loads per lane are in flight; short rows
// one per lane.
template <int G, int GU, bool ONE_PASS, bool TRACK = false>
__device__ __forceinline__ void gains_group(int nb, int lane, int pass, i32 ps, i32 lo, i32 hi,
                                            const unsigned short* __restrict__ partf, i64 r0, i32 L, i32 w,
                                            i64& saving, u32* bins, Touched tt = Touched{nullptr}) {
    if (wave_max(L) <= kLaneRow) {
        u32 pp[kLaneRow];
#pragma unroll
        for (int u = 0; u < kLaneRow; ++u) pp[u] = u < L ? (u32)partf[r0 + u] : 0xFFFFFFFFu;
#pragma unroll
        for (int u = 0; u < kLaneRow; ++u)
            gains_entry<ONE_PASS, TRACK>(pp[u], (u32)w, pass, ps, lo, hi, saving, bins, tt);
        return;
    }
    for (int i0 = 0; i0 < nb; i0 += G) {
        const unsigned short* rp[G];
        i32 sl[G];
        u32 sw[G];
        i32 maxl = 0;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int src = min(i0 + g, kWave - 1);
            rp[g] = partf + bcast(r0, src);  // wave-uniform row base
            const i32 l = bcast(L, src);
            sl[g] = i0 + g < nb ? l : 0;
            sw[g] = (u32)bcast(w, src);
            maxl = max(maxl, sl[g]);
        }
        for (i32 q0 = 0; q0 < maxl; q0 += GU * kWave) {
            u32 pp[G][GU];
#pragma unroll
            for (int g = 0; g < G; ++g)
#pragma unroll
                for (int u = 0; u < GU; ++u) {
                    const i32 q = q0 + u * kWave + lane;
                    pp[g][u] = q < sl[g] ? (u32)rp[g][q] : 0xFFFFFFFFu;
                }
#pragma unroll
            for (int g = 0; g < G; ++g)
#pragma unroll
                for (int u = 0; u < GU; ++u)
                    gains_entry<ONE_PASS, TRACK>(pp[g][u], sw[g], pass, ps, lo, hi, saving, bins, tt);
        }
    }
}

template <bool ONE_PASS>
__global__ __launch_bounds__(kGainsWaves * kWave) void k_gains16(
    i32 N, i32 nparts, const i64* __restrict__ inc_off, const i32* __restrict__ inc, const i64* __restrict__ he_off,
    const unsigned short* __restrict__ partf, const i32* __restrict__ len, const i32* __restrict__ hw,
    const i32* __restrict__ nw, const i32* __restrict__ rho, const i64* __restrict__ psize, i64 omega,
    i32* move_dst, i64* move_gain, i32* move_dst_sa, i64* move_gain_sa, int R, unsigned long long* work) {
    extern __shared__ u32 bins[];  // R bins: one pass covers R consecutive partition ids
    __shared__ i64 red[16];
    __shared__ i64 red_g[16], red_g2[16];
    __shared__ i32 red_p[16], red_p2[16];
    const int lane = lane_id(), wv = wave_id(), nwv = blockDim.x / kWave;
    const int npass = ONE_PASS ? 1 : (int)((nparts + R - 1) / R);
    for (int i = threadIdx.x; i < R; i += blockDim.x) bins[i] = 0;
    __syncthreads();
    u64 visits = 0;  // row entries this wave read (work counter when profiling)
    for (i64 r = 0;; ++r) {
        const i64 nx = xcd_item(r, blockIdx.x, gridDim.x);  // neighbouring nodes on one XCD
        if (nx >= N) break;
        const i32 n = (i32)nx;
        const i32 ps = rho[n];
        const i64 a = inc_off[n], b = inc_off[n + 1];
        const i64 deg = b - a;
        const bool one_batch = deg <= (i64)nwv * kWave;
        const i64 chunk = one_batch ? (deg + nwv - 1) / nwv : (i64)kWave;
        i64 saving = 0, wi = 0;
        i64 bg = 0, bg2 = 0;  // best move, and best move that keeps size(p) + size(n) <= Omega
        i32 bp = -1, bp2 = -1;
        i64 r0 = 0;
        i32 L = 0, w = 0;
        const i64 nw_n = nw[n];
        for (int pass = 0; pass < npass; ++pass) {
            const i32 lo = pass * R;
            const i32 hi = min(nparts, lo + R);
            for (i64 kb = a + (i64)wv * chunk; kb < b; kb += (i64)nwv * chunk) {
                const int nb = (int)min((i64)chunk, b - kb);
                if ((pass == 0) | !one_batch) {
                    const i64 k = kb + lane;
                    const int valid = (int)(lane < nb);
                    const i32 e = inc[valid ? k : kb];
                    r0 = he_off[e];
                    const i32 Le = len[e], we = hw[e];
                    L = valid ? Le : 0;
                    w = valid ? we : 0;
                    if (pass == 0) wi += w;
                }
                const i32 tot = wave_sum(L);
                visits += (u64)tot;
                const i32 avg = tot / max(nb, 1);
                if (avg <= 64)
                    gains_group<16, 1, ONE_PASS>(nb, lane, pass, ps, lo, hi, partf, r0, L, w, saving, bins);
                else if (avg <= 128)
                    gains_group<8, 2, ONE_PASS>(nb, lane, pass, ps, lo, hi, partf, r0, L, w, saving, bins);
                else if (avg <= 192)
                    gains_group<6, 3, ONE_PASS>(nb, lane, pass, ps, lo, hi, partf, r0, L, w, saving, bins);
                else
                    gains_group<4, 4, ONE_PASS>(nb, lane, pass, ps, lo, hi, partf, r0, L, w, saving, bins);
            }
            if (pass == 0) {
                saving = block_sum(saving, red);
                wi = block_sum(wi, red);
            } else {
                __syncthreads();
            }
            // Only partitions with conn(n,p) > W_I(n) - saving(n) give a positive gain.
            const i64 need = wi - saving;
            const int used = hi - lo;
            for (int sidx = threadIdx.x; sidx < used; sidx += blockDim.x) {
                const u32 v = bins[sidx];
                if (v == 0) continue;
                bins[sidx] = 0;
                if ((i64)v <= need) continue;
                const i32 p = lo + sidx;
                const i64 g = (i64)v - need;
                const int fits = (int)(nw_n + psize[p] <= omega);
                const bool t = lex_better(g, p, bg, bp);
                bg = t ? g : bg;
                bp = t ? p : bp;
                const bool t2 = (fits & (int)lex_better(g, p, bg2, bp2)) != 0;
                bg2 = t2 ? g : bg2;
                bp2 = t2 ? p : bp2;
            }
            __syncthreads();
        }
        wave_lexmax_i64(bg, bp);
        wave_lexmax_i64(bg2, bp2);
        if (lane == 0) {
            red_g[wv] = bg;
            red_p[wv] = bp;
            red_g2[wv] = bg2;
            red_p2[wv] = bp2;
        }
        __syncthreads();
        if (threadIdx.x < 2) {
            const i64* rg = threadIdx.x == 0 ? red_g : red_g2;
            const i32* rpp = threadIdx.x == 0 ? red_p : red_p2;
            i64 G = rg[0];
            i32 Pp = rpp[0];
            for (int ww = 1; ww < nwv; ++ww) {
                const i64 g2 = rg[ww];
                const i32 p2 = rpp[ww];
                const bool t = lex_better(g2, p2, G, Pp);
                G = t ? g2 : G;
                Pp = t ? p2 : Pp;
            }
            i32* md = threadIdx.x == 0 ? move_dst : move_dst_sa;
            i64* mg = threadIdx.x == 0 ? move_gain : move_gain_sa;
            md[n] = Pp;
            mg[n] = Pp >= 0 ? G : 0;
        }
        __syncthreads();
    }
    // one device atomic per wave: per node they would all meet on one address
    if ((work != nullptr) & (lane == 0) & (visits != 0)) atomicAdd(work, (unsigned long long)visits);
}

// The same moves with one wave per node, for levels whose nodes have few
// incident h-edges (at most kGainsWaveDeg on average) and at most
// kGainsWaveParts partitions.  Each wave owns R bins, so a node costs no block
// barriers or block reductions; with a 4-wave block per node those dominate
// when a node has a handful of h-edges.
constexpr i32 kGainsWaveParts = 4096;  // 64 KiB of bins for the 4 waves of a block
constexpr i64 kGainsWaveDeg = 256;

// Nodes of at most kGainsFlatChunks * 64 incident h-edges whose rows hold at
// most kGainsFlatRow entries are swept with all their loads issued together.
constexpr int kGainsFlatChunks = 4;
constexpr int kGainsFlatRow = 4;

// One 64-h-edge batch of a node (per-lane row base, length and weight).
__device__ __forceinline__ void gains_chunk(i32 avg, int nb, int lane, i32 ps, i32 nparts,
                                            const unsigned short* __restrict__ partf, i64 r0, i32 L, i32 w,
                                            i64& saving, u32* bins, Touched tt) {
    if (avg <= 64)
        gains_group<8, 1, true, true>(nb, lane, 0, ps, 0, nparts, partf, r0, L, w, saving, bins, tt);
    else if (avg <= 128)
        gains_group<4, 2, true, true>(nb, lane, 0, ps, 0, nparts, partf, r0, L, w, saving, bins, tt);
    else
        gains_group<2, 4, true, true>(nb, lane, 0, ps, 0, nparts, partf, r0, L, w, saving, bins, tt);
}

// A node of at most CH * 64 incident h-edges with all its loads issued
// together: incidence, then offsets, lengths and weights, then (rows of at
// most kGainsFlatRow entries) every row entry, three rounds in all; the next
// node's scalars are prefetched behind the incidence loads.  Longer rows go
// through gains_chunk per 64 h-edges.
template <int CH>
__device__ __forceinline__ void gains_flat(i64 a, i64 b, int lane, i32 ps, i32 nparts, const i32* __restrict__ inc,
                                           const i64* __restrict__ he_off, const unsigned short* __restrict__ partf,
                                           const i32* __restrict__ len, const i32* __restrict__ hw, i64& saving,
                                           i64& wi, u64& visits, u32* bins, Touched tt, i64 n2, i32 N,
                                           const i32* __restrict__ rho, const i64* __restrict__ inc_off,
                                           const i32* __restrict__ nw, i32& ps_n, i64& a_n, i64& b_n, i64& nw_nn) {
    i32 ee[CH], LL[CH], ww[CH];
    i64 rr[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
        const i64 k = a + u * kWave + lane;
        ee[u] = inc[k < b ? k : a];
    }
    if (n2 < N) {
        ps_n = rho[n2];
        a_n = inc_off[n2];
        b_n = inc_off[n2 + 1];
        nw_nn = nw[n2];
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
        rr[u] = he_off[ee[u]];
        LL[u] = len[ee[u]];
        ww[u] = hw[ee[u]];
    }
    i32 lmax = 0;
#pragma unroll
    for (int u = 0; u < CH; ++u) {
        const int in = (int)(a + u * kWave + lane < b);
        LL[u] = in ? LL[u] : 0;
        ww[u] = in ? ww[u] : 0;
        wi += ww[u];
        lmax = max(lmax, LL[u]);
    }
    lmax = wave_max(lmax);
    // Every incident h-edge lies in one partition (its row is p_s alone): no
    // other partition meets n, so n has no move whatever its saving, which is
    // the outcome of sweeping the rows; they are not read (the work counter
    // still counts the method's row visits).
    if (lmax <= 1) {
#pragma unroll
        for (int u = 0; u < CH; ++u) visits += (u64)LL[u];
        return;
    }
    if (lmax <= kGainsFlatRow) {
        // every lane loads; entries past a row read its first entry (a row of
        // an h-edge holding n is never empty) and are dropped at use
        u32 pp[CH][kGainsFlatRow];
#pragma unroll
        for (int u = 0; u < CH; ++u)
#pragma unroll
            for (int v = 0; v < kGainsFlatRow; ++v) pp[u][v] = (u32)partf[rr[u] + (v < LL[u] ? v : 0)];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            visits += (u64)LL[u];
#pragma unroll
            for (int v = 0; v < kGainsFlatRow; ++v)
                gains_entry<true, true>(v < LL[u] ? pp[u][v] : 0xFFFFFFFFu, (u32)ww[u], 0, ps, 0, nparts, saving,
                                        bins, tt);
        }
    } else {
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int nb = (int)min((i64)kWave, b - (a + u * kWave));
            if (nb > 0) {
                const i32 tot = wave_sum(LL[u]);
                visits += (u64)LL[u];
                gains_chunk(tot / nb, nb, lane, ps, nparts, partf, rr[u], LL[u], ww[u], saving, bins, tt);
            }
        }
    }
}

__global__ __launch_bounds__(kGainsWaves * kWave) void k_gains16w(
    i32 N, i32 nparts, const i64* __restrict__ inc_off, const i32* __restrict__ inc, const i64* __restrict__ he_off,
    const unsigned short* __restrict__ partf, const i32* __restrict__ len, const i32* __restrict__ hw,
    const i32* __restrict__ nw, const i32* __restrict__ rho, const i64* __restrict__ psize, i64 omega,
    i32* move_dst, i64* move_gain, i32* move_dst_sa, i64* move_gain_sa, int R, unsigned long long* work) {
    extern __shared__ u32 bins_all[];  // R bins per wave, R >= nparts
    __shared__ u32 t_bits[kGainsWaves][kGainsWaveParts / 32];
    const int lane = lane_id(), wv = wave_id(), nwv = blockDim.x / kWave;
    u32* bins = bins_all + (size_t)wv * R;
    for (int i = lane; i < R; i += kWave) bins[i] = 0;
    const int nwords = (nparts + 31) >> 5;  // nparts <= kGainsWaveParts
    for (int i = lane; i < kGainsWaveParts / 32; i += kWave) t_bits[wv][i] = 0;
    const Touched tt{t_bits[wv]};
    wave_sync();
    u64 visits = 0;  // row entries this lane read (work counter when profiling)
    // node of round r for this wave: each block takes nwv consecutive nodes
    // per round, blocks of one XCD adjacent runs of them
    auto node_of = [&](i64 r) { return xcd_item(r, blockIdx.x, gridDim.x) * nwv + wv; };
    i64 rr = 0;
    i64 n = node_of(0);
    // the node's partition, incidence offsets and size, one node ahead
    i32 ps_n = 0;
    i64 a_n = 0, b_n = 0, nw_nn = 0;
    if (n < N) {
        ps_n = rho[n];
        a_n = inc_off[n];
        b_n = inc_off[n + 1];
        nw_nn = nw[n];
    }
    for (; n < N; n = node_of(++rr)) {
        const i32 ps = ps_n;
        const i64 a = a_n, b = b_n;
        const i64 nw_n = nw_nn;
        i64 saving = 0, wi = 0;
        const i64 deg = b - a;
        const bool flat = (deg > 0) & (deg <= kGainsFlatChunks * kWave);
        const i64 n2 = node_of(rr + 1);  // the next node's scalars, behind this node's first loads
        if (flat) {
            if (deg <= 2 * kWave)
                gains_flat<2>(a, b, lane, ps, nparts, inc, he_off, partf, len, hw, saving, wi, visits, bins, tt, n2,
                              N, rho, inc_off, nw, ps_n, a_n, b_n, nw_nn);
            else
                gains_flat<kGainsFlatChunks>(a, b, lane, ps, nparts, inc, he_off, partf, len, hw, saving, wi, visits,
                                             bins, tt, n2, N, rho, inc_off, nw, ps_n, a_n, b_n, nw_nn);
        } else if (n2 < N) {
            ps_n = rho[n2];
            a_n = inc_off[n2];
            b_n = inc_off[n2 + 1];
            nw_nn = nw[n2];
        }
        for (i64 kb = flat ? b : a; kb < b; kb += kWave) {
            const int nb = (int)min((i64)kWave, b - kb);
            const int valid = (int)(lane < nb);
            const i32 e = inc[valid ? kb + lane : kb];
            const i64 r0 = he_off[e];
            const i32 Le = len[e], we = hw[e];
            const i32 L = valid ? Le : 0;
            const i32 w = valid ? we : 0;
            wi += w;
            const i32 tot = wave_sum(L);
            visits += (u64)L;
            gains_chunk(tot / max(nb, 1), nb, lane, ps, nparts, partf, r0, L, w, saving, bins, tt);
        }
        saving = wave_sum(saving);
        wi = wave_sum(wi);
        wave_sync();  // the wave's bin updates are visible to all its lanes
        // Only partitions with conn(n,p) > W_I(n) - saving(n) give a positive gain.
        const i64 need = wi - saving;
        i64 bg = 0, bg2 = 0;  // best move, and best move that keeps size(p) + size(n) <= Omega
        i32 bp = -1, bp2 = -1;
        auto consider = [&](i32 p) {
            const u32 v = bins[p];
            bins[p] = 0;
            if ((int)(v != 0) & (int)((i64)v > need)) {
                const i64 g = (i64)v - need;
                const int fits = (int)(nw_n + psize[p] <= omega);
                const bool t = lex_better(g, p, bg, bp);
                bg = t ? g : bg;
                bp = t ? p : bp;
                const bool t2 = (fits & (int)lex_better(g, p, bg2, bp2)) != 0;
                bg2 = t2 ? g : bg2;
                bp2 = t2 ? p : bp2;
            }
        };
        for (int wd = lane; wd < nwords; wd += kWave) {
            u32 bits = t_bits[wv][wd];
            if (bits) t_bits[wv][wd] = 0;
            while (bits) {
                const int bt = __builtin_ctz(bits);
                bits &= bits - 1u;
                consider(wd * 32 + bt);
            }
        }
        wave_sync();  // bins and bits cleared before the next node's updates
        wave_lexmax_i64(bg, bp);
        wave_lexmax_i64(bg2, bp2);
        if (lane == 0) {
            move_dst[n] = bp;
            move_gain[n] = bp >= 0 ? bg : 0;
            move_dst_sa[n] = bp2;
            move_gain_sa[n] = bp2 >= 0 ? bg2 : 0;
        }
    }
    // per-lane counts: one reduction per wave, one device atomic per wave
    const i64 vis = work != nullptr ? wave_sum((i64)visits) : 0;
    if ((work != nullptr) & (lane == 0) & (vis != 0)) atomicAdd(work, (unsigned long long)vis);
}

// Lists once each h-edge incident to the nodes nodes[0..cnt); emark[e] takes
// `stamp` and the lane that changed it appends e (order immaterial).  Each
// wave takes a window of listed nodes, one per lane, and walks the window's
// incidence entries as one flat range, kMarkU * 64 at a time: a lane finds
// the node of its entry by a binary search over the window's degree sums, so
// every lane has an entry whatever the degrees, and the loads and exchanges
// of kMarkU entries per lane are in flight together.  Appends gather in a
// per-wave buffer in shared memory and go out kMarkBuf - 64 or more at a
// time, one atomic on the shared list count per batch: one per 64 entries
// put the whole device's waves in line on that one address.
constexpr u32 kMarkBuf = 512;
constexpr int kMarkU = 4;

__global__ __launch_bounds__(256) void k_mark_edges(i32 cnt, const i32* __restrict__ nodes,
                                                    const i64* __restrict__ inc_off, const i32* __restrict__ inc,
                                                    u32* emark, u32 stamp, i32* elist, u32* ecount) {
    __shared__ i32 buf[4][kMarkBuf];
    const int lane = lane_id();
    const int wpb = blockDim.x / kWave;
    i32* wb = buf[wave_id()];
    const u64 lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
    u32 nb = 0;  // buffered entries (wave-uniform)
    auto flush = [&]() {
        u32 base = 0;
        if (lane == 0) base = atomicAdd(ecount, nb);
        base = (u32)__shfl((int)base, 0, kWave);
        wave_sync();  // the buffer's writes are visible to every lane
        for (u32 i = lane; i < nb; i += kWave) elist[base + i] = wb[i];
        wave_sync();  // read out before it is refilled
        nb = 0;
    };
    const i64 nwv = (i64)gridDim.x * wpb, win = wave_window(cnt, nwv);
    for (i64 base = ((i64)blockIdx.x * wpb + wave_id()) * win; base < cnt; base += nwv * win) {
        const i64 j = base + lane;
        const int in = (int)(lane < win) & (int)(j < cnt);
        const i32 n = nodes[in ? j : base];
        const i64 a = inc_off[n];
        const i64 d = in ? inc_off[n + 1] - a : 0;
        const i64 incl = wave_incl_scan(d);
        const i64 start = incl - d;
        const i64 tot = bcast((long long)incl, kWave - 1);
        for (i64 f0 = 0; f0 < tot; f0 += kMarkU * kWave) {
            i32 e[kMarkU];
#pragma unroll
            for (int u = 0; u < kMarkU; ++u) {
                const i64 f = f0 + u * kWave + lane;
                int o = 0;  // the last lane whose range starts at or before f
#pragma unroll
                for (int step = kWave / 2; step >= 1; step >>= 1) {
                    const int cand = o + step;
                    const i64 sc = __shfl(start, cand, kWave);
                    o = sc <= f ? cand : o;
                }
                const i64 ao = __shfl(a, o, kWave), so = __shfl(start, o, kWave);
                const int ok = (int)(f < tot);
                const i32 x = inc[ok ? ao + (f - so) : 0];  // past the end: entry 0, dropped
                e[u] = ok ? x : -1;
            }
            u32 old[kMarkU];
#pragma unroll
            for (int u = 0; u < kMarkU; ++u) old[u] = e[u] >= 0 ? atomicExch(&emark[e[u]], stamp) : stamp;
#pragma unroll
            for (int u = 0; u < kMarkU; ++u) {
                const int first = (int)(old[u] != stamp);
                const u64 bal = __ballot(first);
                if (first) wb[nb + (u32)__popcll(bal & lt_mask)] = e[u];
                nb += (u32)__popcll(bal);
                if (nb > kMarkBuf - kWave) flush();
            }
        }
    }
    if (nb > 0) flush();
}

__global__ void k_move_flags(i32 N, const i32* __restrict__ move_dst, i32* flag) {
    for (i64 n = (i64)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (i64)gridDim.x * blockDim.x)
        flag[n] = move_dst[n] >= 0 ? 1 : 0;
}

// Sort key (p_s asc, gain desc) (Sec. VI-C); nodes enter in id order and the
// sort is stable, so ties keep ascending node ids.  Gains are below 2^31.
__global__ void k_move_keys(i32 N, const i32* __restrict__ flag, const i32* __restrict__ pos,
                            const i32* __restrict__ rho, const i64* __restrict__ gain, u64* keys, i32* vals) {
    for (i64 n = (i64)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (i64)gridDim.x * blockDim.x)
        if (flag[n]) {
            keys[pos[n]] = ((u64)(u32)rho[n] << 32) | (u64)(0x7FFFFFFFll - gain[n]);
            vals[pos[n]] = (i32)n;
        }
}

__global__ void k_sorted_attrs(i32 M, const i32* __restrict__ snode, const i32* __restrict__ rho,
                               const i32* __restrict__ move_dst, const i64* __restrict__ gain,
                               const i32* __restrict__ nw, const i32* __restrict__ nin, i32* sps, i32* spd, i64* sg,
                               i32* snw, i32* snin, i32* sidx) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (i64)gridDim.x * blockDim.x) {
        const i32 n = snode[i];
        sps[i] = rho[n];
        spd[i] = move_dst[n];
        sg[i] = gain[n];
        snw[i] = nw[n];
        snin[i] = nin[n];
        sidx[n] = (i32)i;
    }
}

// Segment [seg_b[p], seg_e[p]) of moves leaving partition p.
__global__ void k_segments(i32 M, const i32* __restrict__ sps, i32* seg_b, i32* seg_e) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (i64)gridDim.x * blockDim.x) {
        const i32 p = sps[i];
        const i32 prev = sps[i > 0 ? i - 1 : 0], next = sps[i + 1 < M ? i + 1 : M - 1];
        if ((int)(i == 0) | (int)(prev != p)) seg_b[p] = (i32)i;
        if ((int)(i == M - 1) | (int)(next != p)) seg_e[p] = (i32)(i + 1);
    }
}

// ---- chain rounds (Sec. VI-C) ----------------------------------------------
// Per-element steps of one synchronous chain round; the multi-block kernels
// below and the single-workgroup k_chain_rounds run the same functions.
__device__ __forceinline__ void predless_elem(i64 i, const i32* __restrict__ pred, i32* pl) {
    pl[i] = pred[i] < 0 ? 1 : 0;
}

__device__ __forceinline__ void compact_elem(i64 i, const i32* __restrict__ pl, const i32* __restrict__ pls, i32* cl,
                                             u64* accG, i32* accN) {
    if (pl[i]) cl[pls[i]] = (i32)i;
    accG[i] = 0;
    accN[i] = -1;
}

// Every move without a successor grades the first kWindow moves without a
// predecessor that leave its destination, and proposes the lexicographic max
// of (grade, node id).  One wave per move.
__device__ __forceinline__ void propose_wave(i64 i, int lane, const i32* __restrict__ succ,
                                             const i32* __restrict__ spd, const i32* __restrict__ seg_b,
                                             const i32* __restrict__ seg_e, const i32* __restrict__ pls,
                                             const i32* __restrict__ cl, const i64* __restrict__ sg,
                                             const i32* __restrict__ snw, const i32* __restrict__ snin,
                                             const i32* __restrict__ snode, i32* prop, i64* propG) {
    if (succ[i] >= 0) {
        if (lane == 0) prop[i] = -1;
        return;
    }
    const i32 p = spd[i];
    const i32 b = seg_b[p], e = seg_e[p];
    i64 bG = 0;
    i32 bn = -1, bj = -1;
    if (b < e) {
        const i32 w0 = pls[b];
        const i32 w1 = min(pls[e], w0 + kWindow);
        const i64 nw_i = snw[i], nin_i = snin[i];
        for (i32 k = w0 + lane; k < w1; k += kWave) {
            const i32 j = cl[k];
            const i64 ds = nw_i - snw[j], dn = nin_i - snin[j];
            const i64 G = sg[j] * kGradeScale - (10 * (ds < 0 ? -ds : ds) + (dn < 0 ? -dn : dn));
            const i32 nj = snode[j];
            const bool t = lex_better(G, nj, bG, bn);
            bG = t ? G : bG;
            bn = t ? nj : bn;
            bj = t ? j : bj;
        }
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const i64 G2 = __shfl_xor(bG, o, kWave);
        const i32 n2 = __shfl_xor(bn, o, kWave);
        const i32 j2 = __shfl_xor(bj, o, kWave);
        const bool t = lex_better(G2, n2, bG, bn);
        bG = t ? G2 : bG;
        bn = t ? n2 : bn;
        bj = t ? j2 : bj;
    }
    if (lane == 0) {
        prop[i] = bj;
        propG[i] = bG;
    }
}

// A successor accepts the lexicographic max of (grade, proposer node id).
__device__ __forceinline__ void accept_a_elem(i64 i, const i32* __restrict__ prop, const i64* __restrict__ propG,
                                              u64* accG) {
    const i32 j = prop[i];
    if (j >= 0) atomicMax((unsigned long long*)&accG[j], (unsigned long long)enc_i64(propG[i]));
}

__device__ __forceinline__ void accept_b_elem(i64 i, const i32* __restrict__ prop, const i64* __restrict__ propG,
                                              const u64* __restrict__ accG, const i32* __restrict__ snode,
                                              i32* accN) {
    const i32 j = prop[i];
    const u64 aj = load_l2(&accG[j >= 0 ? j : 0]);
    if ((int)(j >= 0) & (int)(enc_i64(propG[i]) == aj)) atomicMax(&accN[j], snode[i]);
}

__device__ __forceinline__ int link_elem(i64 i, const i32* __restrict__ prop, const i64* __restrict__ propG,
                                         const u64* __restrict__ accG, const i32* __restrict__ accN,
                                         const i32* __restrict__ snode, i32* pred, i32* succ) {
    const i32 j = prop[i];
    const i32 jj = j >= 0 ? j : 0;
    const u64 aj = load_l2(&accG[jj]);
    const i32 nj = load_l2(&accN[jj]);
    const int ok = (int)(j >= 0) & (int)(enc_i64(propG[i]) == aj) & (int)(nj == snode[i]);
    if (ok) {
        succ[i] = j;
        pred[j] = (i32)i;
    }
    return ok;
}

#define HGP_GRID_LOOP(i, n) for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (i64)gridDim.x * blockDim.x)

// The first step of a device-wide chain round in one look-back scan: the
// moves without a predecessor are flagged (as predless_elem does), their flags
// scanned into pls (with pls[M] their count), listed in cl in move order and
// the round's accumulators reset (as compact_elem does), in one launch.
__global__ __launch_bounds__(kLbBlock) void k_predless_compact(i32 M, const unsigned long long* __restrict__ rs,
                                                                const i32* __restrict__ pred, i32* pls, i32* cl,
                                                                u64* accG, i32* accN, ScanState st, u64 tag,
                                                                u64 ticket0, i64 tiles) {
    lookback_scan_tile(
        M, st, tag, ticket0, tiles, rs[0] != 0, [&](i64 i) { return (i64)(pred[i] < 0); },
        [&](i64 i, i64 prefix, i64 flag) {
            pls[i] = (i32)prefix;
            if (flag) cl[prefix] = (i32)i;
            accG[i] = 0;
            accN[i] = -1;
        },
        [&](i64 sum) { pls[M] = (i32)sum; });
}

__global__ __launch_bounds__(256) void k_chain_propose(i32 M, const unsigned long long* __restrict__ rs,
                                                       const i32* __restrict__ succ, const i32* __restrict__ spd,
                                                       const i32* __restrict__ seg_b, const i32* __restrict__ seg_e,
                                                       const i32* __restrict__ pls, const i32* __restrict__ cl,
                                                       const i64* __restrict__ sg, const i32* __restrict__ snw,
                                                       const i32* __restrict__ snin, const i32* __restrict__ snode,
                                                       i32* prop, i64* propG) {
    if (!rs[0]) return;
    const int wpb = blockDim.x / kWave;
    for (i64 i = (i64)blockIdx.x * wpb + wave_id(); i < M; i += (i64)gridDim.x * wpb)
        propose_wave(i, lane_id(), succ, spd, seg_b, seg_e, pls, cl, sg, snw, snin, snode, prop, propG);
}

__global__ void k_chain_accept_a(i32 M, const unsigned long long* __restrict__ rs, const i32* __restrict__ prop,
                                 const i64* __restrict__ propG, u64* accG) {
    if (!rs[0]) return;
    HGP_GRID_LOOP(i, M) accept_a_elem(i, prop, propG, accG);
}

__global__ void k_chain_accept_b(i32 M, const unsigned long long* __restrict__ rs, const i32* __restrict__ prop,
                                 const i64* __restrict__ propG, const u64* __restrict__ accG,
                                 const i32* __restrict__ snode, i32* accN) {
    if (!rs[0]) return;
    HGP_GRID_LOOP(i, M) accept_b_elem(i, prop, propG, accG, snode, accN);
}

__global__ void k_chain_link(i32 M, unsigned long long* rs, const i32* __restrict__ prop,
                             const i64* __restrict__ propG, const u64* __restrict__ accG,
                             const i32* __restrict__ accN, const i32* __restrict__ snode, i32* pred, i32* succ) {
    if (!rs[0]) return;
    unsigned long long c = 0;
    HGP_GRID_LOOP(i, M) c += (unsigned long long)link_elem(i, prop, propG, accG, accN, snode, pred, succ);
    c = wave_sum(c);
    if (lane_id() == 0 && c) atomicAdd(&rs[1], c);
}

__global__ void k_set_flag(unsigned long long* rs) { rs[0] = 1; }

__global__ void k_round_end(unsigned long long* rs) {
    if (!rs[0]) return;
    if (rs[1] == 0) rs[0] = 0;
    rs[2] += rs[1];
    rs[1] = 0;
}

// Largest move count of k_chain_compact1 / k_chain_tail1.  One workgroup
// takes about 2 us per 1,000 moves per round; the device-wide round (eight
// launches) about 50 us, so larger move sets take the device-wide kernels.
constexpr i64 kChainCompactMax = 1 << 14;

// First step of a chain round for at most kChainCompactMax moves, in one
// workgroup: fold the previous round's links into the totals (the
// k_round_end step; a round that linked nothing ends the rounds), then the
// moves without a predecessor, their exclusive scan and compaction, and the
// reset of the acceptance accumulators.  Replaces three launches per round.
__global__ __launch_bounds__(1024) void k_chain_compact1(i32 M, int round, unsigned long long* rs,
                                                         const i32* __restrict__ pred, i32* pls, i32* cl, u64* accG,
                                                         i32* accN) {
    __shared__ i32 red[16];
    __shared__ int active;
    if (threadIdx.x == 0) {
        unsigned long long a = rs[0];
        if (a && round > 0) {
            if (rs[1] == 0) a = 0;
            rs[2] += rs[1];
            rs[1] = 0;
            rs[0] = a;
        }
        active = (int)(a != 0);
    }
    __syncthreads();
    if (!active) return;
    i32 carry = 0;
    for (i64 base = 0; base < M; base += blockDim.x) {
        const i64 i = base + threadIdx.x;
        const i32 v = i < M ? (pred[i] < 0 ? 1 : 0) : 0;
        i32 tot;
        const i32 ex = block_excl_scan(v, red, &tot);
        if (i < M) {
            pls[i] = carry + ex;
            if (v) cl[carry + ex] = (i32)i;
            accG[i] = 0;
            accN[i] = -1;
        }
        carry += tot;
    }
    if (threadIdx.x == 0) pls[M] = carry;
}

// The rest of a chain round after the proposals, in one workgroup (up to
// kChainCompactMax moves): acceptance (both phases), links and their count
// folded into the totals (a round that links nothing ends the rounds), and,
// when another round follows, its moves without a predecessor, their scan and
// compaction and the reset of the accumulators.  Replaces four launches per
// round.
__global__ __launch_bounds__(1024) void k_chain_tail1(i32 M, int next, unsigned long long* rs, i32* pred, i32* succ,
                                                      i32* pls, i32* cl, u64* accG, i32* accN,
                                                      const i32* __restrict__ snode, const i32* __restrict__ prop,
                                                      const i64* __restrict__ propG) {
    __shared__ i32 red[16];
    __shared__ unsigned long long red_l[16];
    __shared__ int active;
    if (threadIdx.x == 0) active = (int)(rs[0] != 0);
    __syncthreads();
    if (!active) return;
    for (i64 i = threadIdx.x; i < M; i += blockDim.x) accept_a_elem(i, prop, propG, accG);
    __syncthreads();
    for (i64 i = threadIdx.x; i < M; i += blockDim.x) accept_b_elem(i, prop, propG, accG, snode, accN);
    __syncthreads();
    unsigned long long lk = 0;
    for (i64 i = threadIdx.x; i < M; i += blockDim.x)
        lk += (unsigned long long)link_elem(i, prop, propG, accG, accN, snode, pred, succ);
    lk = block_sum(lk, red_l);  // ends with a barrier
    if (threadIdx.x == 0) {
        rs[2] += lk;
        rs[1] = 0;
        if (lk == 0) rs[0] = 0;
    }
    if ((lk == 0) | !next) return;
    i32 carry = 0;
    for (i64 base = 0; base < M; base += blockDim.x) {
        const i64 i = base + threadIdx.x;
        const i32 v = i < M ? (pred[i] < 0 ? 1 : 0) : 0;
        i32 tot;
        const i32 ex = block_excl_scan(v, red, &tot);
        if (i < M) {
            pls[i] = carry + ex;
            if (v) cl[carry + ex] = (i32)i;
            accG[i] = 0;
            accN[i] = -1;
        }
        carry += tot;
    }
    if (threadIdx.x == 0) pls[M] = carry;
}

// All chain rounds in one workgroup, for move counts so small that per-round
// launches and host checks would dominate (beyond a few hundred moves the
// windowed proposals, one wave per move, need the whole GPU).  Same steps,
// separated by block barriers; stops after the first round that links
// nothing, and adds the links to rs[2].
constexpr int kChainSingleMax = 256;

__global__ __launch_bounds__(1024) void k_chain_rounds(
    i32 M, unsigned long long* rs, i32* pred, i32* succ, i32* pl, i32* pls, i32* cl, u64* accG, i32* accN,
    const i32* __restrict__ spd, const i32* __restrict__ seg_b, const i32* __restrict__ seg_e,
    const i64* __restrict__ sg, const i32* __restrict__ snw, const i32* __restrict__ snin,
    const i32* __restrict__ snode, i32* prop, i64* propG) {
    __shared__ i32 red[16];
    __shared__ unsigned long long red_l[16];
    const int nwv = blockDim.x / kWave;
    unsigned long long total = 0;
    for (int round = 0; round < kChainRounds; ++round) {
        for (i64 i = threadIdx.x; i < M; i += blockDim.x) predless_elem(i, pred, pl);
        __syncthreads();
        // exclusive scan of pl into pls (kScanItems-free: one pass per 1024 entries)
        i32 carry = 0;
        for (i64 base = 0; base < M; base += blockDim.x) {
            const i64 i = base + threadIdx.x;
            const i32 v = i < M ? pl[i] : 0;
            i32 tot;
            const i32 ex = block_excl_scan(v, red, &tot);
            if (i < M) pls[i] = carry + ex;
            carry += tot;
        }
        if (threadIdx.x == 0) pls[M] = carry;
        __syncthreads();
        for (i64 i = threadIdx.x; i < M; i += blockDim.x) compact_elem(i, pl, pls, cl, accG, accN);
        __syncthreads();
        for (i64 i = wave_id(); i < M; i += nwv)
            propose_wave(i, lane_id(), succ, spd, seg_b, seg_e, pls, cl, sg, snw, snin, snode, prop, propG);
        __syncthreads();
        for (i64 i = threadIdx.x; i < M; i += blockDim.x) accept_a_elem(i, prop, propG, accG);
        __syncthreads();
        for (i64 i = threadIdx.x; i < M; i += blockDim.x) accept_b_elem(i, prop, propG, accG, snode, accN);
        __syncthreads();
        unsigned long long c = 0;
        for (i64 i = threadIdx.x; i < M; i += blockDim.x)
            c += (unsigned long long)link_elem(i, prop, propG, accG, accN, snode, pred, succ);
        c = block_sum(c, red_l);  // ends with a barrier
        total += c;
        if (c == 0) break;
    }
    if (threadIdx.x == 0) {
        rs[2] += total;
        rs[0] = 0;
    }
}

// ---- chain extraction and ranking (Sec. VI-C) -------------------------------
__global__ void k_cyc_init(i32 M, const i32* __restrict__ succ, const i32* __restrict__ snode, i32* J, i32* MN) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (i64)gridDim.x * blockDim.x) {
        J[i] = succ[i];
        MN[i] = snode[i];
    }
}

// Pointer doubling along successors: after enough steps a node on a cycle
// still points somewhere and holds the smallest node id of its cycle.
__device__ __forceinline__ void cyc_elem(i64 i, const i32* __restrict__ J, const i32* __restrict__ MN, i32* J2,
                                         i32* MN2) {
    const i32 j = J[i];
    if (j >= 0) {
        MN2[i] = min(MN[i], MN[j]);
        J2[i] = J[j];
    } else {
        MN2[i] = MN[i];
        J2[i] = j;
    }
}

__global__ void k_cyc_step(i32 M, const i32* __restrict__ J, const i32* __restrict__ MN, i32* J2, i32* MN2) {
    HGP_GRID_LOOP(i, M) cyc_elem(i, J, MN, J2, MN2);
}

// K doubling steps in one workgroup (small M); buffers alternate as in K
// launches of k_cyc_step, so the result lands where the host expects it.
constexpr int kJumpSingleMax = 16384;

__global__ __launch_bounds__(1024) void k_cyc_steps(i32 M, int K, i32* J, i32* MN, i32* J2, i32* MN2) {
    for (int it = 0; it < K; ++it) {
        for (i64 i = threadIdx.x; i < M; i += blockDim.x) cyc_elem(i, J, MN, J2, MN2);
        __syncthreads();
        i32* t = J;
        J = J2;
        J2 = t;
        t = MN;
        MN = MN2;
        MN2 = t;
    }
}

// Chain heads: path heads, and the smallest node of every cycle.
__global__ void k_heads(i32 M, const i32* __restrict__ J, const i32* __restrict__ MN, const i32* __restrict__ pred,
                        const i32* __restrict__ snode, i32* P, i32* R, i32* H, i32* head) {
    // Branch-free on purpose: every operand is loaded unconditionally and the
    // condition combined with bitwise operators, so the head test and the four
    // selects below share one predicate (a short-circuit form of this test was
    // lowered by the device compiler into code that dropped the select for H).
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (i64)gridDim.x * blockDim.x) {
        const i32 pr = pred[i], j = J[i], sn = snode[i], mn = MN[i];
        const int h = (int)(pr < 0) | ((int)(j >= 0) & (int)(sn == mn));
        head[i] = h;
        P[i] = h ? -1 : pr;
        R[i] = h ? 0 : 1;
        H[i] = h ? (i32)i : pr;
    }
}

// List ranking: distance to the chain head and the head itself.
__device__ __forceinline__ void rank_elem(i64 i, const i32* __restrict__ P, const i32* __restrict__ R,
                                          const i32* __restrict__ H, i32* P2, i32* R2, i32* H2) {
    const i32 p = P[i];
    if (p >= 0) {
        R2[i] = R[i] + R[p];
        H2[i] = H[p];
        P2[i] = P[p];
    } else {
        R2[i] = R[i];
        H2[i] = H[i];
        P2[i] = p;
    }
}

__global__ void k_rank_step(i32 M, const i32* __restrict__ P, const i32* __restrict__ R, const i32* __restrict__ H,
                            i32* P2, i32* R2, i32* H2) {
    HGP_GRID_LOOP(i, M) rank_elem(i, P, R, H, P2, R2, H2);
}

__global__ __launch_bounds__(1024) void k_rank_steps(i32 M, int K, i32* P, i32* R, i32* H, i32* P2, i32* R2,
                                                     i32* H2) {
    for (int it = 0; it < K; ++it) {
        for (i64 i = threadIdx.x; i < M; i += blockDim.x) rank_elem(i, P, R, H, P2, R2, H2);
        __syncthreads();
        i32* t = P;
        P = P2;
        P2 = t;
        t = R;
        R = R2;
        R2 = t;
        t = H;
        H = H2;
        H2 = t;
    }
}

__global__ void k_chain_accum(i32 M, const i32* __restrict__ H, const i64* __restrict__ sg, i64* cg, i32* clen) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (i64)gridDim.x * blockDim.x) {
        atomicAdd((unsigned long long*)&cg[H[i]], (unsigned long long)sg[i]);
        atomicAdd(&clen[H[i]], 1);
    }
}

// Heads listed in node-id order (so a stable sort by gain breaks ties by the
// first node's id).
__global__ void k_head_flags(i32 N, const i32* __restrict__ sidx, const i32* __restrict__ head, i32* hf) {
    for (i64 n = (i64)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (i64)gridDim.x * blockDim.x) {
        const i32 i = sidx[n];
        const i32 hd = head[i >= 0 ? i : 0];
        hf[n] = ((int)(i >= 0) & (int)(hd != 0)) ? 1 : 0;
    }
}

__global__ void k_head_keys(i32 N, const i32* __restrict__ hf, const i32* __restrict__ hpos,
                            const i32* __restrict__ sidx, const i64* __restrict__ cg, u64* keys, i32* vals) {
    for (i64 n = (i64)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (i64)gridDim.x * blockDim.x)
        if (hf[n]) {
            const i32 i = sidx[n];
            keys[hpos[n]] = (u64)(0x3FFFFFFFFFFFFFFFll - cg[i]);
            vals[hpos[n]] = i;
        }
}

__global__ void k_ranked_len(i32 C, const i32* __restrict__ rh, const i32* __restrict__ clen, i32* lr) {
    for (i64 c = (i64)blockIdx.x * blockDim.x + threadIdx.x; c < C; c += (i64)gridDim.x * blockDim.x)
        lr[c] = clen[rh[c]];
}

__global__ void k_chain_start(i32 C, const i32* __restrict__ rh, const i32* __restrict__ lrs, i32* cstart) {
    for (i64 c = (i64)blockIdx.x * blockDim.x + threadIdx.x; c < C; c += (i64)gridDim.x * blockDim.x)
        cstart[rh[c]] = lrs[c];
}

__global__ void k_positions(i32 M, const i32* __restrict__ H, const i32* __restrict__ R,
                            const i32* __restrict__ cstart, const i32* __restrict__ snode, const i32* __restrict__ sps,
                            const i32* __restrict__ spd, i32* seqn, i32* seqs, i32* seqd, i32* posn) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (i64)gridDim.x * blockDim.x) {
        const i32 h = H[i];
        const int hok = (int)(h >= 0) & (int)(h < M);
        const i32 cs = cstart[hok ? h : 0];
        const i32 q = hok ? cs + R[i] : -1;
        if ((int)(q < 0) | (int)(q >= M)) continue;  // unreachable when the chain links are consistent
        seqn[q] = snode[i];
        seqs[q] = sps[i];
        seqd[q] = spd[i];
        posn[snode[i]] = q;
    }
}


// In-sequence gains (Sec. VI-C), h-edge side.  One wave per h-edge: the
// h-edge's pins(p,e) rows are staged in shared memory and its movers gathered
// with their sequence positions.  For each mover, the counts of its source and
// destination parts in e just before it moves are the row counts plus the
// moves of e's earlier movers into and out of those parts.  From them follow
// the mover's gain on e, w(e) * ([pins(p_s) = 1] - [pins(p_d) = 0]), and (for a
// destination pin) whether p_s loses e from its inbound set and p_d gains it.
// The outcome is one byte at the mover's pin slot:
//   bit 0: pins(p_s, e) = 1,  bit 1: pins(p_d, e) = 0,
//   bit 2: p_s loses e from D, bit 3: p_d gains e in D.
// The per-mover sums run in k_inseq_movers, so no atomics are needed.
struct MoverRec {
    i32 q, ps, pd, slot;  // slot = (pin offset in e) << 1 | destination flag
};
constexpr int kInseqListMax = 256;  // largest h-edge of the event-list kernel
constexpr int kInseqGroup = 64;     // largest h-edge of its 16-lane groups
constexpr int kInseqU = 4;          // row entries / pins per lane loaded together

__device__ __forceinline__ i32 lds_row(const i32* __restrict__ rp, const u32* __restrict__ rc, i32 L, i32 p,
                                       i32& ci) {
    i32 lo = 0, hi = L;
    while (lo < hi) {
        const i32 mid = (lo + hi) >> 1;
        const int lt = (int)(rp[mid] < p);
        lo = lt ? mid + 1 : lo;
        hi = lt ? hi : mid;
    }
    const i32 at = lo < L ? lo : L - 1;
    const int hit = (int)(lo < L) & (int)(rp[at] == p);
    const u32 v = rc[at];
    ci = hit ? (i32)(v >> 16) : 0;
    return hit ? (i32)(v & 0xFFFFu) : 0;
}

// Algorithmic bytes of one h-edge's in-sequence pass: offsets, |src| and
// lambda (20), its pins and their sequence positions (8 per pin), its row (12
// per entry), and per mover its two partitions read and its outcome byte
// written (9).
__device__ __forceinline__ u64 inseq_edge_bytes(i64 card, i32 rows, int movers) {
    return 20 + 8 * (u64)card + 12 * (u64)rows + 9 * (u64)movers;
}

// All pairs of movers: for h-edges larger than the event-list kernel below
// takes (skip_le is the largest card it handles; those are skipped here).
__global__ __launch_bounds__(64) void k_inseq_edges(
    i32 E, i32 M, const i64* __restrict__ he_off, const i32* __restrict__ he_nsrc, const i32* __restrict__ pins,
    const i32* __restrict__ posn, const i32* __restrict__ rho, const i32* __restrict__ move_dst,
    const i32* __restrict__ part, const i32* __restrict__ cnt, const i32* __restrict__ cin,
    const i32* __restrict__ len, unsigned char* code, int cap, i32 skip_le, const i32* __restrict__ elist,
    const u32* __restrict__ ecount, unsigned long long* bytes) {
    // shared memory: cap movers, then cap row parts and cap packed row counts
    extern __shared__ __align__(16) unsigned char smem_raw[];
    MoverRec* mv = (MoverRec*)smem_raw;
    i32* rp = (i32*)(mv + cap);
    u32* rc = (u32*)(rp + cap);
    const int lane = threadIdx.x;
    const u64 lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
    u64 acc = 0;
    const i64 ne = elist ? (i64)*ecount : (i64)E;
    const i64 win = wave_window(ne, gridDim.x);
    // h-edges a window of list entries at a time; those of more than skip_le
    // pins are kept by ballot and handled one after another
    for (i64 base = (i64)blockIdx.x * win; base < ne; base += (i64)gridDim.x * win) {
      const i64 il = base + lane;
      const int in = (int)(lane < win) & (int)(il < ne);
      const i64 el = in ? (elist ? (i64)elist[il] : il) : 0;
      const i64 al = he_off[el], bl = he_off[el + 1];
      const i32 nsl = he_nsrc[el], Ll = len[el];
      u64 todo = __ballot(in & (int)(bl - al > (i64)skip_le));
      while (todo) {
        const int src = __builtin_ctzll(todo);
        todo &= todo - 1;
        const i64 a = __shfl(al, src, kWave), b = __shfl(bl, src, kWave);
        const i64 d0 = a + __shfl(nsl, src, kWave);
        const i32 L = __shfl(Ll, src, kWave);
        for (i32 r = lane; r < L; r += kWave) {
            rp[r] = part[a + r];
            rc[r] = (u32)cnt[a + r] | ((u32)cin[a + r] << 16);  // both <= |e| <= 4096
        }
        int k = 0;
        for (i64 base = a; base < b; base += kWave) {
            const i64 j = base + lane;
            const int inb = (int)(j < b);
            const i32 m = pins[inb ? j : a];
            const i32 q = posn[m];
            const int is_mv = inb & (int)(q < M);
            const u64 mask = __ballot(is_mv);
            if (is_mv) {
                MoverRec r;
                r.q = q;
                r.ps = rho[m];
                r.pd = move_dst[m];
                r.slot = (i32)((j - a) << 1) | (i32)(j >= d0);
                mv[k + __popcll(mask & lt_mask)] = r;
            }
            k += __popcll(mask);
        }
        __syncthreads();
        for (int i = lane; i < k; i += kWave) {
            const MoverRec me = mv[i];
            i32 xs = 0, xd = 0, xis = 0, xid = 0;
            for (int jj = 0; jj < k; ++jj) {
                const MoverRec o = mv[jj];
                const i32 before = (i32)(o.q < me.q);
                const i32 dj = o.slot & 1;
                const i32 es = before * ((i32)(o.pd == me.ps) - (i32)(o.ps == me.ps));
                const i32 ed = before * ((i32)(o.pd == me.pd) - (i32)(o.ps == me.pd));
                xs += es;
                xd += ed;
                xis += dj * es;
                xid += dj * ed;
            }
            i32 cis, cid;
            const i32 cs = lds_row(rp, rc, L, me.ps, cis) + xs;
            const i32 cd = lds_row(rp, rc, L, me.pd, cid) + xd;
            const i32 di = me.slot & 1;
            const u32 bits = (u32)(cs == 1) | ((u32)(cd == 0) << 1) | ((u32)(di & (int)(cis + xis == 1)) << 2) |
                             ((u32)(di & (int)(cid + xid == 0)) << 3);
            code[a + (me.slot >> 1)] = (unsigned char)bits;
        }
        acc += inseq_edge_bytes(b - a, L, k);
        __syncthreads();
      }
    }
    if ((bytes != nullptr) & (lane == 0) & (acc != 0)) atomicAdd(bytes, (unsigned long long)acc);
}

// Same outcome bytes with per-part event lists instead of all pairs.  The
// movers' source and destination parts go into a hash table in shared memory;
// each mover pushes a leave event (q, -1) on its source part's list and an
// enter event (q, +1) on its destination part's list.  A mover's count of a
// part just before it moves is the part's row count plus the events of that
// part's list with an earlier sequence position.  Lists are as long as the
// number of movers touching a part, usually a few, so a mover reads a few
// events where the all-pairs kernel compares it with every mover of e.
// For h-edges of at most cap pins; T = 2^tbits >= 2 * cap table slots.  The
// table also carries e's row counts, so no search of the row is needed.
__device__ __forceinline__ i32 part_slot(i32* tkey, int tbits, i32 p, int& inserted) {
    const u32 tmask = (1u << tbits) - 1u;
    u32 h = ((u32)p * 0x9E3779B1u) >> (32 - tbits);
    inserted = 0;
    for (u32 probe = 0; probe <= tmask; ++probe) {
        const i32 k = tkey[h];
        if (k == p) return (i32)h;
        if (k == -1) {
            const i32 prev = atomicCAS(&tkey[h], -1, p);
            if (prev == -1) {
                inserted = 1;
                return (i32)h;
            }
            if (prev == p) return (i32)h;
        }
        h = (h + 1u) & tmask;
    }
    return -1;  // unreachable: the table has a slot for every part of 2 * cap movers
}

// Shared memory of a lane group (GW lanes, one h-edge at a time): per mover
// its sequence position, node and packed (source slot | destination slot << 10
// | pin slot << 20 | destination pin << 30); per row entry its table slot; the
// table (keys, list heads, packed row counts); one 32-bit link per event:
// ((next event + 1) << 1) | destination-pin flag, where event 2i leaves mover
// i's source part and 2i + 1 enters its destination part.  24 bytes per mover
// slot and 12 per table slot.
//
// A wave takes its h-edges a window of list entries at a time (up to 64, fewer
// when the list is short for the grid), reading their offsets,
// source counts and row lengths one per lane and keeping (by ballot) those of
// more than `lo` and at most cap pins; its 64 / GW lane groups then handle
// them GW at a time, each group its own h-edge with its own shared memory.
// Every global load of an h-edge is issued unconditionally (out-of-range lanes
// read entry 0 of the same h-edge, an idle group the first pin slot), so each
// dependent step (row and pins, positions, the movers' partitions) is one
// round trip.  The table is cleared once; each h-edge resets the slots it
// used.  One wave per block, so wave-level fences order shared memory.
template <int GW>
__global__ __launch_bounds__(64) void k_inseq_lists(
    i32 E, i32 M, const i64* __restrict__ he_off, const i32* __restrict__ he_nsrc, const i32* __restrict__ pins,
    const i32* __restrict__ posn, const i32* __restrict__ rho, const i32* __restrict__ move_dst,
    const i32* __restrict__ part, const i32* __restrict__ cnt, const i32* __restrict__ cin,
    const i32* __restrict__ len, unsigned char* code, int cap, int tbits, int lo, const i32* __restrict__ elist,
    const u32* __restrict__ ecount, unsigned long long* bytes) {
    constexpr int NG = kWave / GW;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ i32 s_list[kWave];
    const int T = 1 << tbits;
    const int lane = threadIdx.x, g = lane / GW, gl = lane % GW;
    const u64 gmask = GW == kWave ? ~0ull : (((1ull << GW) - 1ull) << (g * GW));
    const u64 lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
    const u64 glt = lt_mask & gmask;
    i32* mq = (i32*)smem_raw + (size_t)g * (6 * cap + 3 * T);  // cap
    i32* mnode = mq + cap;                                       // cap
    u32* mpk = (u32*)(mnode + cap);                              // cap
    i32* rslot = (i32*)(mpk + cap);                              // cap
    i32* tkey = rslot + cap;                                     // T
    i32* thead = tkey + T;                                       // T
    u32* tcnt = (u32*)(thead + T);                               // T
    i32* ev = (i32*)(tcnt + T);                                  // 2 * cap
    u64 acc_bytes = 0;
    const i64 ne = elist ? (i64)*ecount : (i64)E;
    for (int t = gl; t < T; t += GW) {
        tkey[t] = -1;
        thead[t] = -1;
    }
    wave_sync();
    const i64 win = wave_window(ne, gridDim.x);
    for (i64 base = (i64)blockIdx.x * win; base < ne; base += (i64)gridDim.x * win) {
        const i64 il = base + lane;
        const int in = (int)(lane < win) & (int)(il < ne);
        const i64 el = in ? (elist ? (i64)elist[il] : il) : 0;
        const i64 al = he_off[el], bl = he_off[el + 1];
        const i32 nsl = he_nsrc[el], Ll = len[el];
        const i32 cardl = (i32)(bl - al);
        const int mine = in & (int)(cardl > lo) & (int)(cardl <= cap);
        const u64 todo = __ballot(mine);
        const int nt = __popcll(todo);
        if (mine) s_list[__popcll(todo & lt_mask)] = lane;
        wave_sync();
        for (int r0 = 0; r0 < nt; r0 += NG) {
            const int act = (int)(r0 + g < nt);
            const int src = s_list[act ? r0 + g : 0];
            // the shuffles run on every lane (a lane left out of a shuffle
            // cannot serve as another group's source), then idle groups
            // take an empty h-edge at pin slot 0
            const i64 a_s = __shfl(al, src, kWave);
            const i32 card_s = __shfl(cardl, src, kWave), ns_s = __shfl(nsl, src, kWave);
            const i32 L_s = __shfl(Ll, src, kWave);
            const i64 a = act ? a_s : 0;
            const i32 card = act ? card_s : 0;
            const i64 d0 = a + ns_s;
            const i32 L = act ? L_s : 0;
            // row entries and pins, then the pins' sequence positions
            i32 pp[kInseqU], mm[kInseqU], qq[kInseqU];
            u32 cc[kInseqU];
#pragma unroll
            for (int u = 0; u < kInseqU; ++u) {
                const i32 r = u * GW + gl;
                const i64 ri = a + (r < L ? r : 0);
                pp[u] = part[ri];
                cc[u] = (u32)cnt[ri] | ((u32)cin[ri] << 16);  // both <= |e| <= 4096
                mm[u] = pins[a + (r < card ? r : 0)];
            }
#pragma unroll
            for (int u = 0; u < kInseqU; ++u) qq[u] = posn[mm[u]];
            // e's row parts with their counts (distinct parts)
#pragma unroll
            for (int u = 0; u < kInseqU; ++u) {
                const i32 r = u * GW + gl;
                if (r < L) {
                    int ins;
                    const i32 t = part_slot(tkey, tbits, pp[u], ins);
                    tcnt[t] = cc[u];
                    rslot[r] = t;
                }
            }
            // movers, indexed by the group's ballot bits
            int k = 0;
#pragma unroll
            for (int u = 0; u < kInseqU; ++u) {
                const i32 j = u * GW + gl;
                const int is_mv = (int)(j < card) & (int)(qq[u] < M);
                const u64 mask = __ballot(is_mv) & gmask;
                if (is_mv) {
                    const i32 i = k + __popcll(mask & glt);
                    mq[i] = qq[u];
                    mnode[i] = mm[u];
                    mpk[i] = (u32)j << 20 | ((u32)(a + j >= d0) << 30);
                }
                k += __popcll(mask);
            }
            wave_sync();
            // the movers' partitions, one lane per mover, then their table
            // slots (a source part is in the row; a destination part may be
            // new, with no pins in e) and their two events on the parts' lists
            i32 ps[kInseqU], pd[kInseqU];
#pragma unroll
            for (int u = 0; u < kInseqU; ++u) {
                const i32 i = u * GW + gl;
                const i32 nd0 = mnode[i < k ? i : 0];
                const i32 nd = k > 0 ? nd0 : 0;  // node 0 when the group has no mover
                ps[u] = rho[nd];
                pd[u] = move_dst[nd];
            }
#pragma unroll
            for (int u = 0; u < kInseqU; ++u) {
                const i32 i = u * GW + gl;
                if (i < k) {
                    int ins_s, ins_d;
                    const i32 ts = part_slot(tkey, tbits, ps[u], ins_s);
                    const i32 td = part_slot(tkey, tbits, pd[u], ins_d);
                    if (ins_s) tcnt[ts] = 0u;  // not reached: p_s has a pin of e in the row
                    if (ins_d) tcnt[td] = 0u;
                    const u32 pk = mpk[i];
                    const i32 dj = (i32)((pk >> 30) & 1u);
                    const i32 hs = atomicExch(&thead[ts], 2 * i);
                    const i32 hd = atomicExch(&thead[td], 2 * i + 1);
                    ev[2 * i] = ((hs + 1) << 1) | dj;
                    ev[2 * i + 1] = ((hd + 1) << 1) | dj;
                    mpk[i] = pk | (u32)ts | ((u32)td << 10);
                }
            }
            wave_sync();
            for (int i = gl; i < k; i += GW) {
                const i32 q = mq[i];
                const u32 pk = mpk[i];
                const i32 ts = (i32)(pk & 1023u), td = (i32)((pk >> 10) & 1023u);
                i32 x[2], xi[2];
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    i32 sacc = 0, sacci = 0;
                    i32 idx = thead[side ? td : ts];
                    while (idx >= 0) {
                        const i32 lk = ev[idx];
                        const i32 sg = (i32)(mq[idx >> 1] < q) * ((idx & 1) ? 1 : -1);
                        sacc += sg;
                        sacci += sg * (lk & 1);
                        idx = (lk >> 1) - 1;
                    }
                    x[side] = sacc;
                    xi[side] = sacci;
                }
                const u32 c0s = tcnt[ts], c0d = tcnt[td];
                const i32 cs = (i32)(c0s & 0xFFFFu) + x[0];
                const i32 cd = (i32)(c0d & 0xFFFFu) + x[1];
                const i32 cis = (i32)(c0s >> 16) + xi[0];
                const i32 cid = (i32)(c0d >> 16) + xi[1];
                const i32 di = (i32)((pk >> 30) & 1u);
                const u32 bits = (u32)(cs == 1) | ((u32)(cd == 0) << 1) | ((u32)(di & (int)(cis == 1)) << 2) |
                                 ((u32)(di & (int)(cid == 0)) << 3);
                code[a + ((pk >> 20) & 1023u)] = (unsigned char)bits;
            }
            if ((gl == 0) & act) acc_bytes += inseq_edge_bytes(card, L, k);
            wave_sync();
            // reset the slots this h-edge used: its row parts and its movers' parts
#pragma unroll
            for (int u = 0; u < kInseqU; ++u) {
                const i32 r = u * GW + gl;
                if (r < L) {
                    tkey[rslot[r]] = -1;
                    thead[rslot[r]] = -1;
                }
            }
            for (int i = gl; i < k; i += GW) {
                const u32 pk = mpk[i];
                const i32 ts = (i32)(pk & 1023u), td = (i32)((pk >> 10) & 1023u);
                tkey[ts] = -1;
                thead[ts] = -1;
                tkey[td] = -1;
                thead[td] = -1;
            }
            wave_sync();
        }
    }
    const u64 tot = bytes != nullptr ? (u64)wave_sum((i64)acc_bytes) : 0;
    if ((bytes != nullptr) & (lane == 0) & (tot != 0)) atomicAdd(bytes, (unsigned long long)tot);
}

// The same outcome bytes for h-edges of at most kInseqSmall pins, one lane per
// h-edge, everything in registers: a mover's counts of p_s and p_d just before
// it moves are the row counts plus the moves of the h-edge's earlier movers,
// compared all pairs (at most kInseqSmall^2 per h-edge).
constexpr int kInseqSmall = 8;

__global__ __launch_bounds__(256) void k_inseq_small(
    i32 E, i32 M, const i64* __restrict__ he_off, const i32* __restrict__ he_nsrc, const i32* __restrict__ pins,
    const i32* __restrict__ posn, const i32* __restrict__ rho, const i32* __restrict__ move_dst,
    const i32* __restrict__ part, const i32* __restrict__ cnt, const i32* __restrict__ cin,
    const i32* __restrict__ len, unsigned char* code, const i32* __restrict__ elist, const u32* __restrict__ ecount,
    unsigned long long* bytes) {
    constexpr int S = kInseqSmall;
    const i64 ne = elist ? (i64)*ecount : (i64)E;
    u64 acc = 0;
    for (i64 ie = (i64)blockIdx.x * blockDim.x + threadIdx.x; ie < ne; ie += (i64)gridDim.x * blockDim.x) {
        const i64 e = elist ? (i64)elist[ie] : ie;
        const i64 a = he_off[e], b = he_off[e + 1];
        const i32 card = (i32)(b - a);
        if ((card <= 0) | (card > S)) continue;
        const i64 d0 = a + he_nsrc[e];
        const i32 L = len[e];
        i32 m[S], q[S];
#pragma unroll
        for (int j = 0; j < S; ++j) m[j] = pins[a + (j < card ? j : 0)];
#pragma unroll
        for (int j = 0; j < S; ++j) q[j] = j < card ? posn[m[j]] : 0x7FFFFFFF;
        int nmv = 0;
#pragma unroll
        for (int j = 0; j < S; ++j) nmv += (int)(q[j] < M);
        if (nmv > 0) {
            i32 ps[S], pd[S], rp[S];
            u32 rc[S];
#pragma unroll
            for (int j = 0; j < S; ++j) {
                const int mv = (int)(q[j] < M);
                ps[j] = mv ? rho[m[j]] : -1;
                pd[j] = mv ? move_dst[m[j]] : -1;
            }
#pragma unroll
            for (int r = 0; r < S; ++r) {
                const i64 ri = a + (r < L ? r : 0);
                const i32 pr = part[ri];
                const u32 cr = (u32)cnt[ri] | ((u32)cin[ri] << 16);
                rp[r] = r < L ? pr : -1;
                rc[r] = r < L ? cr : 0u;
            }
#pragma unroll
            for (int j = 0; j < S; ++j) {
                if (q[j] < M) {
                    i32 xs = 0, xd = 0, xis = 0, xid = 0;
#pragma unroll
                    for (int o = 0; o < S; ++o) {
                        const i32 before = (i32)(q[o] < q[j]);
                        const i32 dj = (i32)(a + o >= d0);
                        const i32 es = before * ((i32)(pd[o] == ps[j]) - (i32)(ps[o] == ps[j]));
                        const i32 ed = before * ((i32)(pd[o] == pd[j]) - (i32)(ps[o] == pd[j]));
                        xs += es;
                        xd += ed;
                        xis += dj * es;
                        xid += dj * ed;
                    }
                    u32 c0s = 0, c0d = 0;
#pragma unroll
                    for (int r = 0; r < S; ++r) {
                        c0s = rp[r] == ps[j] ? rc[r] : c0s;
                        c0d = rp[r] == pd[j] ? rc[r] : c0d;
                    }
                    const i32 cs = (i32)(c0s & 0xFFFFu) + xs;
                    const i32 cd = (i32)(c0d & 0xFFFFu) + xd;
                    const i32 cis = (i32)(c0s >> 16) + xis;
                    const i32 cid = (i32)(c0d >> 16) + xid;
                    const i32 di = (i32)(a + j >= d0);
                    const u32 bits = (u32)(cs == 1) | ((u32)(cd == 0) << 1) | ((u32)(di & (int)(cis == 1)) << 2) |
                                     ((u32)(di & (int)(cid == 0)) << 3);
                    code[a + j] = (unsigned char)bits;
                }
            }
        }
        acc += inseq_edge_bytes(card, nmv ? L : 0, nmv);
    }
    const u64 tot = bytes != nullptr ? (u64)wave_sum((i64)acc) : 0;
    if ((bytes != nullptr) & (lane_id() == 0) & (tot != 0)) atomicAdd(bytes, (unsigned long long)tot);
}

// In-sequence gains, mover side: one wave per sequence position q sums the
// outcome bytes over the mover's incidence list.  Loads are issued for four
// entries per lane at once, out-of-range lanes reading the list's first entry;
// the next position's node is read two positions ahead and its offsets one
// ahead.
__global__ __launch_bounds__(256) void k_inseq_movers(i32 M, const i32* __restrict__ seqn,
                                                      const i64* __restrict__ inc_off, const i32* __restrict__ inc,
                                                      const i32* __restrict__ inc_pos, const i32* __restrict__ hw,
                                                      const unsigned char* __restrict__ code, i64* gseq, i32* dds,
                                                      i32* ddd, unsigned long long* bytes) {
    const int lane = lane_id();
    const int wpb = blockDim.x / kWave;
    const i64 stride = (i64)gridDim.x * wpb;
    u64 acc = 0;
    i64 q = (i64)blockIdx.x * wpb + wave_id();
    if (q >= M) return;
    i32 n_nn = seqn[q + stride < M ? q + stride : q];
    const i32 n0 = seqn[q];
    i64 s_n = inc_off[n0], t_n = inc_off[n0 + 1];
    for (; q < M; q += stride) {
        const i64 s = s_n, t = t_n;
        const i32 n1 = n_nn;
        n_nn = seqn[q + 2 * stride < M ? q + 2 * stride : q];
        s_n = inc_off[n1];
        t_n = inc_off[n1 + 1];
        i64 g = 0;
        i32 ls = 0, gd = 0;
        for (i64 i0 = s; i0 < t; i0 += 4 * kWave) {
            i32 pos[4], hh[4], cc[4], ww[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const i64 i = i0 + u * kWave + lane;
                const i64 ii = i < t ? i : s;
                pos[u] = inc_pos[ii];
                hh[u] = inc[ii];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                cc[u] = (i32)code[pos[u]];
                ww[u] = hw[hh[u]];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int in = (int)(i0 + u * kWave + lane < t);
                const i32 c = in ? cc[u] : 0;
                g += (i64)(in ? ww[u] : 0) * (i64)((c & 1) - ((c >> 1) & 1));
                ls += (c >> 2) & 1;
                gd += (c >> 3) & 1;
            }
        }
        g = wave_sum(g);
        ls = wave_sum(ls);
        gd = wave_sum(gd);
        if (lane == 0) {
            gseq[q] = g;
            dds[q] = -ls;
            ddd[q] = gd;
        }
        // the mover's id and offsets (20), per incidence entry its h-edge,
        // pin slot, weight and outcome byte (13), the three results (16)
        acc += 36 + 13 * (u64)(t - s);
    }
    if ((bytes != nullptr) & (lane == 0) & (acc != 0)) atomicAdd(bytes, (unsigned long long)acc);
}

// Two events per mover: (p_s, q) and (p_d, q) with their size and D deltas.
__global__ void k_events_build(i32 M, const i32* __restrict__ seqn, const i32* __restrict__ seqs,
                               const i32* __restrict__ seqd, const i32* __restrict__ nw, const i32* __restrict__ dds,
                               const i32* __restrict__ ddd, u32* evk, i64* evds, i64* evdd) {
    for (i64 q = (i64)blockIdx.x * blockDim.x + threadIdx.x; q < M; q += (i64)gridDim.x * blockDim.x) {
        const i64 s = nw[seqn[q]];
        evk[2 * q] = (u32)seqs[q];
        evds[2 * q] = -s;
        evdd[2 * q] = dds[q];
        evk[2 * q + 1] = (u32)seqd[q];
        evds[2 * q + 1] = s;
        evdd[2 * q + 1] = ddd[q];
    }
}

__global__ void k_ev_gather(i64 n2, const i32* __restrict__ idx, const i64* __restrict__ ds,
                            const i64* __restrict__ dd, i64* es, i64* ed) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (i64)gridDim.x * blockDim.x) {
        es[i] = ds[idx[i]];
        ed[i] = dd[idx[i]];
    }
}

__global__ void k_ev_segstart(i64 n2, const u32* __restrict__ key, i32* segst) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (i64)gridDim.x * blockDim.x) {
        const u32 k = key[i], kp = key[i > 0 ? i - 1 : 0];
        if ((int)(i == 0) | (int)(k != kp)) segst[k] = (i32)i;
    }
}

// Events sorted by (p, sequence position): running size and D of p after each
// event give its validity; a change of validity adds +1 / -1 to the violation
// count at that position (Sec. VI-D).
__global__ void k_ev_transitions(i64 n2, const u32* __restrict__ key, const i32* __restrict__ idx,
                                 const i32* __restrict__ segst, const i64* __restrict__ sex,
                                 const i64* __restrict__ dex, const i64* __restrict__ psize,
                                 const i64* __restrict__ pD, i64 omega, i64 delta, i32* dvq) {
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (i64)gridDim.x * blockDim.x) {
        const u32 p = key[i];
        const i64 s = segst[p];
        const i64 sz0 = psize[p], d0 = pD[p];
        const i64 s_s = sex[s], s_i = sex[i], s_i1 = sex[i + 1];
        const i64 d_s = dex[s], d_i = dex[i], d_i1 = dex[i + 1];
        const int after = (int)(sz0 + s_i1 - s_s > omega) | (int)(d0 + d_i1 - d_s > delta);
        const int before = (int)(sz0 + s_i - s_s > omega) | (int)(d0 + d_i - d_s > delta);
        const int d = after - before;
        if (d) atomicAdd(&dvq[idx[i] >> 1], d);
    }
}

// k* = smallest k maximising C_k over k = 0 or V_k = 0 (Sec. VI-D).
__global__ __launch_bounds__(1024) void k_select(i32 M, const i64* __restrict__ cex, const i64* __restrict__ vex,
                                                 unsigned long long* rs) {
    __shared__ i64 sg[16];
    __shared__ i32 sk[16];
    const i64 v0 = (i64)rs[5];
    i64 bg = 0;
    i32 bk = 0;
    for (i32 k = threadIdx.x + 1; k <= M; k += blockDim.x) {
        const i64 vk = vex[k], c = cex[k];
        const bool t = (int)(v0 + vk == 0) & (int)lex_gt(c, -k, bg, -bk);
        bg = t ? c : bg;
        bk = t ? k : bk;
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const i64 g2 = __shfl_xor(bg, o, kWave);
        const i32 k2 = __shfl_xor(bk, o, kWave);
        const bool t = lex_gt(g2, -k2, bg, -bk);
        bg = t ? g2 : bg;
        bk = t ? k2 : bk;
    }
    if (lane_id() == 0) {
        sg[wave_id()] = bg;
        sk[wave_id()] = bk;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        i64 G = 0;
        i32 K = 0;
        for (int w = 0; w < (int)(blockDim.x / kWave); ++w) {
            const i64 g2 = sg[w];
            const i32 k2 = sk[w];
            const bool t = lex_gt(g2, -k2, G, -K);
            G = t ? g2 : G;
            K = t ? k2 : K;
        }
        rs[3] = (unsigned long long)K;
        rs[4] = (unsigned long long)G;
    }
}

__global__ void k_apply(const unsigned long long* __restrict__ rs, const i32* __restrict__ seqn,
                        const i32* __restrict__ seqd, i32* rho) {
    const i64 K = (i64)rs[3];
    for (i64 q = (i64)blockIdx.x * blockDim.x + threadIdx.x; q < K; q += (i64)gridDim.x * blockDim.x)
        rho[seqn[q]] = seqd[q];
}

__global__ void k_project(i32 N, const i32* __restrict__ rc, const i32* __restrict__ gamma, i32* rf) {
    for (i64 n = (i64)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (i64)gridDim.x * blockDim.x)
        rf[n] = rc[gamma[n]];
}

// Eq. connectivity and Eq. cut-net from the row lengths lambda(e).
__global__ void k_conn(i32 E, const i32* __restrict__ len, const i32* __restrict__ hw, unsigned long long* out) {
    __shared__ i64 red[16];
    i64 conn = 0, cut = 0;
    for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += (i64)gridDim.x * blockDim.x) {
        conn += (i64)hw[e] * (len[e] - 1);
        cut += len[e] > 1 ? hw[e] : 0;
    }
    conn = block_sum(conn, red);
    cut = block_sum(cut, red);
    if (threadIdx.x == 0) {
        atomicAdd(&out[0], (unsigned long long)conn);
        atomicAdd(&out[1], (unsigned long long)cut);
    }
}

__global__ void k_part_eval(i32 nparts, const i64* __restrict__ psize, const i64* __restrict__ pD, i64 omega,
                            i64 delta, unsigned long long* out) {
    unsigned long long ms = 0, md = 0, viol = 0, ne = 0;
    for (i64 p = (i64)blockIdx.x * blockDim.x + threadIdx.x; p < nparts; p += (i64)gridDim.x * blockDim.x) {
        ms = ms > (u64)psize[p] ? ms : (u64)psize[p];
        md = md > (u64)pD[p] ? md : (u64)pD[p];
        const i64 sz = psize[p], dd = pD[p];
        viol += ((int)(sz > omega) | (int)(dd > delta)) ? 1 : 0;
        ne += psize[p] > 0 ? 1 : 0;
    }
    ms = wave_max(ms);
    md = wave_max(md);
    viol = wave_sum(viol);
    ne = wave_sum(ne);
    if (lane_id() == 0) {
        atomicMax(&out[2], ms);
        atomicMax(&out[3], md);
        atomicAdd(&out[4], viol);
        atomicAdd(&out[5], ne);
    }
}

int bits_for(u64 v) {
    int b = 0;
    while (b < 64 && (v >> b) != 0) ++b;
    return b;
}

struct PhiBufs {
    i32 *part, *cnt, *cin, *len;
    i64 *psize, *pD;
    unsigned short* part16;  // flagged 16-bit copy of part when nparts <= kGainsFlagParts, else null
};


// Whether listing the h-edges of `movers` nodes beats sweeping all h-edges.
// The list costs one device atomic per incidence entry of a mover (about
// movers * P / N), the sweep reads every pin and its sequence position (2P);
// the list is taken while the movers are under a quarter of the nodes, where
// it also spares the per-h-edge work of every h-edge without a mover.
bool few_touched(const Ctx* c, const Level& L, i64 movers) {
    const i64 gate = c->opt.tune[1] ? c->opt.tune[1] : 4;
    return L.N > 0 && movers * gate < (i64)L.N;
}

// Blocks of k_mark_edges for `cnt` listed nodes: a wave per about
// kMarkPerWave incidence entries at the level's mean degree, so that nodes of
// many h-edges still spread over many waves and nodes of few share one.
constexpr i64 kMarkPerWave = 512;
int mark_grid(const Ctx* c, const Level& L, i64 cnt) {
    const i64 deg = std::max<i64>(1, L.P / std::max<i64>(1, (i64)L.N));
    const i64 waves = std::max(ceil_div(cnt * deg, kMarkPerWave), ceil_div(cnt, (i64)kWave));
    return grid_for(waves, 4, c->num_cu * 16);
}

// Partition sizes and D(p) of rho from its Phi rows; psize and pD start at 0.
void part_stats(Ctx* c, const Level& L, const i32* rho, i32 nparts, const i32* part, const i32* cin, const i32* len,
                i64* psize, i64* pD) {
    const int nbins = nparts <= 16384 ? nparts : 0;  // 64 KiB of shared memory at most
    // blocks resident at once with this much shared memory, 8 per CU at most
    const int per_cu = std::max(1, std::min(8, (int)(160 * 1024 / (sizeof(u32) * nbins + 4096))));
    LAUNCH(c, KF_PART_STATS, k_part_sizes, grid_for(L.N, 256, c->num_cu * per_cu), 256, sizeof(u32) * nbins, L.N,
           rho, L.nw(), psize, nbins, prof_bytes(c, KF_PART_STATS));
    if (L.E > 0)
        LAUNCH(c, KF_PART_STATS, k_part_inbound, grid_for(L.E, 256, c->num_cu * per_cu), 256, sizeof(u32) * nbins,
               L.E, L.he_off(), part, cin, len, pD, nbins, prof_bytes(c, KF_PART_STATS));
}

PhiBufs phi_bufs(Ctx* c, const Level& L, i32 nparts) {
    PhiBufs f;
    f.part = wsp<i32>(c, WS_PHI_PART, (size_t)L.P + 1);
    f.cnt = wsp<i32>(c, WS_PHI_CNT, (size_t)L.P + 1);
    f.cin = wsp<i32>(c, WS_PHI_CIN, (size_t)L.P + 1);
    f.len = wsp<i32>(c, WS_PHI_LEN, (size_t)L.E + 1);
    f.psize = wsp<i64>(c, WS_PSIZE, nparts);
    f.pD = wsp<i64>(c, WS_PD, nparts);
    f.part16 = nparts <= kGainsFlagParts ? wsp<unsigned short>(c, WS_PHI_PART16, (size_t)L.P + 1) : nullptr;
    return f;
}

// Phi rows (with their 16-bit copy when the partition ids fit), partition
// sizes and D(p).  With elist, only the listed h-edges' rows are rebuilt: the
// others are those of the previous repetition, whose moves left them as they
// were.
// With elist, moved_k > 0 moves of the previous repetition were applied (its
// sequence buffers still hold them): the sizes and D of that repetition are
// updated from those moves and the listed rows instead of recomputed.
PhiBufs phi_and_parts(Ctx* c, const Level& L, const i32* rho, i32 nparts, unsigned char* single = nullptr,
                      const i32* elist = nullptr, const u32* ecount = nullptr, i64 moved_k = 0) {
    PhiBufs f;
    f.part = wsp<i32>(c, WS_PHI_PART, (size_t)L.P + 1);
    f.cnt = wsp<i32>(c, WS_PHI_CNT, (size_t)L.P + 1);
    f.cin = wsp<i32>(c, WS_PHI_CIN, (size_t)L.P + 1);
    f.len = wsp<i32>(c, WS_PHI_LEN, (size_t)L.E + 1);
    f.psize = wsp<i64>(c, WS_PSIZE, nparts);
    f.pD = wsp<i64>(c, WS_PD, nparts);
    f.part16 = (nparts <= kGainsFlagParts && L.P > 0) ? wsp<unsigned short>(c, WS_PHI_PART16, (size_t)L.P + 1)
                                                       : nullptr;
    if (elist && moved_k > 0) {
        const int nbins = nparts <= 16384 ? nparts : 0;  // 64 KiB of shared memory at most
        const size_t lds = sizeof(i32) * (size_t)nbins;
        const int per_cu = std::max(1, std::min(8, (int)(160 * 1024 / (lds + 4096))));
        const int grid = grid_for(L.E, 256, c->num_cu * per_cu);
        LAUNCH(c, KF_PART_STATS, k_inbound_listed, grid, 256, lds, elist, ecount, L.he_off(), f.part, f.cin, f.len,
               f.pD, nbins, -1);
        build_phi(c, L, rho, f.part, f.cnt, f.cin, f.len, single, f.part16, elist, ecount);
        LAUNCH(c, KF_PART_STATS, k_inbound_listed, grid, 256, lds, elist, ecount, L.he_off(), f.part, f.cin, f.len,
               f.pD, nbins, 1);
        const i32* seqn = wsp<i32>(c, WS_SEQN, (size_t)moved_k);
        const i32* seqs = wsp<i32>(c, WS_SEQS, (size_t)moved_k);
        const i32* seqd = wsp<i32>(c, WS_SEQD, (size_t)moved_k);
        LAUNCH(c, KF_PART_STATS, k_sizes_moved, grid_for(moved_k, 256, c->num_cu * per_cu), 256, lds, moved_k, seqn,
               seqs, seqd, L.nw(), f.psize, nbins);
        return f;
    }
    build_phi(c, L, rho, f.part, f.cnt, f.cin, f.len, single, f.part16, elist, ecount);
    fill_many(c, {{f.psize, 2 * (i64)nparts, 0u}, {f.pD, 2 * (i64)nparts, 0u}});
    part_stats(c, L, rho, nparts, f.part, f.cin, f.len, f.psize, f.pD);
    return f;
}

}  // namespace

RepInfo refine_rep(Ctx* c, const Level& L, i32* rho, i32 nparts, int rep, int theta, RepTrace* trace,
                   bool reuse, i64 incr_k) {
    RepInfo info;
    const i32 N = L.N;
    const int nbN = grid_for(N, 256, c->num_cu * 8);
    // h-edge marks of this repetition: stamp 1 lists the h-edges whose rows the
    // previous repetition's applied moves changed, stamp 2 those holding a
    // mover of this one.
    u32* emark = wsp<u32>(c, WS_EMARK, (size_t)(L.E > 0 ? L.E : 1));
    u32* ecount = wsp<u32>(c, WS_ECOUNT, 2);
    i32* elist = wsp<i32>(c, WS_ELIST, (size_t)(L.E > 0 ? L.E : 1));
    bool marks_clear = false;  // emark and the counts zeroed in this repetition
    auto clear_marks = [&]() {
        if (!marks_clear) fill_many(c, {{emark, (i64)L.E, 0u}, {ecount, 2, 0u}});
        marks_clear = true;
    };
    // With incr_k > 0, the previous repetition on this level applied the first
    // incr_k moves of its sequence (still in the sequence buffer): only the
    // rows of their h-edges changed.  Listing them costs one device atomic per
    // incidence entry of a mover, so the list is used only while those entries
    // (about incr_k * P / N) stay well below the h-edges swept without it.
    const bool incremental = !reuse && incr_k > 0 && L.E > 0 && few_touched(c, L, incr_k);
    if (incremental) {
        clear_marks();
        const i32* prev_seq = wsp<i32>(c, WS_SEQN, (size_t)incr_k);
        LAUNCH(c, KF_PHI, k_mark_edges, mark_grid(c, L, incr_k), 256, 0, (i32)incr_k, prev_seq,
               L.inc_off(), L.inc(), emark, 1u, elist, ecount);
    }
    // With `reuse`, rho is unchanged since the previous repetition (it applied
    // nothing): its pins rows, sizes, D and both move variants still hold.
    // Small levels take the moves from a dense MFMA product, which needs one
    // byte per pin slot from the Phi kernel (pins(rho(m), e) = 1).
    const bool dense_gains = !reuse && use_dense_gains(c, L, nparts);
    unsigned char* single = dense_gains ? wsp<unsigned char>(c, WS_SINGLE, (size_t)(L.P > 0 ? L.P : 1)) : nullptr;
    PhiBufs f = reuse ? phi_bufs(c, L, nparts)
                      : phi_and_parts(c, L, rho, nparts, single, incremental ? elist : nullptr, ecount,
                                      incremental ? incr_k : 0);
    unsigned long long* rs = wsp<unsigned long long>(c, WS_RSTATS, 8);
    HIPC(hipMemsetAsync(rs, 0, 8 * sizeof(u64), c->stream));
    LAUNCH(c, KF_PART_STATS, k_initial_violations, grid_for(nparts, 256, c->num_cu * 4), 256, 0, nparts, f.psize,
           f.pD, c->omega, c->delta, rs + 5);

    // Moves (Sec. VI-B): both the unconstrained and the size-aware variant.
    i32* mdst_any = wsp<i32>(c, WS_MDST, N);
    i64* mgain_any = wsp<i64>(c, WS_MGAIN, N);
    i32* mdst_sa = wsp<i32>(c, WS_MDST_SA, N);
    i64* mgain_sa = wsp<i64>(c, WS_MGAIN_SA, N);
    const bool size_aware = rep >= theta / 2;
    if (dense_gains) {
        gains_dense(c, L, rho, nparts, f.part, f.len, single, f.psize, mdst_any, mgain_any, mdst_sa, mgain_sa);
    } else if (!reuse) {
        const int R = (int)std::min<i64>(16384, std::max<i64>(64, nparts));
        const size_t lds = sizeof(u32) * (size_t)R;
        const int per_cu = std::max(1, std::min(8, (int)(160 * 1024 / (lds + 3 * 1024))));
        const int grid = (int)std::min<i64>(N, (i64)c->num_cu * per_cu * 2);
        if (f.part16 && nparts <= kGainsWaveParts && (i64)L.P <= kGainsWaveDeg * (i64)N) {
            // few h-edges per node: one wave per node, bins per wave
            const int Rw = (nparts + kWave - 1) / kWave * kWave;
            const size_t ldsw = sizeof(u32) * (size_t)Rw * kGainsWaves;
            const int gridw = (int)std::min<i64>((N + kGainsWaves - 1) / kGainsWaves, (i64)c->num_cu * 16);
            LAUNCH(c, KF_GAINS, k_gains16w, gridw, kGainsWaves * kWave, ldsw, N, nparts, L.inc_off(), L.inc(),
                   L.he_off(), (const unsigned short*)f.part16, f.len, c->hw(), L.nw(), rho, f.psize, c->omega,
                   mdst_any, mgain_any, mdst_sa, mgain_sa, Rw, prof_work(c, KF_GAINS));
        } else if (f.part16 && nparts <= R)  // half the bytes per row visit, one pass
            LAUNCH(c, KF_GAINS, k_gains16<true>, grid, kGainsWaves * kWave, lds, N, nparts, L.inc_off(), L.inc(),
                   L.he_off(), (const unsigned short*)f.part16, f.len, c->hw(), L.nw(), rho, f.psize, c->omega,
                   mdst_any, mgain_any, mdst_sa, mgain_sa, R, prof_work(c, KF_GAINS));
        else if (f.part16)
            LAUNCH(c, KF_GAINS, k_gains16<false>, grid, kGainsWaves * kWave, lds, N, nparts, L.inc_off(), L.inc(),
                   L.he_off(), (const unsigned short*)f.part16, f.len, c->hw(), L.nw(), rho, f.psize, c->omega,
                   mdst_any, mgain_any, mdst_sa, mgain_sa, R, prof_work(c, KF_GAINS));
        else
            LAUNCH(c, KF_GAINS, k_gains<i32>, grid, kGainsWaves * kWave, lds, N, nparts, L.inc_off(), L.inc(),
                   L.he_off(), (const i32*)f.part, f.cnt, f.len, c->hw(), L.nw(), rho, f.psize, c->omega, mdst_any,
                   mgain_any, mdst_sa, mgain_sa, R);
    }
    i32* mdst = size_aware ? mdst_sa : mdst_any;
    i64* mgain = size_aware ? mgain_sa : mgain_any;
    i32* mflag = wsp<i32>(c, WS_MFLAG, N);
    i32* mpos = wsp<i32>(c, WS_MPOS, (size_t)N + 1);
    LAUNCH(c, KF_MOVES, k_move_flags, nbN, 256, 0, N, mdst, mflag);
    scan_excl_i32(c, mflag, mpos, N);
    if (trace && trace->move_dst)
        HIPC(hipMemcpyAsync(trace->move_dst, mdst, sizeof(i32) * N, hipMemcpyDeviceToHost, c->stream));
    if (trace && trace->move_gain)
        HIPC(hipMemcpyAsync(trace->move_gain, mgain, sizeof(i64) * N, hipMemcpyDeviceToHost, c->stream));
    i64 M = 0;
    read_back(c, mpos + N, &M, 1, 4);
    info.moves = M;
    if (M == 0) return info;
    const int nbM = grid_for(M, 256, c->num_cu * 8);
    // Every buffer of the rest of the repetition that starts from a constant,
    // set in one launch.
    i32* sidx = wsp<i32>(c, WS_SIDX, N);
    i32* segb = wsp<i32>(c, WS_SEGB, nparts);
    i32* sege = wsp<i32>(c, WS_SEGE, nparts);
    i32* pred = wsp<i32>(c, WS_PRED, M);
    i32* succ = wsp<i32>(c, WS_SUCC, M);
    i64* cg = wsp<i64>(c, WS_CG, M);
    i32* clen = wsp<i32>(c, WS_CLEN, M);
    i32* dvq = wsp<i32>(c, WS_DVQ, M);
    fill_many(c, {{sidx, N, ~0u},
                  {segb, nparts, 0u},
                  {sege, nparts, 0u},
                  {pred, M, ~0u},
                  {succ, M, ~0u},
                  {cg, 2 * M, 0u},
                  {clen, M, 0u},
                  {dvq, M, 0u}});

    // Moves sorted by (p_s, -gain, id) (Sec. VI-C).
    u64* mkey = wsp<u64>(c, WS_MKEY, M);
    u64* mkey2 = wsp<u64>(c, WS_MKEY2, M);
    i32* mval = wsp<i32>(c, WS_MVAL, M);
    i32* snode = wsp<i32>(c, WS_SNODE, M);
    LAUNCH(c, KF_MOVES, k_move_keys, nbN, 256, 0, N, mflag, mpos, rho, mgain, mkey, mval);
    sort_pairs_u64(c, mkey, mkey2, mval, snode, M, 32 + bits_for((u64)nparts));
    i32* sps = wsp<i32>(c, WS_SPS, M);
    i32* spd = wsp<i32>(c, WS_SPD, M);
    i64* sg = wsp<i64>(c, WS_SG, M);
    i32* snw = wsp<i32>(c, WS_SNW, M);
    i32* snin = wsp<i32>(c, WS_SNIN, M);
    LAUNCH(c, KF_MOVES, k_sorted_attrs, nbM, 256, 0, (i32)M, snode, rho, mdst, mgain, L.nw(), L.inc_nin(), sps, spd,
           sg, snw, snin, sidx);
    LAUNCH(c, KF_MOVES, k_segments, nbM, 256, 0, (i32)M, sps, segb, sege);

    // Chain rounds.
    i32* pl = wsp<i32>(c, WS_PL, M);
    i32* pls = wsp<i32>(c, WS_PLS, M + 1);
    i32* cl = wsp<i32>(c, WS_CL, M);
    i32* prop = wsp<i32>(c, WS_PROP, M);
    i64* propG = wsp<i64>(c, WS_PROPG, M);
    u64* accG = wsp<u64>(c, WS_ACCG, M);
    i32* accN = wsp<i32>(c, WS_ACCN, M);
    LAUNCH(c, KF_CHAINS, k_set_flag, 1, 1, 0, rs);
    const int wblocks = grid_for(M, 4, c->num_cu * 16);
    // flags bit 5: the ablation without chain rounds (every move its own chain)
    const int rounds = (c->opt.flags & 32) ? 0 : kChainRounds;
    if (M <= kChainSingleMax && rounds > 0)
        LAUNCH(c, KF_CHAINS, k_chain_rounds, 1, 1024, 0, (i32)M, rs, pred, succ, pl, pls, cl, accG, accN, spd, segb,
               sege, sg, snw, snin, snode, prop, propG);
    // Up to kChainCompactMax moves, everything but the windowed proposals of
    // a round runs in single-workgroup launches: two launches per round.
    const bool one = M <= kChainCompactMax;
    if (one && M > kChainSingleMax && rounds > 0)
        LAUNCH(c, KF_CHAINS, k_chain_compact1, 1, 1024, 0, (i32)M, 0, rs, pred, pls, cl, accG, accN);
    for (int round = 0; round < rounds && M > kChainSingleMax && one; ++round) {
        // proposals on the whole device, the rest of the round (and the next
        // round's compaction) in one workgroup
        LAUNCH(c, KF_CHAINS, k_chain_propose, wblocks, 256, 0, (i32)M, rs, succ, spd, segb, sege, pls, cl, sg, snw,
               snin, snode, prop, propG);
        LAUNCH(c, KF_CHAINS, k_chain_tail1, 1, 1024, 0, (i32)M, (int)(round + 1 < rounds), rs, pred, succ, pls, cl,
               accG, accN, snode, prop, propG);
        if (round == 1 || round == 3 || round == 7) {
            i64 active = 0;
            read_back(c, rs, &active, 1, 8);
            if (!active) break;
        }
    }
    for (int round = 0; round < rounds && M > kChainSingleMax && !one; ++round) {
        {
            const ScanLaunch sl = scan_launch(c, M);
            LAUNCH(c, KF_CHAINS, k_predless_compact, (int)sl.tiles, kLbBlock, 0, (i32)M, rs, (const i32*)pred, pls,
                   cl, accG, accN, sl.st, sl.tag, sl.ticket0, sl.tiles);
        }
        LAUNCH(c, KF_CHAINS, k_chain_propose, wblocks, 256, 0, (i32)M, rs, succ, spd, segb, sege, pls, cl, sg, snw,
               snin, snode, prop, propG);
        LAUNCH(c, KF_CHAINS, k_chain_accept_a, nbM, 256, 0, (i32)M, rs, prop, propG, accG);
        LAUNCH(c, KF_CHAINS, k_chain_accept_b, nbM, 256, 0, (i32)M, rs, prop, propG, accG, snode, accN);
        LAUNCH(c, KF_CHAINS, k_chain_link, nbM, 256, 0, (i32)M, rs, prop, propG, accG, accN, snode, pred, succ);
        LAUNCH(c, KF_CHAINS, k_round_end, 1, 1, 0, rs);
        // Later rounds of a finished chain build are no-ops; stop issuing them.
        if (round == 1 || round == 3 || round == 7) {
            i64 active = 0;
            read_back(c, rs, &active, 1, 8);
            if (!active) break;
        }
    }

    // Chains: cycles, heads, ranks.
    const int K = bits_for((u64)M) + 1;
    i32 *J0 = wsp<i32>(c, WS_J0, M), *J1 = wsp<i32>(c, WS_J1, M);
    i32 *MN0 = wsp<i32>(c, WS_MN0, M), *MN1 = wsp<i32>(c, WS_MN1, M);
    LAUNCH(c, KF_RANK, k_cyc_init, nbM, 256, 0, (i32)M, succ, snode, J0, MN0);
    if (M <= kJumpSingleMax)
        LAUNCH(c, KF_RANK, k_cyc_steps, 1, 1024, 0, (i32)M, K, J0, MN0, J1, MN1);
    for (int it = 0; it < K; ++it) {
        if (M > kJumpSingleMax) LAUNCH(c, KF_RANK, k_cyc_step, nbM, 256, 0, (i32)M, J0, MN0, J1, MN1);
        std::swap(J0, J1);
        std::swap(MN0, MN1);
    }
    i32 *P0 = wsp<i32>(c, WS_P0, M), *P1 = wsp<i32>(c, WS_P1, M);
    i32 *R0 = wsp<i32>(c, WS_R0, M), *R1 = wsp<i32>(c, WS_R1, M);
    i32 *H0 = wsp<i32>(c, WS_H0, M), *H1 = wsp<i32>(c, WS_H1, M);
    i32* head = wsp<i32>(c, WS_HEAD, M);
    LAUNCH(c, KF_RANK, k_heads, nbM, 256, 0, (i32)M, J0, MN0, pred, snode, P0, R0, H0, head);
    if (M <= kJumpSingleMax)
        LAUNCH(c, KF_RANK, k_rank_steps, 1, 1024, 0, (i32)M, K, P0, R0, H0, P1, R1, H1);
    for (int it = 0; it < K; ++it) {
        if (M > kJumpSingleMax) LAUNCH(c, KF_RANK, k_rank_step, nbM, 256, 0, (i32)M, P0, R0, H0, P1, R1, H1);
        std::swap(P0, P1);
        std::swap(R0, R1);
        std::swap(H0, H1);
    }
    LAUNCH(c, KF_RANK, k_chain_accum, nbM, 256, 0, (i32)M, H0, sg, cg, clen);
    i32* hf = wsp<i32>(c, WS_HF, N);
    i32* hpos = wsp<i32>(c, WS_HPOS, (size_t)N + 1);
    LAUNCH(c, KF_RANK, k_head_flags, nbN, 256, 0, N, sidx, head, hf);
    scan_excl_i32(c, hf, hpos, N);
    i64 C = 0;
    read_back(c, hpos + N, &C, 1, 4);
    u64* hkey = wsp<u64>(c, WS_HKEY, C);
    u64* hkey2 = wsp<u64>(c, WS_HKEY2, C);
    i32* hval = wsp<i32>(c, WS_HVAL, C);
    i32* rh = wsp<i32>(c, WS_HVAL2, C);
    LAUNCH(c, KF_RANK, k_head_keys, nbN, 256, 0, N, hf, hpos, sidx, cg, hkey, hval);
    sort_pairs_u64(c, hkey, hkey2, hval, rh, C, 62);
    i32* lr = wsp<i32>(c, WS_LR, C);
    i32* lrs = wsp<i32>(c, WS_LRS, C + 1);
    i32* cstart = wsp<i32>(c, WS_CSTART, M);
    const int nbC = grid_for(C, 256, c->num_cu * 8);
    LAUNCH(c, KF_RANK, k_ranked_len, nbC, 256, 0, (i32)C, rh, clen, lr);
    scan_excl_i32(c, lr, lrs, C);
    LAUNCH(c, KF_RANK, k_chain_start, nbC, 256, 0, (i32)C, rh, lrs, cstart);
    i32* seqn = wsp<i32>(c, WS_SEQN, M);
    i32* seqs = wsp<i32>(c, WS_SEQS, M);
    i32* seqd = wsp<i32>(c, WS_SEQD, M);
    i32* posn = wsp<i32>(c, WS_POSN, N);
    fill_i32(c, posn, 0x7FFFFFFF, N);
    LAUNCH(c, KF_RANK, k_positions, nbM, 256, 0, (i32)M, H0, R0, cstart, snode, sps, spd, seqn, seqs, seqd, posn);

    // In-sequence gains and events.
    i64* gseq = wsp<i64>(c, WS_GSEQ, M);
    const i64 M2 = 2 * M;
    u32* evk = wsp<u32>(c, WS_EVK, M2);
    u32* evk2 = wsp<u32>(c, WS_EVK2, M2);
    i32* evi = wsp<i32>(c, WS_EVI, M2);
    i32* evi2 = wsp<i32>(c, WS_EVI2, M2);
    i64* evds = wsp<i64>(c, WS_EVDS, M2);
    i64* evdd = wsp<i64>(c, WS_EVDD, M2);
    i32* dds = wsp<i32>(c, WS_DDS, M);
    i32* ddd = wsp<i32>(c, WS_DDD, M);
    unsigned char* code = wsp<unsigned char>(c, WS_CODE, (size_t)(L.P > 0 ? L.P : 1));
    if (L.E > 0) {
        // Only h-edges holding a mover have in-sequence effects: when the
        // movers are few, list those once each (stamp 2) and sweep only them.
        const bool listed = few_touched(c, L, M);
        i32* elist2 = listed ? wsp<i32>(c, WS_ELIST2, (size_t)L.E) : nullptr;
        if (listed) {
            clear_marks();
            LAUNCH(c, KF_INSEQ, k_mark_edges, mark_grid(c, L, M), 256, 0, (i32)M, (const i32*)seqn,
                   L.inc_off(), L.inc(), emark, 2u, elist2, ecount + 1);
        }
        // H-edges of at most kInseqSmall pins one lane each; event lists for
        // up to kInseqGroup pins in 16-lane groups, up to kInseqListMax in whole
        // waves; all pairs beyond.
        const int cap = std::max(1, c->max_card);
        const int capl = std::min(cap, kInseqListMax);
        auto table_bits = [](int pins_max) {
            int tb = 1;
            while ((1 << tb) < 2 * pins_max) ++tb;
            return tb;
        };
        LAUNCH(c, KF_INSEQ, k_inseq_small, grid_for(L.E, 256, c->num_cu * 8), 256, 0, L.E, (i32)M, L.he_off(),
               L.he_nsrc(), L.pins(), posn, rho, mdst, f.part, f.cnt, f.cin, f.len, code, (const i32*)elist2,
               (const u32*)(ecount + 1), prof_bytes(c, KF_INSEQ));
        const int nbw = (int)std::min<i64>(ceil_div(L.E, (i64)kWindowMin), (i64)c->num_cu * 32);
        if (cap > kInseqSmall) {
            const int capg = std::min(cap, kInseqGroup), tbg = table_bits(capg);
            const size_t lds_g = (size_t)(kWave / 16) * ((size_t)24 * capg + (size_t)12 * ((size_t)1 << tbg));
            LAUNCH(c, KF_INSEQ, k_inseq_lists<16>, nbw, kWave, lds_g, L.E, (i32)M, L.he_off(), L.he_nsrc(), L.pins(),
                   posn, rho, mdst, f.part, f.cnt, f.cin, f.len, code, capg, tbg, kInseqSmall, (const i32*)elist2,
                   (const u32*)(ecount + 1), prof_bytes(c, KF_INSEQ));
        }
        if (cap > kInseqGroup) {
            const int tbl = table_bits(capl);
            const size_t lds_l = (size_t)24 * capl + (size_t)12 * ((size_t)1 << tbl);
            LAUNCH(c, KF_INSEQ, k_inseq_lists<64>, nbw, kWave, lds_l, L.E, (i32)M, L.he_off(), L.he_nsrc(), L.pins(),
                   posn, rho, mdst, f.part, f.cnt, f.cin, f.len, code, capl, tbl, kInseqGroup, (const i32*)elist2,
                   (const u32*)(ecount + 1), prof_bytes(c, KF_INSEQ));
        }
        if (cap > capl)
            LAUNCH(c, KF_INSEQ, k_inseq_edges, nbw, kWave,
                   (sizeof(MoverRec) + 2 * sizeof(i32)) * cap, L.E, (i32)M, L.he_off(), L.he_nsrc(), L.pins(), posn,
                   rho, mdst, f.part, f.cnt, f.cin, f.len, code, cap, (i32)capl, (const i32*)elist2,
                   (const u32*)(ecount + 1), prof_bytes(c, KF_INSEQ));
    }
    LAUNCH(c, KF_INSEQ, k_inseq_movers, grid_for(M, 4, c->num_cu * 16), 256, 0, (i32)M, seqn, L.inc_off(), L.inc(),
           L.inc_pos(), c->hw(), code, gseq, dds, ddd, prof_bytes(c, KF_INSEQ));
    LAUNCH(c, KF_EVENTS, k_events_build, nbM, 256, 0, (i32)M, seqn, seqs, seqd, L.nw(), dds, ddd, evk, evds, evdd);
    iota_i32(c, evi, M2);
    sort_pairs_u32(c, evk, evk2, evi, evi2, M2, bits_for((u64)nparts));
    i64* es = wsp<i64>(c, WS_ES, M2);
    i64* ed = wsp<i64>(c, WS_ED, M2);
    const int nbE = grid_for(M2, 256, c->num_cu * 8);
    LAUNCH(c, KF_EVENTS, k_ev_gather, nbE, 256, 0, M2, evi2, evds, evdd, es, ed);
    i64* sex = wsp<i64>(c, WS_SEX, M2 + 1);
    i64* dex = wsp<i64>(c, WS_DEX, M2 + 1);
    scan_excl_i64(c, es, sex, M2);
    scan_excl_i64(c, ed, dex, M2);
    i32* segst = wsp<i32>(c, WS_SEGST, nparts);
    LAUNCH(c, KF_EVENTS, k_ev_segstart, nbE, 256, 0, M2, evk2, segst);
    LAUNCH(c, KF_EVENTS, k_ev_transitions, nbE, 256, 0, M2, evk2, evi2, segst, sex, dex, f.psize, f.pD, c->omega,
           c->delta, dvq);
    i64* cex = wsp<i64>(c, WS_CEX, M + 1);
    i64* vex = wsp<i64>(c, WS_VEX, M + 1);
    scan_excl_i64(c, gseq, cex, M);
    scan_excl_i32_to_i64(c, dvq, vex, M);
    LAUNCH(c, KF_SELECT, k_select, 1, 1024, 0, (i32)M, cex, vex, rs);
    LAUNCH(c, KF_APPLY, k_apply, nbM, 256, 0, rs, seqn, seqd, rho);
    i64 out[6];
    read_back(c, rs, out, 6, 8);
    info.links = out[2];
    info.kstar = out[3];
    info.gain = out[4];
    if (trace) {
        auto copy = [&](void* host, const void* dev, size_t bytes) {
            if (host && bytes) HIPC(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, c->stream));
        };
        copy(trace->seq, seqn, sizeof(i32) * M);
        copy(trace->seq_dst, seqd, sizeof(i32) * M);
        copy(trace->gseq, gseq, sizeof(i64) * M);
        copy(trace->prefix_gain, cex, sizeof(i64) * (M + 1));
        copy(trace->prefix_viol, vex, sizeof(i64) * (M + 1));
        HIPC(hipStreamSynchronize(c->stream));
        if (trace->prefix_viol)
            for (i64 k = 0; k <= M; ++k) trace->prefix_viol[k] += out[5];  // V_k = V_0 + changes
    }
    return info;
}

void project_rho(Ctx* c, const i32* rho_coarse, const i32* gamma, i32* rho_fine, i32 N) {
    LAUNCH(c, KF_PROJECT, k_project, grid_for(N, 256, c->num_cu * 8), 256, 0, N, rho_coarse, gamma, rho_fine);
}

void evaluate_dev(Ctx* c, const Level& L, const i32* rho, i32 nparts, hgp_eval* out) {
    PhiBufs f = phi_and_parts(c, L, rho, nparts);
    unsigned long long* rs = wsp<unsigned long long>(c, WS_RSTATS, 8);
    HIPC(hipMemsetAsync(rs, 0, 8 * sizeof(u64), c->stream));
    if (L.E > 0)
        LAUNCH(c, KF_EVAL, k_conn, grid_for(L.E, 256, c->num_cu * 4), 256, 0, L.E, f.len, c->hw(), rs);
    LAUNCH(c, KF_EVAL, k_part_eval, grid_for(nparts, 256, c->num_cu * 4), 256, 0, nparts, f.psize, f.pD, c->omega,
           c->delta, rs);
    i64 v[6];
    read_back(c, rs, v, 6, 8);
    out->conn = v[0];
    out->cutnet = v[1];
    out->max_size = v[2];
    out->max_inbound = v[3];
    out->violations = v[4];
    out->n_parts = v[5];
}

// Entries of rho outside [0, nparts).
__global__ void k_rho_check(i32 N, const i32* __restrict__ rho, i32 nparts, unsigned long long* bad) {
    unsigned long long c = 0;
    for (i64 n = (i64)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (i64)gridDim.x * blockDim.x)
        c += (u32)rho[n] >= (u32)nparts ? 1 : 0;
    c = wave_sum(c);
    if (lane_id() == 0 && c) atomicAdd(bad, c);
}

void* noalloc_scratch_init(int device) {
    static std::mutex mu;
    static std::map<int, void*> addr;  // device ordinal -> address of `scratch` there
    std::lock_guard<std::mutex> lock(mu);
    const auto it = addr.find(device);
    if (it != addr.end()) return it->second;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
        (void)hipGetLastError();
        fail(HGP_E_DEVICE, std::string("hipGetSymbolAddress of the static workspace: ") + hipGetErrorString(e));
    }
    addr[device] = p;
    return p;
}

namespace {

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Workspace layout: results (8 words: conn, cut-net, max size, max D,
// violations, non-empty parts, invalid rho entries), psize [nparts], D
// [nparts], lambda [E], then the rows part / cnt / cnt_in [P] each.
struct NoAllocLayout {
    size_t res, psize, pD, len, part, cnt, cin, total;
    NoAllocLayout(const Level& L, i32 nparts) {
        size_t o = 0;
        res = o;
        o += align256(8 * sizeof(u64));
        psize = o;
        o += align256(sizeof(i64) * (size_t)nparts);
        pD = o;
        o += align256(sizeof(i64) * (size_t)nparts);
        len = o;
        o += align256(sizeof(i32) * (size_t)std::max<i32>(L.E, 1));
        part = o;
        o += align256(sizeof(i32) * (size_t)std::max<i64>(L.P, 1));
        cnt = o;
        o += align256(sizeof(i32) * (size_t)std::max<i64>(L.P, 1));
        cin = o;
        o += align256(sizeof(i32) * (size_t)std::max<i64>(L.P, 1));
        total = o;
    }
};

// Records no profiling events while alive (event creation allocates).
struct ProfPause {
    Ctx* c;
    int saved;
    explicit ProfPause(Ctx* cc) : c(cc), saved(cc->opt.profile) { c->opt.profile = 0; }
    ~ProfPause() { c->opt.profile = saved; }
};

}  // namespace

size_t noalloc_eval_bytes(const Level& L, i32 nparts) { return NoAllocLayout(L, nparts).total; }

void evaluate_noalloc(Ctx* c, const Level& L, const i32* rho, i32 nparts, hgp_eval* out) {
    const NoAllocLayout lay(L, nparts);
    if (lay.total > kNoAllocScratchBytes)
        fail(HGP_E_UNSUPPORTED, "hgp_evaluate_noalloc needs " + std::to_string(lay.total) +
                                    " bytes of workspace (12 per pin, 4 per h-edge, 16 per partition); the static "
                                    "workspace holds " +
                                    std::to_string(kNoAllocScratchBytes));
    if (c->noalloc_scratch == nullptr) fail(HGP_E_STATE, "static workspace not set up on this device");
    unsigned char* base = (unsigned char*)c->noalloc_scratch;
    unsigned long long* res = (unsigned long long*)(base + lay.res);
    i64* psize = (i64*)(base + lay.psize);
    i64* pD = (i64*)(base + lay.pD);
    i32* len = (i32*)(base + lay.len);
    i32* part = (i32*)(base + lay.part);
    i32* cnt = (i32*)(base + lay.cnt);
    i32* cin = (i32*)(base + lay.cin);
    ProfPause pause(c);
    // The workspace keeps the previous call's contents: clear what the
    // atomics accumulate into (the rows are rewritten whole).
    fill_many(c, {{res, 16, 0u}, {psize, 2 * (i64)nparts, 0u}, {pD, 2 * (i64)nparts, 0u}});
    LAUNCH(c, KF_EVAL, k_rho_check, grid_for(L.N, 256, c->num_cu * 8), 256, 0, L.N, rho, nparts, res + 6);
    i64 bad = 0;
    read_back(c, res + 6, &bad, 1, 8);
    if (bad != 0) fail(HGP_E_INVALID, std::to_string(bad) + " entries of rho outside [0, n_parts)");
    build_phi(c, L, rho, part, cnt, cin, len, nullptr);
    part_stats(c, L, rho, nparts, part, cin, len, psize, pD);
    if (L.E > 0)
        LAUNCH(c, KF_EVAL, k_conn, grid_for(L.E, 256, c->num_cu * 4), 256, 0, L.E, (const i32*)len, c->hw(), res);
    LAUNCH(c, KF_EVAL, k_part_eval, grid_for(nparts, 256, c->num_cu * 4), 256, 0, nparts, (const i64*)psize,
           (const i64*)pD, c->omega, c->delta, res);
    i64 v[6];
    read_back(c, res, v, 6, 8);
    out->conn = v[0];
    out->cutnet = v[1];
    out->max_size = v[2];
    out->max_inbound = v[3];
    out->violations = v[4];
    out->n_parts = v[5];
}

// Phi rows of level-0 for export: copies of the last built rows.
void phi_export(Ctx* c, const Level& L, const i32* rho, i32 nparts, i32** part, i32** cnt, i32** cin, i32** len) {
    PhiBufs f = phi_and_parts(c, L, rho, nparts);
    *part = f.part;
    *cnt = f.cnt;
    *cin = f.cin;
    *len = f.len;
}

}  // namespace hgp
