// Candidate proposal for small levels as matrix products on the MFMA units
// (Sec. V-C).  With H the node x h-edge incidence (1 where n is a pin of e),
// H_in its destination part and T = diag(t(e)), the histogram values of every
// pair are eta = H T H^T and inter = H_in H_in^T.  Once a level has a few
// thousand nodes, nearly every pair shares an h-edge and the products are
// dense; they are computed exactly in int8 x int8 -> int32 MFMA by splitting
// t(e) into 7-bit digit planes.  The candidates are then selected from each
// node's dense row by the same rules as the histogram kernel: score = eta +
// noise, validity through sizes and |in(n)| + |in(m)| - inter, top PI by
// (score desc, id desc).
#include <algorithm>

#include "dev_util.h"
#include "top_select.h"

namespace hgp {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kTile = 128;      // output rows and columns per workgroup
constexpr int kMaxPlanes = 3;   // 7-bit digit planes of t(e): t < 2^21
constexpr int kSelU = 8;        // row entries per thread per step of the selection

enum { WS_DN_A = 170, WS_DN_D = 171, WS_DN_DIG = 172, WS_DN_PART = 173, WS_DG_B = 174, WS_DG_WI = 175,
       WS_DG_SAV = 176, WS_DG_DIG = 177 };

// Bit rows, one block per node: bit e of row n is set iff n is a pin of e
// (A) or a destination of e (D, skipped when null).  Rows are W4 words (a
// multiple of 4); rows from N to the padded count are zero.
__global__ __launch_bounds__(256) void k_dense_bits(i32 N, i32 Npad, i32 W4, const i64* __restrict__ inc_off,
                                                    const i32* __restrict__ inc_nin, const i32* __restrict__ inc,
                                                    u32* A, u32* D) {
    extern __shared__ u32 row[];  // 2 * W4 words
    for (i32 n = blockIdx.x; n < Npad; n += gridDim.x) {
        for (int i = threadIdx.x; i < 2 * W4; i += blockDim.x) row[i] = 0;
        __syncthreads();
        if (n < N) {
            const i64 a = inc_off[n], b = inc_off[n + 1];
            const i32 nin = inc_nin[n];
            for (i64 k = a + threadIdx.x; k < b; k += blockDim.x) {
                const i32 e = inc[k];
                atomicOr(&row[e >> 5], 1u << (e & 31));
                if ((D != nullptr) & (k - a < nin)) atomicOr(&row[W4 + (e >> 5)], 1u << (e & 31));  // inbound entries come first
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < W4; i += blockDim.x) {
            A[(i64)n * W4 + i] = row[i];
            if (D) D[(i64)n * W4 + i] = row[W4 + i];
        }
        __syncthreads();
    }
}

// Digit planes of the normalised weights: dig[p][e] = (t(e) >> 7p) & 127
// (with `raw`, of the h-edge weights w(e) themselves).
__global__ void k_dense_digits(i32 E, i32 Epad, int NP, const i64* __restrict__ he_off, const i32* __restrict__ hw,
                               signed char* dig, int raw) {
    for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < Epad; e += (i64)gridDim.x * blockDim.x) {
        const u64 t = e < E ? (raw ? (u64)(u32)hw[e] : norm_weight(hw[e], he_off[e + 1] - he_off[e])) : 0;
        for (int p = 0; p < NP; ++p) dig[(i64)p * Epad + e] = (signed char)((t >> (7 * p)) & 127);
    }
}

// 0 / 1 bytes -> 0x00 / 0x7F bytes: 0x80 - b per byte never borrows across
// bytes, and the low 7 bits cover every 7-bit digit it is ANDed with.  (A
// shift and subtract, x * 255, is turned into a quarter-rate multiply.)
__device__ __forceinline__ v4i digit_mask(v4i b) {
    const v4i k80 = {(int)0x80808080u, (int)0x80808080u, (int)0x80808080u, (int)0x80808080u};
    return (k80 - b) & 0x7F7F7F7F;
}

// 16 bits -> 16 bytes of 0 / 1, bit j into byte j (four nibbles, each spread
// by one multiply: the shifted copies do not overlap, so nothing carries).
// Both factors fit 24 bits, so the full-rate 24-bit multiply is exact.
__device__ __forceinline__ v4i spread16(u32 bits) {
    v4i r;
    r.x = (int)(__umul24((bits >> 0) & 15u, 0x00204081u) & 0x01010101u);
    r.y = (int)(__umul24((bits >> 4) & 15u, 0x00204081u) & 0x01010101u);
    r.z = (int)(__umul24((bits >> 8) & 15u, 0x00204081u) & 0x01010101u);
    r.w = (int)(__umul24((bits >> 12) & 15u, 0x00204081u) & 0x01010101u);
    return r;
}

// Workgroups are handed to the 8 XCDs round robin (b mod 8), each XCD with
// its own L2.  The product tiles are remapped so that each XCD takes a
// contiguous run of tile indices, whose neighbours share a row tile: its bit
// rows stay in that XCD's L2 instead of being fetched by all eight.  A
// bijection on the first 8 * (nb / 8) indices, the identity on the rest.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int q = nb / kXcds;
    return b < q * kXcds ? (b % kXcds) * q + b / kXcds : b;
}

__device__ __forceinline__ u32 word_of(const uint4& q, int s) {
    return s == 0 ? q.x : s == 1 ? q.y : s == 2 ? q.z : q.w;
}

// One workgroup per (upper-triangle tile pair, K split): 4 waves, each a
// 64 x 64 block of the 128 x 128 tile as 2 x 2 MFMA blocks of 32 x 32, for NP
// digit planes of eta and one plane of inter.  Bit rows are loaded 128
// h-edges at a time (4 words per row; thread t holds rows t and t + 256 of
// the tile's A rows, D rows, A columns, D columns).  For each 32 h-edges the
// threads expand their words once into bytes in shared memory (A columns as
// 0x00 / 0x7F masks, ready to be ANDed with the digit bytes), double
// buffered, and every wave reads its MFMA operands from there: the expansion
// is done once per workgroup instead of once per wave that uses a row.
// Lane l holds row (l mod 32) of its A-side block and column (l mod 32) of
// its B-side block, for the 16 h-edges 16*(l / 32) .. +15 of each 32-edge
// step; accumulator entry i is output (8*(i/4) + 4*(l/32) + i mod 4, l mod 32).
// The packed partial (eta << ib) | inter of each pair is written for both
// orientations into the split's own N x N slice.
constexpr int kRowB = 48;  // bytes per expanded row: 32 h-edges + 16 spare (conflict-free 16-byte reads)

template <int NP>
__global__ __launch_bounds__(256, NP <= 2 ? 2 : 1) void k_dense_gemm(int ntile, i32 W4, i32 wsplit, const u32* __restrict__ A,
                                                    const u32* __restrict__ D, const signed char* __restrict__ dig,
                                                    i32 Epad, u64* part, i64 Npad, int ib) {
    __shared__ __align__(16) unsigned char sx[2][4][kTile][kRowB];  // [buffer][A rows, D rows, A cols, D cols]
    __shared__ uint4 sdig[2][NP][8];  // [buffer][plane][16-byte group of the 128 h-edges]
    int ti = 0, rem = xcd_tile(blockIdx.x, gridDim.x);
    while (rem >= ntile - ti) {
        rem -= ntile - ti;
        ++ti;
    }
    const int tj = ti + rem;
    const i32 wbeg = blockIdx.y * wsplit;
    const i32 wend = min(W4, wbeg + wsplit);
    const int t = threadIdx.x;
    const int wv = t >> 6, l = t & 63, lr = l & 31, kh = l >> 5;
    const int wr = (wv >> 1) * 64, wc = (wv & 1) * 64;  // the wave's block within the tile
    const i64 R0 = (i64)ti * kTile, C0 = (i64)tj * kTile;
    // thread t expands row t & 127 of matrix t >> 7 (A or D rows) and of
    // matrix 2 + (t >> 7) (A or D columns); the A-column half is waves 0-1
    const int mrow = t >> 7, rr = t & (kTile - 1);
    const bool amask = mrow == 0;
    auto src = [&](int q, i32 w) -> const uint4* {
        const int which = q >> 7, row = q & (kTile - 1);
        const u32* M = (which & 1) ? D : A;
        const i64 base = (which < 2 ? R0 : C0) + row;
        return (const uint4*)&M[base * W4 + w];
    };
    v16i acc[NP + 1][2][2];
#pragma unroll
    for (int p = 0; p <= NP; ++p)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int i = 0; i < 16; ++i) acc[p][a][b][i] = 0;
    uint4 x0 = make_uint4(0u, 0u, 0u, 0u), x1 = make_uint4(0u, 0u, 0u, 0u);
    if (wbeg < wend) {
        x0 = *src(t, wbeg);
        x1 = *src(t + 256, wbeg);
        if (t < NP * 8) sdig[0][t >> 3][t & 7] = *(const uint4*)&dig[(i64)(t >> 3) * Epad + (i64)wbeg * 32 + (t & 7) * 16];
    }
    int dcur = 0, buf = 0;
    for (i32 w = wbeg; w < wend; w += 4) {
        const bool more = w + 4 < wend;
        uint4 y0 = x0, y1 = x1, yd = make_uint4(0u, 0u, 0u, 0u);
        if (more) {
            y0 = *src(t, w + 4);
            y1 = *src(t + 256, w + 4);
            if (t < NP * 8) yd = *(const uint4*)&dig[(i64)(t >> 3) * Epad + (i64)(w + 4) * 32 + (t & 7) * 16];
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            {  // expand word s of the thread's two rows
                const u32 wa = word_of(x0, s), wb = word_of(x1, s);
                const v4i e0 = spread16(wa & 0xFFFFu), e1 = spread16(wa >> 16);
                v4i f0 = spread16(wb & 0xFFFFu), f1 = spread16(wb >> 16);
                if (amask) {
                    f0 = digit_mask(f0);
                    f1 = digit_mask(f1);
                }
                *(v4i*)&sx[buf][mrow][rr][0] = e0;
                *(v4i*)&sx[buf][mrow][rr][16] = e1;
                *(v4i*)&sx[buf][2 + mrow][rr][0] = f0;
                *(v4i*)&sx[buf][2 + mrow][rr][16] = f1;
            }
            __syncthreads();
            v4i fa[2], mk[2];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                fa[b] = *(const v4i*)&sx[buf][0][wr + b * 32 + lr][kh * 16];
                mk[b] = *(const v4i*)&sx[buf][2][wc + b * 32 + lr][kh * 16];
            }
#pragma unroll
            for (int p = 0; p < NP; ++p) {  // eta planes: digit-masked columns, one plane at a time
                const uint4 q = sdig[dcur][p][2 * s + kh];
                const v4i dg = v4i{(int)q.x, (int)q.y, (int)q.z, (int)q.w};
                const v4i fb0 = mk[0] & dg, fb1 = mk[1] & dg;
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    acc[p][a][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[a], fb0, acc[p][a][0], 0, 0, 0);
                    acc[p][a][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[a], fb1, acc[p][a][1], 0, 0, 0);
                }
            }
            {  // inter
                v4i fd[2], fdc[2];
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    fd[b] = *(const v4i*)&sx[buf][1][wr + b * 32 + lr][kh * 16];
                    fdc[b] = *(const v4i*)&sx[buf][3][wc + b * 32 + lr][kh * 16];
                }
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
                        acc[NP][a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fd[a], fdc[b], acc[NP][a][b], 0, 0, 0);
            }
            buf ^= 1;
        }
        // the next chunk's digits: read after the next expansion's barrier;
        // the other buffer's last readers passed this chunk's barriers
        if (more & (t < NP * 8)) sdig[dcur ^ 1][t >> 3][t & 7] = yd;
        dcur ^= 1;
        x0 = y0;
        x1 = y1;
    }
    const i64 r0 = R0 + wr, c0 = C0 + wc;
    u64* out = part + (i64)blockIdx.y * Npad * Npad;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const i64 r = r0 + a * 32 + 8 * (i / 4) + 4 * kh + (i % 4);
                const i64 c = c0 + b * 32 + lr;
                u64 eta = 0;
#pragma unroll
                for (int p = 0; p < NP; ++p) eta += (u64)(u32)acc[p][a][b][i] << (7 * p);
                const u64 v = (eta << ib) | (u64)(u32)acc[NP][a][b][i];
                out[r * Npad + c] = v;
                out[c * Npad + r] = v;
            }
}

// ---- In-isolation moves on small levels (Sec. VI-B) --------------------------
// conn(n,p) = sum of w(e) over e in I(n) with pins(p,e) > 0 is the product
// H diag(w) B^T of the node incidence H (N x E bits) and the partition
// presence B (P x E bits, bit (p,e) set iff pins(p,e) > 0, stored word-major), computed exactly
// with int8 MFMA over 7-bit digit planes of w.  The saving of n comes from
// one byte per pin slot (pins(rho(m),e) = 1, from the Phi kernel) summed over
// n's incidence; the moves are then chosen from each node's dense row by the
// sparse kernel's rules.

// B stored word-major, Bt[w][p] = bits of h-edges 32w .. 32w+31 for
// partition p: one block per word column collects its 32 h-edges' Phi rows in
// shared memory (Ppad words) and writes the column with coalesced stores.
__global__ __launch_bounds__(256) void k_part_bits(i32 E, i32 W4, i32 Ppad, const i64* __restrict__ he_off,
                                                   const i32* __restrict__ len, const i32* __restrict__ part, u32* Bt) {
    extern __shared__ u32 words[];  // Ppad
    const int lane = lane_id(), nwv = blockDim.x / kWave;
    for (i32 w = blockIdx.x; w < W4; w += gridDim.x) {
        for (int p = threadIdx.x; p < Ppad; p += blockDim.x) words[p] = 0u;
        __syncthreads();
        for (int j = wave_id(); j < 32; j += nwv) {
            const i64 e = (i64)w * 32 + j;
            if (e >= E) continue;
            const i64 a = he_off[e];
            const i32 L = len[e];
            for (i32 r = lane; r < L; r += kWave) atomicOr(&words[part[a + r]], 1u << j);
        }
        __syncthreads();
        for (int p = threadIdx.x; p < Ppad; p += blockDim.x) Bt[(i64)w * Ppad + p] = words[p];
        __syncthreads();
    }
}

// W_I(n) = sum of w(e) over I(n) and the saving of n, one wave per node.
__global__ __launch_bounds__(256) void k_saving(i32 N, const i64* __restrict__ inc_off, const i32* __restrict__ inc,
                                                const i32* __restrict__ inc_pos, const i32* __restrict__ hw,
                                                const unsigned char* __restrict__ single, i64* wi, i64* sav) {
    const int lane = lane_id(), wpb = blockDim.x / kWave;
    for (i64 n = (i64)blockIdx.x * wpb + wave_id(); n < N; n += (i64)gridDim.x * wpb) {
        const i64 s0 = inc_off[n], s1 = inc_off[n + 1];
        i64 w = 0, sv = 0;
        for (i64 i0 = s0; i0 < s1; i0 += 4 * kWave) {
            i32 ww[4], ss[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const i64 i = i0 + u * kWave + lane;
                const int in = (int)(i < s1);
                ww[u] = in ? hw[inc[i]] : 0;
                ss[u] = in ? (i32)single[inc_pos[i]] : 0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                w += ww[u];
                sv += ss[u] ? ww[u] : 0;
            }
        }
        w = wave_sum(w);
        sv = wave_sum(sv);
        if (lane == 0) {
            wi[n] = w;
            sav[n] = sv;
        }
    }
}

// One workgroup per (node tile, partition tile, K split), 4 waves of 64 x 64
// as in k_dense_gemm: node rows expanded to 0/1 bytes, partition rows (B
// word-major) to 0x00 / 0x7F masks ANDed with the weight digits, once per
// workgroup per 32 h-edges in shared memory.  Writes conn partials (int32) of
// the split.
template <int NP>
__global__ __launch_bounds__(256, 2) void k_conn_gemm(int ntile_p, i32 W4, i32 wsplit, const u32* __restrict__ A,
                                                      const u32* __restrict__ B, const signed char* __restrict__ dig,
                                                      i32 Epad, i32* out, i64 Npad, i64 Ppad) {
    __shared__ __align__(16) unsigned char sx[2][2][kTile][kRowB];  // [buffer][node rows, partition rows]
    __shared__ uint4 sdig[2][NP][8];
    const int tb = xcd_tile(blockIdx.x, gridDim.x);
    const int ti = tb / ntile_p, tj = tb % ntile_p;
    const i32 wbeg = blockIdx.y * wsplit;
    const i32 wend = min(W4, wbeg + wsplit);
    const int t = threadIdx.x;
    const int wv = t >> 6, l = t & 63, lr = l & 31, kh = l >> 5;
    const int wr = (wv >> 1) * 64, wc = (wv & 1) * 64;
    const i64 R0 = (i64)ti * kTile, C0 = (i64)tj * kTile;
    const int mrow = t >> 7, rr = t & (kTile - 1);  // thread t expands row rr of matrix mrow
    // node rows are row-major (4 words per 16-byte load), partition rows are
    // word-major (Bt[w][p], 4 loads of 4 bytes)
    const u32* arow = &A[(R0 + rr) * W4];
    const u32* bcol = &B[C0 + rr];
    auto load4 = [&](i32 w) -> uint4 {
        if (mrow == 0) return *(const uint4*)&arow[w];
        return make_uint4(bcol[(i64)w * Ppad], bcol[(i64)(w + 1) * Ppad], bcol[(i64)(w + 2) * Ppad],
                          bcol[(i64)(w + 3) * Ppad]);
    };
    v16i acc[NP][2][2];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int i = 0; i < 16; ++i) acc[p][a][b][i] = 0;
    uint4 x = make_uint4(0u, 0u, 0u, 0u);
    if (wbeg < wend) {
        x = load4(wbeg);
        if (t < NP * 8) sdig[0][t >> 3][t & 7] = *(const uint4*)&dig[(i64)(t >> 3) * Epad + (i64)wbeg * 32 + (t & 7) * 16];
    }
    int dcur = 0, buf = 0;
    for (i32 w = wbeg; w < wend; w += 4) {
        const bool more = w + 4 < wend;
        uint4 y = x, yd = make_uint4(0u, 0u, 0u, 0u);
        if (more) {
            y = load4(w + 4);
            if (t < NP * 8) yd = *(const uint4*)&dig[(i64)(t >> 3) * Epad + (i64)(w + 4) * 32 + (t & 7) * 16];
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            {
                const u32 wd = word_of(x, s);
                v4i e0 = spread16(wd & 0xFFFFu), e1 = spread16(wd >> 16);
                if (mrow) {
                    e0 = digit_mask(e0);
                    e1 = digit_mask(e1);
                }
                *(v4i*)&sx[buf][mrow][rr][0] = e0;
                *(v4i*)&sx[buf][mrow][rr][16] = e1;
            }
            __syncthreads();
            v4i fa[2], mk[2];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                fa[b] = *(const v4i*)&sx[buf][0][wr + b * 32 + lr][kh * 16];
                mk[b] = *(const v4i*)&sx[buf][1][wc + b * 32 + lr][kh * 16];
            }
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const uint4 q = sdig[dcur][p][2 * s + kh];
                const v4i dg = v4i{(int)q.x, (int)q.y, (int)q.z, (int)q.w};
                const v4i fb0 = mk[0] & dg, fb1 = mk[1] & dg;
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    acc[p][a][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[a], fb0, acc[p][a][0], 0, 0, 0);
                    acc[p][a][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[a], fb1, acc[p][a][1], 0, 0, 0);
                }
            }
            buf ^= 1;
        }
        if (more & (t < NP * 8)) sdig[dcur ^ 1][t >> 3][t & 7] = yd;
        dcur ^= 1;
        x = y;
    }
    i32* o = out + (i64)blockIdx.y * Npad * Ppad;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const i64 r = R0 + wr + a * 32 + 8 * (i / 4) + 4 * kh + (i % 4);
                const i64 c = C0 + wc + b * 32 + lr;
                u32 v = 0;
#pragma unroll
                for (int p = 0; p < NP; ++p) v += (u32)acc[p][a][b][i] << (7 * p);
                o[r * Ppad + c] = (i32)v;
            }
}

// Moves from the dense conn rows, one block per node: gain(n,p) = conn(n,p) -
// (W_I(n) - saving(n)) for p != rho(n), positive gains only, ties to the
// larger id; the second variant keeps size(n) + size(p) <= Omega.
__global__ __launch_bounds__(256) void k_conn_select(i32 N, i32 nparts, int ksplit, const i32* __restrict__ part,
                                                     i64 Npad, i64 Ppad, const i64* __restrict__ wi,
                                                     const i64* __restrict__ sav, const i32* __restrict__ rho,
                                                     const i32* __restrict__ nw, const i64* __restrict__ psize,
                                                     i64 omega, i32* move_dst, i64* move_gain, i32* move_dst_sa,
                                                     i64* move_gain_sa) {
    __shared__ i64 red_g[16], red_g2[16];
    __shared__ i32 red_p[16], red_p2[16];
    const int lane = lane_id(), wv = wave_id(), nwv = blockDim.x / kWave;
    for (i32 n = blockIdx.x; n < N; n += gridDim.x) {
        const i32 ps = rho[n];
        const i64 need = wi[n] - sav[n];
        const i64 nw_n = nw[n];
        i64 bg = 0, bg2 = 0;
        i32 bp = -1, bp2 = -1;
        const i32* row = part + (i64)n * Ppad;
        for (i32 p = threadIdx.x; p < nparts; p += blockDim.x) {
            i64 v = 0;
            for (int k = 0; k < ksplit; ++k) v += (i64)row[(i64)k * Npad * Ppad + p];
            if ((int)(p == ps) | (int)(v <= need)) continue;
            const i64 g = v - need;
            const int fits = (int)(nw_n + psize[p] <= omega);
            const bool t = lex_better(g, p, bg, bp);
            bg = t ? g : bg;
            bp = t ? p : bp;
            const bool t2 = (fits & (int)lex_better(g, p, bg2, bp2)) != 0;
            bg2 = t2 ? g : bg2;
            bp2 = t2 ? p : bp2;
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
            for (int w = 1; w < nwv; ++w) {
                const i64 g2 = rg[w];
                const i32 p2 = rpp[w];
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

// Candidate selection from the dense rows, one block per node, with the
// histogram kernel's selection (top_select.h): the same pruning bound, queue,
// validity rules and block merge.
template <int PI>
__global__ __launch_bounds__(256) void k_dense_select(i32 N, i64 Npad, int ksplit, const u64* __restrict__ part,
                                                      const i32* __restrict__ inc_nin, const i32* __restrict__ nw,
                                                      i64 omega, i64 delta, u64 seed,
                                                      const unsigned long long* __restrict__ stats, int ib,
                                                      i32* cand, u64* score) {
    __shared__ u64 red_s[16];
    __shared__ i32 red_m[16];
    __shared__ SelQueue<u64> selq[4];
    __shared__ unsigned long long s_floor;
    SelNode sn;
    sn.seed = seed;
    sn.cap = stats[4];
    sn.ndiv.m = stats[8];
    sn.ndiv.sh1 = (u32)stats[9];
    sn.ndiv.sh2 = (u32)(stats[9] >> 32);
    sn.ndiv.d = stats[10];
    sn.ib = ib;
    sn.omega = omega;
    sn.delta = delta;
    sn.nw = nw;
    sn.inc_nin = inc_nin;
    sn.floor = &s_floor;
    sn.union_floor = 0;  // dense rows fill the lane lists with high scores early: the bound would not pay
    const int wv = wave_id();
    for (i32 n = blockIdx.x; n < N; n += gridDim.x) {
        sn.n = n;
        sn.nin_n = inc_nin[n];
        sn.nw_n = nw[n];
        sn.all_valid = (int)(sn.nw_n + (i64)stats[11] <= omega) & (int)((i64)sn.nin_n + (i64)stats[1] <= delta);
        if (threadIdx.x == 0) s_floor = 0;
        __syncthreads();
        TopList<PI> top;
        top.clear();
        u32 qh = 0, qn = 0;
        const u64* rowp = part + (i64)n * Npad;
        for (i32 s0 = 0; s0 < N; s0 += kSelU * (i32)blockDim.x) {
            u64 vv[kSelU];
#pragma unroll
            for (int u = 0; u < kSelU; ++u) {
                const i32 m = s0 + u * (i32)blockDim.x + (i32)threadIdx.x;
                const int in = (int)(m < N) & (int)(m != n);
                u64 v = 0;
                for (int k = 0; k < ksplit; ++k) v += in ? rowp[(i64)k * Npad * Npad + m] : 0ull;
                vv[u] = v;
            }
            const u64 vmin = sel_vmin<u64, PI>(top, sn);
#pragma unroll
            for (int u = 0; u < kSelU; ++u)
                sel_push(selq[wv], qh, qn, (int)(vv[u] >= vmin), s0 + u * (i32)blockDim.x + (i32)threadIdx.x, vv[u],
                         top, sn);
        }
        sel_flush(selq[wv], qh, qn, top, sn);
        __syncthreads();
        sel_merge(top, red_s, red_m, cand + (i64)n * PI, score + (i64)n * PI);
    }
}

}  // namespace

int dense_planes(u64 max_t) {
    int p = 1;
    while (p <= kMaxPlanes && (max_t >> (7 * p)) != 0) ++p;
    return p <= kMaxPlanes ? p : 0;
}

bool dense_proposal_fits(i32 N, i32 E, u64 max_t) {
    return N >= 2 && E >= 1 && E <= (1 << 18) && N <= 12288 && dense_planes(max_t) > 0;
}

// Estimated times of the two proposals: MFMA products over the padded
// upper triangle at 40 % of the int8 peak, against the histogram's
// Sigma |e|^2 updates at the rate it sustains on such levels.
bool prefer_dense_proposal(const Ctx* c, i32 N, i32 E, u64 max_t, u64 sum_card_sq) {
    if (!dense_proposal_fits(N, E, max_t)) return false;
    const double Npad = (double)((N + kTile - 1) / kTile * kTile);
    const double Epad = (double)(((E + 31) / 32 + 3) / 4 * 4 * 32);
    const double macs = Npad * (Npad + kTile) / 2.0 * Epad * (dense_planes(max_t) + 1);
    const double dense_s = macs / (2.5e15 * c->num_cu / 256.0 / 2.5) + 60e-6;
    const double sparse_s = (double)sum_card_sq / 4.0e11;
    return dense_s < sparse_s;
}

void propose_dense(Ctx* c, const Level& L, int Pi, const unsigned long long* stats, int ib, u64 max_t, i32* cand,
                   u64* score) {
    const i32 N = L.N, E = L.E;
    const int NP = dense_planes(max_t);
    const i32 Npad = (N + kTile - 1) / kTile * kTile;
    const i32 W4 = ((E + 31) / 32 + 3) / 4 * 4;
    const i32 Epad = W4 * 32;
    u32* A = wsp<u32>(c, WS_DN_A, (size_t)Npad * W4);
    u32* D = wsp<u32>(c, WS_DN_D, (size_t)Npad * W4);
    signed char* dig = wsp<signed char>(c, WS_DN_DIG, (size_t)NP * Epad);
    LAUNCH(c, KF_PROPOSE_DENSE, k_dense_bits, std::min<i64>(Npad, (i64)c->num_cu * 8), 256, sizeof(u32) * 2 * W4, N, Npad,
           W4, L.inc_off(), L.inc_nin(), L.inc(), A, D);
    LAUNCH(c, KF_PROPOSE_DENSE, k_dense_digits, grid_for(Epad, 256, c->num_cu * 4), 256, 0, E, Epad, NP, L.he_off(),
           c->hw(), dig, 0);
    const int ntile = Npad / kTile;
    const int pairs = ntile * (ntile + 1) / 2;
    // K splits so that the grid covers the device a few times over
    int ksplit = std::max(1, std::min(W4 / 4, (4 * c->num_cu + pairs - 1) / pairs));
    ksplit = std::min(ksplit, 16);
    const i32 wsplit = ((W4 / 4 + ksplit - 1) / ksplit) * 4;
    ksplit = (W4 + wsplit - 1) / wsplit;
    u64* part = wsp<u64>(c, WS_DN_PART, (size_t)ksplit * Npad * Npad);
    const dim3 grid(pairs, ksplit);
    prof_add_work(c, KF_DENSE_GEMM, (i64)pairs * kTile * kTile * Epad * (NP + 1));  // int8 MACs
    switch (NP) {
        case 1:
            LAUNCH(c, KF_DENSE_GEMM, k_dense_gemm<1>, grid, 256, 0, ntile, W4, wsplit, A, D, dig, Epad, part, (i64)Npad, ib);
            break;
        case 2:
            LAUNCH(c, KF_DENSE_GEMM, k_dense_gemm<2>, grid, 256, 0, ntile, W4, wsplit, A, D, dig, Epad, part, (i64)Npad, ib);
            break;
        default:
            LAUNCH(c, KF_DENSE_GEMM, k_dense_gemm<3>, grid, 256, 0, ntile, W4, wsplit, A, D, dig, Epad, part, (i64)Npad, ib);
            break;
    }
    const int grid_s = (int)std::min<i64>(N, (i64)c->num_cu * 8);
#define HGP_DSEL(PIV)                                                                                             \
    case PIV:                                                                                                     \
        LAUNCH(c, KF_PROPOSE_DENSE, k_dense_select<PIV>, grid_s, 256, 0, N, (i64)Npad, ksplit, (const u64*)part,        \
               L.inc_nin(), L.nw(), c->omega, c->delta, c->opt.seed, stats, ib, cand, score);                    \
        break;
    switch (Pi) {
        HGP_DSEL(1) HGP_DSEL(2) HGP_DSEL(3) HGP_DSEL(4) HGP_DSEL(5) HGP_DSEL(6) HGP_DSEL(7) HGP_DSEL(8)
        default: fail(HGP_E_INVALID, "pi must be in 1..8");
    }
#undef HGP_DSEL
}

// Dense moves when the product over the padded node x partition grid at the
// measured MFMA rate (plus the bit rows, saving and selection) beats the
// sparse sweep's row visits, estimated as sum_e |e| min(|e|, P) x 0.8 at the
// rate it sustains on such levels.
bool use_dense_gains(const Ctx* c, const Level& L, i32 nparts) {
    const int planes = dense_planes((u64)c->max_hw);
    const bool fits = L.N >= 1 && L.E >= 1 && L.E <= (1 << 18) && L.N <= 12288 && nparts >= 1 && nparts <= 12288 &&
                      planes > 0;
    if (!fits || (c->opt.flags & 16)) return false;
    if (c->opt.flags & 8) return true;
    const double Npad = (double)((L.N + kTile - 1) / kTile * kTile);
    const double Ppad = (double)((nparts + kTile - 1) / kTile * kTile);
    const double Epad = (double)(((L.E + 31) / 32 + 3) / 4 * 4 * 32);
    const double dense_s = Npad * Ppad * Epad * planes / (1.0e15 * c->num_cu / 256.0) + 250e-6;
    const double avg = (double)L.P / (double)L.E;
    const double sparse_s = (double)L.P * std::min(avg, (double)nparts) * 0.8 / 1.3e12;
    return dense_s < sparse_s;
}

void gains_dense(Ctx* c, const Level& L, const i32* rho, i32 nparts, const i32* part, const i32* len,
                 const unsigned char* single, const i64* psize, i32* mdst_any, i64* mgain_any, i32* mdst_sa,
                 i64* mgain_sa) {
    const i32 N = L.N, E = L.E;
    const int NP = dense_planes((u64)c->max_hw);
    const i32 Npad = (N + kTile - 1) / kTile * kTile;
    const i32 Ppad = (nparts + kTile - 1) / kTile * kTile;
    const i32 W4 = ((E + 31) / 32 + 3) / 4 * 4;
    const i32 Epad = W4 * 32;
    u32* A = wsp<u32>(c, WS_DN_A, (size_t)Npad * W4);
    u32* B = wsp<u32>(c, WS_DG_B, (size_t)Ppad * W4);
    signed char* dig = wsp<signed char>(c, WS_DG_DIG, (size_t)NP * Epad);
    i64* wi = wsp<i64>(c, WS_DG_WI, N);
    i64* sav = wsp<i64>(c, WS_DG_SAV, N);
    LAUNCH(c, KF_GAINS, k_dense_bits, std::min<i64>(Npad, (i64)c->num_cu * 8), 256, sizeof(u32) * 2 * W4, N, Npad, W4,
           L.inc_off(), L.inc_nin(), L.inc(), A, (u32*)nullptr);
    LAUNCH(c, KF_GAINS, k_part_bits, std::min<i64>(W4, (i64)c->num_cu * 8), 256, sizeof(u32) * (size_t)Ppad, E, W4,
           Ppad, L.he_off(), len, part, B);
    LAUNCH(c, KF_GAINS, k_dense_digits, grid_for(Epad, 256, c->num_cu * 4), 256, 0, E, Epad, NP, L.he_off(), c->hw(),
           dig, 1);
    LAUNCH(c, KF_GAINS, k_saving, grid_for(N, 4, c->num_cu * 16), 256, 0, N, L.inc_off(), L.inc(), L.inc_pos(),
           c->hw(), single, wi, sav);
    const int tn = Npad / kTile, tp = Ppad / kTile;
    const int tiles = tn * tp;
    int ksplit = std::max(1, std::min(W4 / 4, (4 * c->num_cu + tiles - 1) / tiles));
    ksplit = std::min(ksplit, 16);
    const i32 wsplit = ((W4 / 4 + ksplit - 1) / ksplit) * 4;
    ksplit = (W4 + wsplit - 1) / wsplit;
    i32* out = wsp<i32>(c, WS_DN_PART, (size_t)ksplit * Npad * Ppad);
    const dim3 grid(tiles, ksplit);
    prof_add_work(c, KF_GAINS_GEMM, (i64)Npad * Ppad * Epad * NP);  // int8 MACs
    switch (NP) {
        case 1:
            LAUNCH(c, KF_GAINS_GEMM, k_conn_gemm<1>, grid, 256, 0, tp, W4, wsplit, A, B, dig, Epad, out, (i64)Npad,
                   (i64)Ppad);
            break;
        case 2:
            LAUNCH(c, KF_GAINS_GEMM, k_conn_gemm<2>, grid, 256, 0, tp, W4, wsplit, A, B, dig, Epad, out, (i64)Npad,
                   (i64)Ppad);
            break;
        default:
            LAUNCH(c, KF_GAINS_GEMM, k_conn_gemm<3>, grid, 256, 0, tp, W4, wsplit, A, B, dig, Epad, out, (i64)Npad,
                   (i64)Ppad);
            break;
    }
    LAUNCH(c, KF_GAINS, k_conn_select, (int)std::min<i64>(N, (i64)c->num_cu * 8), 256, 0, N, nparts, ksplit,
           (const i32*)out, (i64)Npad, (i64)Ppad, (const i64*)wi, (const i64*)sav, rho, L.nw(), psize, c->omega,
           mdst_any, mgain_any, mdst_sa, mgain_sa);
}

}  // namespace hgp
