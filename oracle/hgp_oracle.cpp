// Serial reference ("oracle") of the constrained multilevel hypergraph
// partitioner of "Hypergraph Partitioning on GPU with Distinct Incident
// Hyperedges and Size Constraints".
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
// CPU statement of what the HIP library computes.  Only the test suite, the
// smoke check and the benchmark's CPU-baseline leg may load it; the product
// path never does.  It shares no header, helper, table or constant with the
// HIP sources.
//
// Everything is integer.  Where the paper is silent or ambiguous the reading
// taken is named inline as "Reading Rk" and stated where it is applied.
//
// Parity status per function (what pins each one; see tests/test_oracle_*.py):
//   evaluate / phi            pinned: incidence-matrix products, closed forms,
//                             brute force over all partitions of tiny graphs
//   pair / propose            pinned: matrix-product histogram, symmetry, sort
//   match_round               pinned: brute-force maximum-weight matching
//   match_round_greedy        pinned: hand-worked proposal forests (Reading
//                             R28; an ablation, not the method)
//   contract                  pinned: score/connectivity duality, level
//                             invariance of Conn and D, size conservation
//   gain / moves              pinned: Conn difference of single moves
//   refine_rep (sequence,     pinned: C_k equals the Conn drop after k moves,
//   in-sequence gain, events) V_k equals the recomputed violation count
//   sort_moves,               pinned: hand-worked move lists whose sequence
//   sequence_moves            follows from Readings R15-R17 alone (grade
//                             terms and weights, the 256-move window, both
//                             tie-breaks, acceptance, retries, cycle start,
//                             ranking), plus the structural checks
//   isolated pairing, noise   pinned: hand-worked cases of Readings R8, R3
//   cap, k-way seating        and R21
//   partition (driver)        pinned by validity, Conn >= brute-force optimum,
//                             special cases, and the early exit against the
//                             run of all repetitions (Reading R25); the paper
//                             prints no worked example of a whole run
// tests/test_oracle_mutants.py builds single-slip copies of this file and
// checks that the pins above catch each one.

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <utility>
#include <vector>

typedef int32_t i32;
typedef int64_t i64;
typedef uint64_t u64;
typedef uint32_t u32;

namespace {

// ---------------------------------------------------------------------------
// Hypergraph (Sec. II-A) in the dual compressed layout of Sec. IV-B.
// ---------------------------------------------------------------------------
struct Graph {
    i32 N = 0, E = 0;
    std::vector<i64> he_off;   // E+1
    std::vector<i32> he_nsrc;  // E   |src(e)|, sources stored first
    std::vector<i32> pins;     // P
    std::vector<i64> hw;       // E   omega(e)
    std::vector<i64> nw;       // N   size(n)
    std::vector<i64> inc_off;  // N+1
    std::vector<i32> inc_nin;  // N   |in(n)|, inbound h-edges stored first
    std::vector<i32> inc;      // P
    i64 P() const { return he_off[E]; }
    i64 card(i32 e) const { return he_off[e + 1] - he_off[e]; }
    bool is_dst_pos(i32 e, i64 j) const { return j >= he_off[e] + he_nsrc[e]; }
};

// Incidence sets in(n), out(n) of Sec. II-A, inbound first (Sec. IV-B).
// Each block is ascending by h-edge id (Reading R11).
void build_incidence(Graph& g) {
    std::vector<std::vector<i32>> in(g.N), out(g.N);
    for (i32 e = 0; e < g.E; ++e)
        for (i64 j = g.he_off[e]; j < g.he_off[e + 1]; ++j) {
            if (g.is_dst_pos(e, j)) in[g.pins[j]].push_back(e);
            else out[g.pins[j]].push_back(e);
        }
    g.inc_off.assign(g.N + 1, 0);
    g.inc_nin.assign(g.N, 0);
    g.inc.clear();
    g.inc.reserve(g.P());
    for (i32 n = 0; n < g.N; ++n) {
        g.inc_nin[n] = (i32)in[n].size();
        g.inc.insert(g.inc.end(), in[n].begin(), in[n].end());
        g.inc.insert(g.inc.end(), out[n].begin(), out[n].end());
        g.inc_off[n + 1] = (i64)g.inc.size();
    }
}

std::string validate_and_build(Graph& g) {
    if (g.N < 1) return "need at least one node";
    if (g.E < 0) return "negative h-edge count";
    if (g.he_off[0] != 0) return "he_off[0] must be 0";
    i64 wsum = 0, nsum = 0;
    std::vector<char> mark(g.N, 0);
    for (i32 e = 0; e < g.E; ++e) {
        i64 a = g.he_off[e], b = g.he_off[e + 1];
        if (b <= a) return "empty h-edge " + std::to_string(e);
        if (g.he_nsrc[e] < 0 || g.he_nsrc[e] > b - a) return "bad source count";
        if (g.hw[e] < 1) return "h-edge weight must be >= 1";
        wsum += g.hw[e];
        for (i64 j = a; j < b; ++j) {
            i32 m = g.pins[j];
            if (m < 0 || m >= g.N) return "pin out of range";
            bool first_of_block = (j == a) || (j == a + g.he_nsrc[e]);
            if (!first_of_block && g.pins[j - 1] >= m) return "pin blocks must be strictly ascending";
            if (mark[m]) return "src(e) and dst(e) intersect";  // Sec. II-A: no self-cycles
            mark[m] = 1;
        }
        for (i64 j = a; j < b; ++j) mark[g.pins[j]] = 0;
    }
    for (i32 n = 0; n < g.N; ++n) {
        if (g.nw[n] < 1) return "node weight must be >= 1";
        nsum += g.nw[n];
    }
    if (wsum >= (i64(1) << 31)) return "total h-edge weight must be < 2^31";
    if (nsum >= (i64(1) << 31)) return "total node weight must be < 2^31";
    build_incidence(g);
    return "";
}

// ---------------------------------------------------------------------------
// Evaluation (Sec. II-B): pins(p,e), pins_in(p,e), sizes, D(p), Conn, cut-net.
// ---------------------------------------------------------------------------
struct PhiEntry { i32 part; i32 cnt; i32 cnt_in; };

// Per h-edge row of (p, pins(p,e), pins_in(p,e)) over partitions with pins(p,e)>0,
// ascending by p.
std::vector<std::vector<PhiEntry>> phi_rows(const Graph& g, const i32* rho) {
    std::vector<std::vector<PhiEntry>> rows(g.E);
    std::vector<std::pair<i32, i32>> tmp;  // (partition, is destination)
    for (i32 e = 0; e < g.E; ++e) {
        tmp.clear();
        for (i64 j = g.he_off[e]; j < g.he_off[e + 1]; ++j)
            tmp.push_back({rho[g.pins[j]], g.is_dst_pos(e, j) ? 1 : 0});
        std::sort(tmp.begin(), tmp.end());
        for (auto& t : tmp) {
            if (rows[e].empty() || rows[e].back().part != t.first) rows[e].push_back({t.first, 0, 0});
            rows[e].back().cnt += 1;
            rows[e].back().cnt_in += t.second;
        }
    }
    return rows;
}

struct Eval {
    i64 conn = 0, cutnet = 0, max_size = 0, max_inbound = 0, violations = 0, nonempty = 0;
    std::vector<i64> size, inbound;
};

Eval evaluate(const Graph& g, const i32* rho, i32 nparts, i64 omega, i64 delta) {
    Eval r;
    r.size.assign(nparts, 0);
    r.inbound.assign(nparts, 0);
    for (i32 n = 0; n < g.N; ++n) r.size[rho[n]] += g.nw[n];
    auto rows = phi_rows(g, rho);
    for (i32 e = 0; e < g.E; ++e) {
        i64 lambda = (i64)rows[e].size();
        r.conn += g.hw[e] * (lambda - 1);           // Eq. connectivity
        if (lambda > 1) r.cutnet += g.hw[e];         // Eq. cut-net
        for (auto& t : rows[e])
            if (t.cnt_in > 0) r.inbound[t.part] += 1;  // |{e : pins_in(p,e) > 0}|
    }
    for (i32 p = 0; p < nparts; ++p) {
        r.max_size = std::max(r.max_size, r.size[p]);
        r.max_inbound = std::max(r.max_inbound, r.inbound[p]);
        if (r.size[p] > omega || r.inbound[p] > delta) r.violations++;
        if (r.size[p] > 0) r.nonempty++;
    }
    return r;
}

// ---------------------------------------------------------------------------
// Coarsening: candidate proposal (Sec. V-A, V-C).
// ---------------------------------------------------------------------------

// Normalised h-edge weight omega(e)/|e| of Eq. neighbors_histogram in 16-bit
// fixed point, at least 1 so that every shared h-edge scores (Reading R2).
u64 tnorm(const Graph& g, i32 e) {
    u64 t = ((u64)g.hw[e] << 16) / (u64)g.card(e);
    return t ? t : 1;
}

// SplitMix64 output mixing function (Steele, Lea, Flood, "Fast splittable
// pseudorandom number generators", OOPSLA 2014), written from that paper.
u64 mix64(u64 z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Noise cap: 10% of the mean normalised h-edge weight over h-edges with at
// least two pins (Sec. V-C, Reading R3).
u64 noise_cap(const Graph& g) {
    u64 sum = 0, cnt = 0;
    for (i32 e = 0; e < g.E; ++e)
        if (g.card(e) >= 2) { sum += tnorm(g, e); cnt += 1; }
    return cnt ? sum / (10 * cnt) : 0;
}

// Symmetric deterministic noise rng(min(n,m), max(n,m)) (Sec. V-C, Reading R3).
u64 noise(u64 seed, i32 a, i32 b, u64 cap) {
    if (cap == 0) return 0;
    u64 lo = (u64)(u32)std::min(a, b), hi = (u64)(u32)std::max(a, b);
    return mix64(seed ^ mix64((lo << 32) | hi)) % (cap + 1);
}

// eta(n,m) and inter(n,m) straight from their definitions (Eq.
// neighbors_histogram; inter as |in(n) ∩ in(m)|, Sec. V-C).
void pair_values(const Graph& g, i32 n, i32 m, u64* eta, i32* inter) {
    u64 s = 0;
    i32 c = 0;
    for (i64 k = g.inc_off[n]; k < g.inc_off[n + 1]; ++k) {
        i32 e = g.inc[k];
        bool e_in_n = (k - g.inc_off[n]) < g.inc_nin[n];
        for (i64 j = g.he_off[e]; j < g.he_off[e + 1]; ++j)
            if (g.pins[j] == m) {
                s += tnorm(g, e);
                if (e_in_n && g.is_dst_pos(e, j)) c += 1;
            }
    }
    *eta = s;
    *inter = c;
}

struct ProposeScratch {
    std::vector<u64> eta;
    std::vector<i32> inter;
    std::vector<char> seen;
    std::vector<i32> touched;
};

// Top-Pi valid neighbours of n by (score desc, id desc): Eq. proposal_graph
// with max-id tie-break (Reading R1), Pi candidates per Sec. V-D, exact over
// all neighbours (Reading R6).  Returns the number of candidates found.
int propose_node(const Graph& g, i32 n, i64 omega, i64 delta, u64 seed, u64 cap, int Pi,
                 ProposeScratch& s, i32* cand, u64* score) {
    for (i64 k = g.inc_off[n]; k < g.inc_off[n + 1]; ++k) {
        i32 e = g.inc[k];
        bool e_in_n = (k - g.inc_off[n]) < g.inc_nin[n];
        u64 t = tnorm(g, e);
        for (i64 j = g.he_off[e]; j < g.he_off[e + 1]; ++j) {
            i32 m = g.pins[j];
            if (m == n) continue;
            if (!s.seen[m]) { s.seen[m] = 1; s.touched.push_back(m); }
            s.eta[m] += t;
            if (e_in_n && g.is_dst_pos(e, j)) s.inter[m] += 1;
        }
    }
    std::vector<std::pair<u64, i32>> valid;
    for (i32 m : s.touched) {
        bool ok_size = g.nw[n] + g.nw[m] <= omega;
        bool ok_in = (i64)g.inc_nin[n] + g.inc_nin[m] - s.inter[m] <= delta;  // Reading R4
        if (ok_size && ok_in) valid.push_back({s.eta[m] + noise(seed, n, m, cap), m});
        s.eta[m] = 0;
        s.inter[m] = 0;
        s.seen[m] = 0;
    }
    s.touched.clear();
    std::sort(valid.begin(), valid.end(), [](const std::pair<u64, i32>& a, const std::pair<u64, i32>& b) {
        return a.first != b.first ? a.first > b.first : a.second > b.second;
    });
    int found = (int)std::min<size_t>(valid.size(), (size_t)Pi);
    for (int r = 0; r < Pi; ++r) {
        cand[r] = r < found ? valid[r].second : -1;
        score[r] = r < found ? valid[r].first : 0;
    }
    return found;
}

// ---------------------------------------------------------------------------
// Maximum-weight matching on one proposal pseudo-forest (Sec. V-D).
// target[n] = -1 means undefined; active[n] = 0 removes n from the round.
// Returns "" or an error naming the broken invariant.
// ---------------------------------------------------------------------------
std::string match_round(i32 N, const char* active, const i32* target, const u64* sc, i32* match) {
    std::vector<std::vector<i32>> child(N);
    std::vector<char> paired(N, 0);
    for (i32 n = 0; n < N; ++n) {
        match[n] = -1;
        if (!active[n] || target[n] < 0) continue;
        i32 t = target[n];
        if (!active[t]) return "target of an active node is inactive";
        if (target[t] == n) paired[n] = 1;          // the set R of two-cycle roots
        else child[t].push_back(n);
    }
    // Invariant of Sec. V-A: an entering edge never outscores the leaving one.
    for (i32 n = 0; n < N; ++n)
        if (active[n] && target[n] >= 0) {
            i32 t = target[n];
            if (paired[n] && sc[n] != sc[t]) return "two-cycle with unequal scores";
            if (!paired[n] && target[t] >= 0 && sc[n] > sc[t]) return "score decreases along an edge";
        }
    std::vector<i64> A(N, 0), ss0(N, 0), ss10(N, 0), bestv(N, 0);
    std::vector<i32> bestc(N, -1);
    std::vector<char> done(N, 0);
    // Bottom-up (post-order) from every root: ss0 per Eq. ss0, the return of
    // matching with the target ss1-ss0, children outside R only.
    std::vector<std::pair<i32, size_t>> stack;
    for (i32 r = 0; r < N; ++r) {
        if (!active[r] || !(target[r] < 0 || paired[r])) continue;
        stack.push_back({r, 0});
        while (!stack.empty()) {
            auto& top = stack.back();
            i32 n = top.first;
            if (top.second < child[n].size()) {
                i32 c = child[n][top.second++];
                stack.push_back({c, 0});
                continue;
            }
            i64 a = 0;
            i64 bv = 0;
            i32 bc = -1;
            for (i32 c : child[n]) {
                a += ss0[c];
                if (bc < 0 || ss10[c] > bv || (ss10[c] == bv && c > bc)) { bv = ss10[c]; bc = c; }
            }
            A[n] = a;
            bestv[n] = bv;
            bestc[n] = bc;
            i64 take = (bc >= 0 && bv > 0) ? bv : 0;
            ss0[n] = a + take;
            ss10[n] = (target[n] >= 0 && !paired[n]) ? (i64)sc[n] - take : 0;  // Eq. ss1 minus Eq. ss0
            done[n] = 1;
            stack.pop_back();
        }
    }
    for (i32 n = 0; n < N; ++n)
        if (active[n] && !done[n]) return "cycle longer than two in the proposal graph";
    // Top-down: roots first (Eq. match_root), then every node whose parent did
    // not take it picks its best child if that improves the score (Eq. match,
    // Reading R7).
    std::vector<i32> order;
    for (i32 r = 0; r < N; ++r) {
        if (!active[r] || !(target[r] < 0 || paired[r])) continue;
        if (paired[r]) {
            i32 m = target[r];
            if (r < m) {
                i64 ss1 = (i64)sc[r] + A[r] + A[m];  // Eq. ss1_roots
                if (ss1 > ss0[r] + ss0[m]) { match[r] = m; match[m] = r; }
            }
        }
        order.push_back(r);
    }
    for (size_t i = 0; i < order.size(); ++i) {
        i32 n = order[i];
        if (match[n] < 0 && bestc[n] >= 0 && bestv[n] > 0) {
            match[n] = bestc[n];
            match[bestc[n]] = n;
        }
        for (i32 c : child[n]) order.push_back(c);
    }
    return "";
}

// The prototype's greedy matching, the ablation of Sec. VII-D (Reading R28):
// every two-cycle of the proposal graph is matched, and the decision is
// carried down the trees from the roots: a node left unmatched by its parent
// (or a root without a partner) takes the child that proposes to it with the
// highest score, ties to the larger id.
std::string match_round_greedy(i32 N, const char* active, const i32* target, const u64* sc, i32* match) {
    std::vector<std::vector<i32>> child(N);
    std::vector<char> paired(N, 0);
    for (i32 n = 0; n < N; ++n) {
        match[n] = -1;
        if (!active[n] || target[n] < 0) continue;
        i32 t = target[n];
        if (!active[t]) return "target of an active node is inactive";
        if (target[t] == n) paired[n] = 1;
        else child[t].push_back(n);
    }
    std::vector<i32> order;
    for (i32 r = 0; r < N; ++r) {
        if (!active[r] || !(target[r] < 0 || paired[r])) continue;
        if (paired[r]) match[r] = target[r];
        order.push_back(r);
    }
    for (size_t i = 0; i < order.size(); ++i) {
        i32 n = order[i];
        if (match[n] < 0) {
            i32 bc = -1;
            for (i32 c : child[n])
                if (bc < 0 || sc[c] > sc[bc] || (sc[c] == sc[bc] && c > bc)) bc = c;
            if (bc >= 0) {
                match[n] = bc;
                match[bc] = n;
            }
        }
        for (i32 c : child[n]) order.push_back(c);
    }
    if ((i64)order.size() != std::count(active, active + N, (char)1))
        return "cycle longer than two in the proposal graph";
    return "";
}

// Pi matching rounds, matched nodes leaving all later rounds (Sec. V-D), then
// best-effort pairing of nodes with no valid neighbour (Sec. V-C, Reading R8).
// greedy: the prototype's matching of each round instead of the exact one.
std::string match_all(const Graph& g, i64 omega, i64 delta, int Pi, const i32* cand, const u64* score,
                      i32* match, i32* round_pairs, bool greedy = false) {
    i32 N = g.N;
    std::vector<char> U(N, 1);
    std::vector<i32> t(N), mr(N);
    std::vector<u64> s(N);
    for (i32 n = 0; n < N; ++n) match[n] = -1;
    for (int r = 0; r < Pi; ++r) {
        for (i32 n = 0; n < N; ++n) {
            i32 c = cand[(i64)n * Pi + r];
            t[n] = (U[n] && c >= 0 && U[c]) ? c : -1;
            s[n] = score[(i64)n * Pi + r];
        }
        std::string err = greedy ? match_round_greedy(N, U.data(), t.data(), s.data(), mr.data())
                                 : match_round(N, U.data(), t.data(), s.data(), mr.data());
        if (!err.empty()) return err + " (round " + std::to_string(r) + ")";
        i32 pairs = 0;
        for (i32 n = 0; n < N; ++n)
            if (mr[n] >= 0) {
                match[n] = mr[n];
                U[n] = 0;
                if (n < mr[n]) pairs++;
            }
        if (round_pairs) round_pairs[r] = pairs;
    }
    // Isolated nodes: sorted by (size, id); pair the smallest remaining with the
    // largest that fits both caps, the Delta check using |in|+|in| (Reading R8).
    std::vector<i32> iso;
    for (i32 n = 0; n < N; ++n)
        if (cand[(i64)n * Pi] < 0) {
            if (!U[n]) return "isolated node already matched";
            iso.push_back(n);
        }
    std::sort(iso.begin(), iso.end(), [&](i32 a, i32 b) {
        return g.nw[a] != g.nw[b] ? g.nw[a] < g.nw[b] : a < b;
    });
    i32 pairs = 0;
    i64 i = 0, j = (i64)iso.size() - 1;
    while (i < j) {
        i32 a = iso[i], b = iso[j];
        if (g.nw[a] + g.nw[b] <= omega && (i64)g.inc_nin[a] + g.inc_nin[b] <= delta) {
            match[a] = b;
            match[b] = a;
            pairs++;
            i++;
            j--;
        } else {
            j--;
        }
    }
    if (round_pairs) round_pairs[Pi] = pairs;
    return "";
}

// ---------------------------------------------------------------------------
// Coarse hypergraph construction (Sec. III, Sec. V-E).
// ---------------------------------------------------------------------------
// gamma: clusters {n, match(n)}; coarse id = rank of the cluster's smallest
// member (Reading R9).  H-edges keep id and weight, none merged or dropped
// (Reading R10).  dst' = gamma(dst), src' = gamma(src) \ dst' (Sec. V-E).
Graph contract(const Graph& g, const i32* match, i32* gamma) {
    Graph c;
    std::vector<i32> cid(g.N, -1);
    i32 nc = 0;
    for (i32 n = 0; n < g.N; ++n)
        if (match[n] < 0 || match[n] > n) cid[n] = nc++;
    for (i32 n = 0; n < g.N; ++n) gamma[n] = cid[(match[n] < 0 || match[n] > n) ? n : match[n]];
    c.N = nc;
    c.E = g.E;
    c.nw.assign(nc, 0);
    for (i32 n = 0; n < g.N; ++n) c.nw[gamma[n]] += g.nw[n];
    c.hw = g.hw;
    c.he_off.assign(g.E + 1, 0);
    c.he_nsrc.assign(g.E, 0);
    for (i32 e = 0; e < g.E; ++e) {
        std::vector<i32> src, dst;
        for (i64 j = g.he_off[e]; j < g.he_off[e + 1]; ++j)
            (g.is_dst_pos(e, j) ? dst : src).push_back(gamma[g.pins[j]]);
        std::sort(dst.begin(), dst.end());
        dst.erase(std::unique(dst.begin(), dst.end()), dst.end());
        std::sort(src.begin(), src.end());
        src.erase(std::unique(src.begin(), src.end()), src.end());
        std::vector<i32> src2;
        for (i32 x : src)
            if (!std::binary_search(dst.begin(), dst.end(), x)) src2.push_back(x);
        c.he_nsrc[e] = (i32)src2.size();
        c.pins.insert(c.pins.end(), src2.begin(), src2.end());
        c.pins.insert(c.pins.end(), dst.begin(), dst.end());
        c.he_off[e + 1] = (i64)c.pins.size();
    }
    build_incidence(c);
    return c;
}

// ---------------------------------------------------------------------------
// Refinement (Sec. VI).
// ---------------------------------------------------------------------------
struct Move { i32 n, ps, pd; i64 gain; };

struct RepOut {
    std::vector<i32> seq;     // movers in sequence order
    std::vector<i32> seq_pd;  // their destinations
    std::vector<i64> gseq;    // in-sequence gain of each
    std::vector<i64> C;       // C[k] = cumulative in-sequence gain after k moves (C[0]=0)
    std::vector<i64> V;       // V[k] = violated partitions after k moves
    std::vector<i32> chain_len;
    i64 kstar = 0;
    i64 applied_gain = 0;
    i32 links = 0, rounds = 0;
};

// In-isolation move of every node: Eq. refinement_move_selection over p != rho(n)
// with gain > 0 (Reading R14), max-id tie-break, size-aware in the second half
// of the repetitions (Sec. VI-B, Reading R13).
std::vector<Move> propose_moves(const Graph& g, const i32* rho, i32 nparts, int rep, int theta, i64 omega,
                                const std::vector<std::vector<PhiEntry>>& rows, const std::vector<i64>& psize) {
    std::vector<Move> mv;
    std::vector<i64> conn(nparts, 0);
    std::vector<char> seen(nparts, 0);
    std::vector<i32> touched;
    bool size_aware = rep >= theta / 2;
    for (i32 n = 0; n < g.N; ++n) {
        i32 ps = rho[n];
        i64 saving = 0, wi = 0;
        for (i64 k = g.inc_off[n]; k < g.inc_off[n + 1]; ++k) {
            i32 e = g.inc[k];
            wi += g.hw[e];
            for (auto& t : rows[e]) {
                if (t.part == ps) {
                    if (t.cnt == 1) saving += g.hw[e];
                } else {
                    if (!seen[t.part]) { seen[t.part] = 1; touched.push_back(t.part); }
                    conn[t.part] += g.hw[e];
                }
            }
        }
        i64 best_g = 0;
        i32 best_p = -1;
        for (i32 p : touched) {
            i64 gain = saving - (wi - conn[p]);  // loss(n,p) = wi - conn[p]
            bool ok = !size_aware || g.nw[n] + psize[p] <= omega;
            if (ok && gain > 0 && (best_p < 0 || gain > best_g || (gain == best_g && p > best_p))) {
                best_g = gain;
                best_p = p;
            }
            conn[p] = 0;
            seen[p] = 0;
        }
        touched.clear();
        if (best_p >= 0) mv.push_back({n, ps, best_p, best_g});
    }
    return mv;
}

// Moves sorted by (p_s asc, gain desc) (Sec. VI-C), then node id asc
// (Reading R15).
void sort_moves(std::vector<Move>& mv) {
    std::sort(mv.begin(), mv.end(), [](const Move& a, const Move& b) {
        if (a.ps != b.ps) return a.ps < b.ps;
        if (a.gain != b.gain) return a.gain > b.gain;
        return a.n < b.n;
    });
}

// Order of the moves after chaining (Sec. VI-C): `order` lists indices into
// the sorted moves chain by chain, chain_len the length of each chain.
struct Sequence {
    std::vector<i64> order;
    std::vector<i32> chain_len;
    i32 links = 0, rounds = 0;
};

// Chain rounds and ranking over the sorted moves `mv` (Sec. VI-C, Readings
// R16 and R17); nw and nin are the node sizes and |in(n)| the grade uses.
Sequence sequence_moves(const std::vector<Move>& mv, const i64* nw, const i32* nin, int chain_rounds) {
    const i64 M = (i64)mv.size();
    Sequence out;
    std::map<i32, std::pair<i64, i64>> seg;  // part -> [begin, end) in sorted order
    for (i64 i = 0; i < M; ++i) {
        auto it = seg.find(mv[i].ps);
        if (it == seg.end()) seg[mv[i].ps] = {i, i + 1};
        else it->second.second = i + 1;
    }
    // Chain rounds (Reading R16): synchronous; every move without a successor
    // grades the first 256 predecessor-less moves leaving its destination and
    // proposes the lexicographic max of (grade, node id); a successor accepts
    // the max of (grade, proposer id).  Grade = 10^7 x the paper's grade.
    // chain_rounds = 0 is the ablation without chaining (Sec. VII): every move
    // is a chain of its own, so the sequence orders moves by gain alone.
    std::vector<i64> pred(M, -1), succ(M, -1);
    const int kWindow = 256, kRounds = chain_rounds;
    for (int round = 0; round < kRounds; ++round) {
        std::vector<i64> prop(M, -1), propG(M, 0);
        for (i64 i = 0; i < M; ++i) {
            if (succ[i] != -1) continue;
            auto it = seg.find(mv[i].pd);
            if (it == seg.end()) continue;
            int seen = 0;
            i64 bj = -1, bG = 0;
            for (i64 j = it->second.first; j < it->second.second && seen < kWindow; ++j) {
                if (pred[j] != -1) continue;
                seen++;
                i32 a = mv[i].n, b = mv[j].n;
                i64 G = mv[j].gain * 10000000LL -
                        (10 * std::llabs(nw[a] - nw[b]) + std::llabs((i64)nin[a] - nin[b]));
                if (bj < 0 || G > bG || (G == bG && b > mv[bj].n)) { bj = j; bG = G; }
            }
            prop[i] = bj;
            propG[i] = bG;
        }
        std::vector<i64> acc(M, -1);
        for (i64 i = 0; i < M; ++i) {
            i64 j = prop[i];
            if (j < 0) continue;
            i64 a = acc[j];
            if (a < 0 || propG[i] > propG[a] || (propG[i] == propG[a] && mv[i].n > mv[a].n)) acc[j] = i;
        }
        i32 links = 0;
        for (i64 j = 0; j < M; ++j)
            if (acc[j] >= 0) { succ[acc[j]] = j; pred[j] = acc[j]; links++; }
        out.rounds = round + 1;
        out.links += links;
        if (links == 0) break;
    }
    // Chains: paths head to tail, cycles from their smallest node id; ranked by
    // (total in-isolation gain desc, first node id asc) (Reading R17).
    struct Chain { i64 gain; i32 first; std::vector<i64> items; };
    std::vector<Chain> chains;
    std::vector<char> vis(M, 0);
    for (i64 i = 0; i < M; ++i) {
        if (pred[i] != -1) continue;
        Chain c{0, mv[i].n, {}};
        for (i64 j = i; j != -1; j = succ[j]) { vis[j] = 1; c.items.push_back(j); c.gain += mv[j].gain; }
        chains.push_back(std::move(c));
    }
    for (i64 i = 0; i < M; ++i) {
        if (vis[i]) continue;
        std::vector<i64> cyc;
        i64 j = i;
        do { vis[j] = 1; cyc.push_back(j); j = succ[j]; } while (j != i);
        size_t at = 0;
        for (size_t q = 1; q < cyc.size(); ++q) if (mv[cyc[q]].n < mv[cyc[at]].n) at = q;
        Chain c{0, mv[cyc[at]].n, {}};
        for (size_t q = 0; q < cyc.size(); ++q) {
            i64 x = cyc[(at + q) % cyc.size()];
            c.items.push_back(x);
            c.gain += mv[x].gain;
        }
        chains.push_back(std::move(c));
    }
    std::sort(chains.begin(), chains.end(), [](const Chain& a, const Chain& b) {
        return a.gain != b.gain ? a.gain > b.gain : a.first < b.first;
    });
    std::vector<i64>& order = out.order;
    for (auto& c : chains) {
        out.chain_len.push_back((i32)c.items.size());
        for (i64 x : c.items) order.push_back(x);
    }
    return out;
}

// One refinement repetition: moves, sequence of chains (Sec. VI-C), in-sequence
// gains, validity of every prefix (Sec. VI-D) and the applied prefix.
RepOut refine_rep(const Graph& g, i32* rho, i32 nparts, int rep, int theta, i64 omega, i64 delta,
                  int chain_rounds = 16) {
    RepOut out;
    auto rows = phi_rows(g, rho);
    std::vector<i64> psize(nparts, 0), D(nparts, 0);
    for (i32 n = 0; n < g.N; ++n) psize[rho[n]] += g.nw[n];
    for (i32 e = 0; e < g.E; ++e)
        for (auto& t : rows[e]) if (t.cnt_in > 0) D[t.part] += 1;

    std::vector<Move> mv = propose_moves(g, rho, nparts, rep, theta, omega, rows, psize);
    sort_moves(mv);
    const i64 M = (i64)mv.size();
    Sequence sq = sequence_moves(mv, g.nw.data(), g.inc_nin.data(), chain_rounds);
    const std::vector<i64>& order = sq.order;
    out.chain_len = sq.chain_len;
    out.links = sq.links;
    out.rounds = sq.rounds;
    // Simulation of the sequence: the exact connectivity change of each move
    // after all earlier ones (Reading R18), and the violated-partition count
    // after every prefix (Sec. VI-D, Reading R19).
    std::vector<std::vector<PhiEntry>>& cur = rows;  // updated in place from here on
    auto entry = [&](i32 e, i32 p) -> PhiEntry& {
        for (auto& t : cur[e]) if (t.part == p) return t;
        cur[e].push_back({p, 0, 0});
        return cur[e].back();
    };
    auto invalid = [&](i32 p) { return psize[p] > omega || D[p] > delta; };
    i64 V = 0;
    for (i32 p = 0; p < nparts; ++p) V += invalid(p) ? 1 : 0;
    out.C.push_back(0);
    out.V.push_back(V);
    i64 C = 0, bestC = 0, bestK = 0;
    for (i64 i = 0; i < M; ++i) {
        const Move& m = mv[order[i]];
        i32 n = m.n, ps = m.ps, pd = m.pd;
        i64 before = (invalid(ps) ? 1 : 0) + (invalid(pd) ? 1 : 0);
        i64 gs = 0;
        for (i64 k = g.inc_off[n]; k < g.inc_off[n + 1]; ++k) {
            i32 e = g.inc[k];
            bool e_in_n = (k - g.inc_off[n]) < g.inc_nin[n];
            PhiEntry& d = entry(e, pd);  // may grow the row: take it before s
            PhiEntry& s = entry(e, ps);
            if (s.cnt == 1) gs += g.hw[e];
            if (d.cnt == 0) gs -= g.hw[e];
            s.cnt -= 1;
            d.cnt += 1;
            if (e_in_n) {
                if (s.cnt_in == 1) D[ps] -= 1;
                if (d.cnt_in == 0) D[pd] += 1;
                s.cnt_in -= 1;
                d.cnt_in += 1;
            }
        }
        psize[ps] -= g.nw[n];
        psize[pd] += g.nw[n];
        V += (invalid(ps) ? 1 : 0) + (invalid(pd) ? 1 : 0) - before;
        C += gs;
        out.seq.push_back(n);
        out.seq_pd.push_back(pd);
        out.gseq.push_back(gs);
        out.C.push_back(C);
        out.V.push_back(V);
        if (V == 0 && C > bestC) { bestC = C; bestK = i + 1; }
    }
    // Apply the valid prefix of largest cumulative gain, the shortest on ties.
    for (i64 i = 0; i < bestK; ++i) rho[out.seq[i]] = out.seq_pd[i];
    out.kstar = bestK;
    out.applied_gain = bestC;
    return out;
}

// ---------------------------------------------------------------------------
// Multilevel driver (Sec. III) and the k-way adapter (Sec. VII-A).
// ---------------------------------------------------------------------------
// early_exit: bit 0 = Reading R25's early exit of repetitions; bit 1 = the
// ablation without chain rounds; bit 2 = the ablation with the prototype's
// greedy matching (Reading R28).
struct Params { i64 omega, delta; i32 k, Pi, Theta; u64 seed; int early_exit; };

struct LevelLog {
    i64 N, E, P;
    i32 pairs[17];
    double t_coarsen, t_refine;
    i64 conn_after;  // Conn after refinement at this level
    i64 moves_applied;
};

struct Result {
    std::vector<Graph> levels;
    std::vector<std::vector<i32>> gamma;   // gamma[l]: level l -> level l+1
    std::vector<std::vector<i32>> rho;     // rho after refining level l
    std::vector<std::vector<i32>> cand;    // proposal of level l (kept for parity)
    std::vector<std::vector<u64>> score;
    std::vector<std::vector<i32>> match;
    std::vector<LevelLog> log;
    i32 nparts = 0;
    std::string err;
};

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Initial k-way partition of the coarsest nodes (Reading R21): nodes by
// (size desc, id asc), each into the part of smallest (weight, id) that keeps
// both caps.
std::string kway_initial(const Graph& g, i32 k, i64 omega, i64 delta, std::vector<i32>& rho) {
    std::vector<i32> order(g.N);
    for (i32 n = 0; n < g.N; ++n) order[n] = n;
    std::sort(order.begin(), order.end(), [&](i32 a, i32 b) {
        return g.nw[a] != g.nw[b] ? g.nw[a] > g.nw[b] : a < b;
    });
    std::vector<i64> pw(k, 0), D(k, 0);
    std::vector<std::vector<char>> has(k, std::vector<char>(g.E, 0));
    rho.assign(g.N, -1);
    for (i32 n : order) {
        std::vector<i32> parts(k);
        for (i32 p = 0; p < k; ++p) parts[p] = p;
        std::sort(parts.begin(), parts.end(), [&](i32 a, i32 b) { return pw[a] != pw[b] ? pw[a] < pw[b] : a < b; });
        i32 chosen = -1;
        for (i32 p : parts) {
            if (pw[p] + g.nw[n] > omega) continue;
            i64 add = 0;
            for (i64 q = g.inc_off[n]; q < g.inc_off[n] + g.inc_nin[n]; ++q) add += has[p][g.inc[q]] ? 0 : 1;
            if (D[p] + add > delta) continue;
            chosen = p;
            break;
        }
        if (chosen < 0) return "no part can take node " + std::to_string(n);
        rho[n] = chosen;
        pw[chosen] += g.nw[n];
        for (i64 q = g.inc_off[n]; q < g.inc_off[n] + g.inc_nin[n]; ++q)
            if (!has[chosen][g.inc[q]]) { has[chosen][g.inc[q]] = 1; D[chosen]++; }
    }
    return "";
}

void run_partition(Result& R, const Graph& g0, const Params& prm) {
    R.levels.push_back(g0);
    i64 W = 0;
    for (i32 n = 0; n < g0.N; ++n) {
        W += g0.nw[n];
        if (g0.nw[n] > prm.omega) { R.err = "infeasible: a node exceeds Omega"; return; }
        if (g0.inc_nin[n] > prm.delta) { R.err = "infeasible: a node exceeds Delta"; return; }
    }
    i64 target = (W + prm.omega - 1) / prm.omega;  // ceil(W / Omega) (Sec. III, Reading R12)
    const int Pi = prm.Pi;
    // Coarsening (Sec. III, Sec. V).
    for (;;) {
        const Graph& g = R.levels.back();
        LevelLog L{};
        L.N = g.N; L.E = g.E; L.P = g.P();
        if (g.N <= target) { R.log.push_back(L); break; }
        if (prm.k > 0 && g.N < 4096) { R.log.push_back(L); break; }
        double t0 = now_s();
        std::vector<i32> cand((size_t)g.N * Pi);
        std::vector<u64> score((size_t)g.N * Pi);
        ProposeScratch s;
        s.eta.assign(g.N, 0); s.inter.assign(g.N, 0); s.seen.assign(g.N, 0);
        u64 cap = noise_cap(g);
        for (i32 n = 0; n < g.N; ++n)
            propose_node(g, n, prm.omega, prm.delta, prm.seed, cap, Pi, s, &cand[(size_t)n * Pi], &score[(size_t)n * Pi]);
        std::vector<i32> match(g.N);
        std::string err = match_all(g, prm.omega, prm.delta, Pi, cand.data(), score.data(), match.data(), L.pairs,
                                    (prm.early_exit & 4) != 0);
        if (!err.empty()) { R.err = err; return; }
        i64 merges = 0;
        for (i32 n = 0; n < g.N; ++n) merges += match[n] > n ? 1 : 0;
        R.cand.push_back(std::move(cand));
        R.score.push_back(std::move(score));
        R.match.push_back(match);
        if (merges == 0) { L.t_coarsen = now_s() - t0; R.log.push_back(L); break; }
        std::vector<i32> gamma(g.N);
        Graph c = contract(g, match.data(), gamma.data());
        L.t_coarsen = now_s() - t0;
        R.log.push_back(L);
        R.gamma.push_back(std::move(gamma));
        R.levels.push_back(std::move(c));
    }
    // Initial partitioning (Sec. III): the coarsest clusters, or Reading R21.
    int l = (int)R.levels.size() - 1;
    std::vector<i32> rho;
    if (prm.k == 0) {
        rho.resize(R.levels[l].N);
        for (i32 n = 0; n < R.levels[l].N; ++n) rho[n] = n;
        R.nparts = R.levels[l].N;  // Reading R24
    } else {
        std::string err = kway_initial(R.levels[l], prm.k, prm.omega, prm.delta, rho);
        if (!err.empty()) { R.err = "infeasible: " + err; return; }
        R.nparts = prm.k;
    }
    // Uncoarsening with refinement at every level, coarsest included (Reading R26).
    R.rho.resize(l + 1);
    for (int lv = l; lv >= 0; --lv) {
        const Graph& g = R.levels[lv];
        double t0 = now_s();
        if (lv < l) {
            std::vector<i32> r2(g.N);
            for (i32 n = 0; n < g.N; ++n) r2[n] = rho[R.gamma[lv][n]];
            rho.swap(r2);
        }
        i64 applied = 0;
        for (int rep = 0; rep < prm.Theta; ++rep) {
            RepOut o = refine_rep(g, rho.data(), R.nparts, rep, prm.Theta, prm.omega, prm.delta,
                                  (prm.early_exit & 2) ? 0 : 16);
            applied += o.kstar;
            // Reading R25: a repetition that applies nothing leaves rho and the
            // sizes unchanged, so the rest of its half would repeat it exactly.
            if ((prm.early_exit & 1) && o.kstar == 0) {
                if (rep < prm.Theta / 2) rep = prm.Theta / 2 - 1;
                else break;
            }
        }
        R.log[lv].t_refine = now_s() - t0;
        R.log[lv].moves_applied = applied;
        R.log[lv].conn_after = evaluate(g, rho.data(), R.nparts, prm.omega, prm.delta).conn;
        R.rho[lv] = rho;
    }
}

Graph make_graph(i32 N, i32 E, const i64* he_off, const i32* he_nsrc, const i32* pins, const i32* hw,
                 const i32* nw) {
    Graph g;
    g.N = N;
    g.E = E;
    g.he_off.assign(he_off, he_off + E + 1);
    g.he_nsrc.assign(he_nsrc, he_nsrc + E);
    g.pins.assign(pins, pins + he_off[E]);
    g.hw.resize(E);
    g.nw.resize(N);
    for (i32 e = 0; e < E; ++e) g.hw[e] = hw ? hw[e] : 1;
    for (i32 n = 0; n < N; ++n) g.nw[n] = nw ? nw[n] : 1;
    return g;
}

void set_err(char* err, int errlen, const std::string& s) {
    if (err && errlen > 0) {
        std::snprintf(err, (size_t)errlen, "%s", s.c_str());
    }
}

}  // namespace

// ===========================================================================
// C ABI (loaded with ctypes by the tests; never by the library).
// All functions return 0 on success and a negative value on error.
// ===========================================================================
extern "C" {

int hgpo_graph_new(i32 N, i32 E, const i64* he_off, const i32* he_nsrc, const i32* pins, const i32* hw,
                   const i32* nw, void** out, char* err, int errlen) {
    if (N < 1 || E < 0 || !he_off || (E > 0 && (!he_nsrc || !pins))) {
        set_err(err, errlen, "bad arguments");
        return -1;
    }
    Graph* g = new Graph(make_graph(N, E, he_off, he_nsrc, pins, hw, nw));
    std::string e = validate_and_build(*g);
    if (!e.empty()) {
        set_err(err, errlen, e);
        delete g;
        return -1;
    }
    *out = g;
    return 0;
}

void hgpo_graph_free(void* g) { delete (Graph*)g; }

void hgpo_graph_dims(void* gp, i64* out) {
    Graph* g = (Graph*)gp;
    out[0] = g->N; out[1] = g->E; out[2] = g->P();
}

void hgpo_graph_csr(void* gp, i64* he_off, i32* he_nsrc, i32* pins, i32* hw, i32* nw) {
    Graph* g = (Graph*)gp;
    std::copy(g->he_off.begin(), g->he_off.end(), he_off);
    std::copy(g->he_nsrc.begin(), g->he_nsrc.end(), he_nsrc);
    std::copy(g->pins.begin(), g->pins.end(), pins);
    for (i32 e = 0; e < g->E; ++e) hw[e] = (i32)g->hw[e];
    for (i32 n = 0; n < g->N; ++n) nw[n] = (i32)g->nw[n];
}

void hgpo_graph_incidence(void* gp, i64* inc_off, i32* inc_nin, i32* inc) {
    Graph* g = (Graph*)gp;
    std::copy(g->inc_off.begin(), g->inc_off.end(), inc_off);
    std::copy(g->inc_nin.begin(), g->inc_nin.end(), inc_nin);
    std::copy(g->inc.begin(), g->inc.end(), inc);
}

u64 hgpo_mix64(u64 x) { return mix64(x); }
u64 hgpo_noise(u64 seed, i32 a, i32 b, u64 cap) { return noise(seed, a, b, cap); }
u64 hgpo_noise_cap(void* gp) { return noise_cap(*(Graph*)gp); }
u64 hgpo_tnorm(void* gp, i32 e) { return tnorm(*(Graph*)gp, e); }

void hgpo_pair(void* gp, i32 n, i32 m, u64* eta, i32* inter) { pair_values(*(Graph*)gp, n, m, eta, inter); }

// Candidates of the listed nodes (all nodes when nodes == NULL); cand/score
// are count x Pi, row i for nodes[i].
int hgpo_propose(void* gp, i64 omega, i64 delta, u64 seed, i32 Pi, const i32* nodes, i32 count, i32* cand,
                 u64* score) {
    Graph& g = *(Graph*)gp;
    ProposeScratch s;
    s.eta.assign(g.N, 0); s.inter.assign(g.N, 0); s.seen.assign(g.N, 0);
    u64 cap = noise_cap(g);
    i32 cnt = nodes ? count : g.N;
    for (i32 i = 0; i < cnt; ++i) {
        i32 n = nodes ? nodes[i] : i;
        if (n < 0 || n >= g.N) return -1;
        propose_node(g, n, omega, delta, seed, cap, Pi, s, cand + (size_t)i * Pi, score + (size_t)i * Pi);
    }
    return 0;
}

int hgpo_match_round(i32 N, const char* active, const i32* target, const u64* score, i32* match, char* err,
                     int errlen) {
    std::string e = match_round(N, active, target, score, match);
    if (!e.empty()) { set_err(err, errlen, e); return -1; }
    return 0;
}

int hgpo_match_round_greedy(i32 N, const char* active, const i32* target, const u64* score, i32* match, char* err,
                            int errlen) {
    std::string e = match_round_greedy(N, active, target, score, match);
    if (!e.empty()) { set_err(err, errlen, e); return -1; }
    return 0;
}

int hgpo_match(void* gp, i64 omega, i64 delta, i32 Pi, const i32* cand, const u64* score, i32* match,
               i32* round_pairs, char* err, int errlen) {
    std::string e = match_all(*(Graph*)gp, omega, delta, Pi, cand, score, match, round_pairs);
    if (!e.empty()) { set_err(err, errlen, e); return -1; }
    return 0;
}

int hgpo_contract(void* gp, const i32* match, i32* gamma, void** coarse) {
    *coarse = new Graph(contract(*(Graph*)gp, match, gamma));
    return 0;
}

// out: conn, cutnet, max_size, max_inbound, violations, nonempty
int hgpo_evaluate(void* gp, const i32* rho, i32 nparts, i64 omega, i64 delta, i64* out, i64* part_size,
                  i64* part_inbound) {
    Graph& g = *(Graph*)gp;
    for (i32 n = 0; n < g.N; ++n) if (rho[n] < 0 || rho[n] >= nparts) return -1;
    Eval r = evaluate(g, rho, nparts, omega, delta);
    out[0] = r.conn; out[1] = r.cutnet; out[2] = r.max_size; out[3] = r.max_inbound;
    out[4] = r.violations; out[5] = r.nonempty;
    if (part_size) std::copy(r.size.begin(), r.size.end(), part_size);
    if (part_inbound) std::copy(r.inbound.begin(), r.inbound.end(), part_inbound);
    return 0;
}

// Sparse rows of pins(p,e) and pins_in(p,e), ascending p; returns the number of
// entries L.  Pass part == NULL to query L only.
i64 hgpo_phi(void* gp, const i32* rho, i64* row_off, i32* part, i32* cnt, i32* cnt_in) {
    Graph& g = *(Graph*)gp;
    auto rows = phi_rows(g, rho);
    i64 L = 0;
    for (i32 e = 0; e < g.E; ++e) {
        if (row_off) row_off[e] = L;
        for (auto& t : rows[e]) {
            if (part) { part[L] = t.part; cnt[L] = t.cnt; cnt_in[L] = t.cnt_in; }
            L++;
        }
    }
    if (row_off) row_off[g.E] = L;
    return L;
}

// gain(n, p) = saving(n) - loss(n, p) exactly as Eq. refinement_move_selection.
i64 hgpo_gain(void* gp, const i32* rho, i32 n, i32 p) {
    Graph& g = *(Graph*)gp;
    i64 saving = 0, loss = 0;
    for (i64 k = g.inc_off[n]; k < g.inc_off[n + 1]; ++k) {
        i32 e = g.inc[k];
        i32 in_s = 0, in_p = 0;
        for (i64 j = g.he_off[e]; j < g.he_off[e + 1]; ++j) {
            in_s += rho[g.pins[j]] == rho[n];
            in_p += rho[g.pins[j]] == p;
        }
        if (in_s == 1) saving += g.hw[e];
        if (in_p == 0) loss += g.hw[e];
    }
    return saving - loss;
}

// Proposed move of every node: move_dst[n] (-1 = none) and its gain.
int hgpo_moves(void* gp, const i32* rho, i32 nparts, i32 rep, i32 theta, i64 omega, i32* move_dst, i64* gain) {
    Graph& g = *(Graph*)gp;
    auto rows = phi_rows(g, rho);
    std::vector<i64> psize(nparts, 0);
    for (i32 n = 0; n < g.N; ++n) psize[rho[n]] += g.nw[n];
    auto mv = propose_moves(g, rho, nparts, rep, theta, omega, rows, psize);
    for (i32 n = 0; n < g.N; ++n) { move_dst[n] = -1; gain[n] = 0; }
    for (auto& m : mv) { move_dst[m.n] = m.pd; gain[m.n] = m.gain; }
    return 0;
}

// One repetition; rho is updated in place.  Arrays sized N (seq, seq_pd, gseq)
// and N+1 (C, V).  info: M, kstar, applied_gain, links, rounds, n_chains.
int hgpo_refine_rep(void* gp, i32* rho, i32 nparts, i32 rep, i32 theta, i64 omega, i64 delta, i32* seq,
                    i32* seq_pd, i64* gseq, i64* C, i64* V, i32* chain_len, i64* info) {
    Graph& g = *(Graph*)gp;
    RepOut o = refine_rep(g, rho, nparts, rep, theta, omega, delta);
    i64 M = (i64)o.seq.size();
    if (seq) std::copy(o.seq.begin(), o.seq.end(), seq);
    if (seq_pd) std::copy(o.seq_pd.begin(), o.seq_pd.end(), seq_pd);
    if (gseq) std::copy(o.gseq.begin(), o.gseq.end(), gseq);
    if (C) std::copy(o.C.begin(), o.C.end(), C);
    if (V) std::copy(o.V.begin(), o.V.end(), V);
    if (chain_len) std::copy(o.chain_len.begin(), o.chain_len.end(), chain_len);
    info[0] = M; info[1] = o.kstar; info[2] = o.applied_gain; info[3] = o.links; info[4] = o.rounds;
    info[5] = (i64)o.chain_len.size();
    return 0;
}

// Sequence of an explicit move list (Sec. VI-C): moves (node, p_s, p_d, gain)
// are sorted (Reading R15) and chained in `rounds` chain rounds (Readings R16,
// R17).  nw / nin give every node's size and |in(n)| (N entries).  seq
// receives the M node ids in sequence order, chain_len the chain lengths
// (at most M entries); info: links, rounds run, number of chains.
int hgpo_sequence(i32 N, const i64* nw, const i32* nin, i64 M, const i32* node, const i32* ps, const i32* pd,
                  const i64* gain, i32 rounds, i32* seq, i32* chain_len, i64* info) {
    std::vector<Move> mv;
    for (i64 i = 0; i < M; ++i) {
        if (node[i] < 0 || node[i] >= N) return -1;
        mv.push_back({node[i], ps[i], pd[i], gain[i]});
    }
    sort_moves(mv);
    Sequence sq = sequence_moves(mv, nw, nin, rounds);
    for (i64 i = 0; i < M; ++i) seq[i] = mv[sq.order[i]].n;
    std::copy(sq.chain_len.begin(), sq.chain_len.end(), chain_len);
    info[0] = sq.links; info[1] = sq.rounds; info[2] = (i64)sq.chain_len.size();
    return 0;
}

int hgpo_kway_initial(void* gp, i32 k, i64 omega, i64 delta, i32* rho, char* err, int errlen) {
    std::vector<i32> r;
    std::string e = kway_initial(*(Graph*)gp, k, omega, delta, r);
    if (!e.empty()) { set_err(err, errlen, e); return -1; }
    std::copy(r.begin(), r.end(), rho);
    return 0;
}

int hgpo_partition(void* gp, i64 omega, i64 delta, i32 k, i32 Pi, i32 theta, u64 seed, i32 early_exit, void** out,
                   char* err, int errlen) {
    if (Pi < 1 || Pi > 16 || theta < 0 || omega < 1 || delta < 0) {
        set_err(err, errlen, "bad parameters");
        return -1;
    }
    Result* R = new Result();
    Params prm{omega, delta, k, Pi, theta, seed, early_exit};
    run_partition(*R, *(Graph*)gp, prm);
    if (!R->err.empty()) {
        set_err(err, errlen, R->err);
        delete R;
        return -1;
    }
    *out = R;
    return 0;
}

void hgpo_result_free(void* r) { delete (Result*)r; }
i32 hgpo_result_nlevels(void* r) { return (i32)((Result*)r)->levels.size(); }
i32 hgpo_result_nparts(void* r) { return ((Result*)r)->nparts; }
void* hgpo_result_graph(void* r, i32 lv) { return &((Result*)r)->levels[lv]; }

// out: N, E, P, t_coarsen_ns, t_refine_ns, conn_after, moves_applied, pairs[0..16]
void hgpo_result_level(void* rp, i32 lv, i64* out) {
    const LevelLog& L = ((Result*)rp)->log[lv];
    out[0] = L.N; out[1] = L.E; out[2] = L.P;
    out[3] = (i64)(L.t_coarsen * 1e9); out[4] = (i64)(L.t_refine * 1e9);
    out[5] = L.conn_after; out[6] = L.moves_applied;
    for (int i = 0; i < 17; ++i) out[7 + i] = L.pairs[i];
}

// gamma of level lv (maps level lv to lv+1); lv < nlevels-1
void hgpo_result_gamma(void* rp, i32 lv, i32* out) {
    auto& v = ((Result*)rp)->gamma[lv];
    std::copy(v.begin(), v.end(), out);
}

void hgpo_result_rho(void* rp, i32 lv, i32* out) {
    auto& v = ((Result*)rp)->rho[lv];
    std::copy(v.begin(), v.end(), out);
}

// Proposal and matching computed at level lv (levels that were coarsened).
i32 hgpo_result_ncoarsened(void* rp) { return (i32)((Result*)rp)->cand.size(); }
void hgpo_result_proposal(void* rp, i32 lv, i32* cand, u64* score, i32* match) {
    Result* R = (Result*)rp;
    std::copy(R->cand[lv].begin(), R->cand[lv].end(), cand);
    std::copy(R->score[lv].begin(), R->score[lv].end(), score);
    std::copy(R->match[lv].begin(), R->match[lv].end(), match);
}

}  // extern "C"
