// Internal declarations shared by the library's translation units.
// Device helpers, the context layout and the kernel launchers.
#pragma once

#include <initializer_list>

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hgp.h"

typedef int32_t i32;
typedef int64_t i64;
typedef uint32_t u32;
typedef uint64_t u64;

namespace hgp {

// ---------------------------------------------------------------------------
// Errors: thrown inside the library, turned into hgp_status at the ABI.
// ---------------------------------------------------------------------------
struct Error {
    hgp_status st;
    std::string msg;
};

[[noreturn]] void fail(hgp_status st, const std::string& msg);
void hip_check(hipError_t e, const char* what);
#define HIPC(x) ::hgp::hip_check((x), #x)

// ---------------------------------------------------------------------------
// Kernel families timed when profiling is on.
// ---------------------------------------------------------------------------
enum Kf {
    KF_VALIDATE, KF_TRANSPOSE, KF_SORT, KF_SCAN, KF_LEVEL_STATS, KF_PROPOSE, KF_MATCH, KF_ISOLATED,
    KF_GAMMA, KF_CONTRACT_EDGES, KF_PACK, KF_PHI, KF_PART_STATS, KF_GAINS, KF_MOVES, KF_CHAINS,
    KF_RANK, KF_INSEQ, KF_EVENTS, KF_SELECT, KF_APPLY, KF_PROJECT, KF_EVAL, KF_MISC, KF_PROPOSE_DENSE, KF_DENSE_GEMM,
    KF_GAINS_GEMM, KF_COUNT
};
const char* kf_name(int kf);

struct Ctx;
void prof_begin(Ctx* c, int kf);
void prof_end(Ctx* c, int kf);
// Device counter of family kf's work units (e.g. row entries visited), or
// null when the family is not profiled; kernels add to it only when non-null.
unsigned long long* prof_work(Ctx* c, int kf);
// Adds work units known on the host (e.g. the MACs of a dense product) to
// family kf's counter when the family is profiled.
void prof_add_work(Ctx* c, int kf, i64 units);
// Device counter of the algorithmic bytes (compulsory reads and writes) of
// family kf's launches at the current level, or null when kf is not profiled;
// streaming kernels add to it once per wave when non-null.
unsigned long long* prof_bytes(Ctx* c, int kf);
// Attributes the following launches to level `lv`.
void prof_level(Ctx* c, int lv);

#define LAUNCH(ctx, kf, kern, grid, block, shmem, ...)                                  \
    do {                                                                                \
        ::hgp::prof_begin((ctx), (kf));                                                 \
        hipLaunchKernelGGL(kern, dim3(grid), dim3(block), (shmem), (ctx)->stream, __VA_ARGS__); \
        HIPC(hipGetLastError());                                                        \
        ::hgp::prof_end((ctx), (kf));                                                   \
    } while (0)

// ---------------------------------------------------------------------------
// Device memory.
// ---------------------------------------------------------------------------
struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
};

// One hypergraph of the hierarchy, device resident.
struct Level {
    i32 N = 0, E = 0;
    i64 P = 0;
    i64 pairs = 0;
    Buf b_he_off, b_he_nsrc, b_pins, b_nw, b_inc_off, b_inc_nin, b_inc, b_inc_pos, b_gamma, b_cand, b_score, b_match;
    Buf b_pins16;  // 16-bit copy of pins when N <= 65,536 (read by the proposal), else empty
    i64* he_off() const { return (i64*)b_he_off.p; }
    i32* he_nsrc() const { return (i32*)b_he_nsrc.p; }
    i32* pins() const { return (i32*)b_pins.p; }
    i32* nw() const { return (i32*)b_nw.p; }
    i64* inc_off() const { return (i64*)b_inc_off.p; }
    i32* inc_nin() const { return (i32*)b_inc_nin.p; }
    i32* inc() const { return (i32*)b_inc.p; }
    i32* inc_pos() const { return (i32*)b_inc_pos.p; }  // pin position of each incidence entry
    i32* gamma() const { return (i32*)b_gamma.p; }
};

// Launches are attributed to a level: coarsening level l (building G_(l+1)
// from G_l, the load counting as level 0) or the refinement of level l.
constexpr int kProfLevels = 1024;

struct ProfOpen {
    int kf, level;
    hipEvent_t begin, end;
};

struct Prof {
    std::vector<hipEvent_t> pool;
    std::vector<ProfOpen> open;
    i64 launches[KF_COUNT] = {0};
    i64 ns[KF_COUNT] = {0};
    size_t used = 0;
    hipEvent_t cur_begin = nullptr;
    unsigned long long* work = nullptr;  // device, KF_COUNT counters; allocated when first asked for
    Buf b_work;
    i64 host_work[KF_COUNT] = {0};
    int level = 0;                        // level the next launches belong to
    std::vector<i64> lv_launches, lv_ns;  // [level * KF_COUNT + kf]
    // device [kProfLevels * KF_COUNT]: algorithmic bytes counted by the kernels
    unsigned long long* lv_bytes = nullptr;
    Buf b_lv_bytes;
};

struct Ctx {
    i64 max_nbound = 0;  // largest neighbour bound of the level being coarsened
    u64 sum_card_sq = 0;  // sum of |e|^2 over the h-edges of that level
    hgp_options opt{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;
    int num_cu = 256;
    std::string err;

    bool loaded = false, limits_set = false, coarsened = false, refined = false;
    i64 omega = 0, delta = 0;
    i32 k = 0;
    i64 total_nw = 0, total_hw = 0;
    i32 max_card = 1;  // largest input h-edge; bounds every level
    i64 max_hw = 1;    // largest h-edge weight
    bool force_hash_propose = false;  // testing: use the sparse proposal at every level

    Buf b_hw;  // h-edge weights, shared by every level (h-edges keep their id)
    std::vector<Level> levels;
    Buf b_rho;  // partition of level 0 after refinement
    i32 nparts = 0;

    // Growable scratch, reused across levels and repetitions.
    std::vector<Buf> ws;
    void* ws_get(int slot, size_t bytes);

    // State of the single-pass scan (k_prim.hip): a tile ticket counter, an
    // error word, and per tile a status word and two values.  Zeroed when
    // allocated; every scan after that takes a fresh tag and a fresh run of
    // tickets, so no clearing is needed between scans.
    Buf b_scan;
    i64 scan_tiles = 0;   // tiles the state has room for
    u64 scan_tag = 0;     // tag of the last scan
    u64 scan_ticket = 0;  // tickets handed out so far

    // Pinned host staging for scalars read back by the driver.
    i64* host_scalars = nullptr;
    // Device address of the library's static workspace on this context's
    // device (hgp_evaluate_noalloc), looked up once per device at creation.
    void* noalloc_scratch = nullptr;

    // Profiling.
    Prof prof;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> level_ev_coarsen, level_ev_refine;

    Buf alloc(size_t bytes);
    void release(Buf& b);
    void free_level(Level& L);
    void sync();
    const i32* hw() const { return (const i32*)b_hw.p; }
};

template <typename T>
inline T* wsp(Ctx* c, int slot, size_t count) {
    return (T*)c->ws_get(slot, count * sizeof(T) + 16);
}

inline i64 ceil_div(i64 a, i64 b) { return (a + b - 1) / b; }
inline int grid_for(i64 n, int block, int cap = 1 << 20) {
    i64 g = ceil_div(n, block);
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

// ---------------------------------------------------------------------------
// Primitive launchers (k_prim.hip).
// ---------------------------------------------------------------------------
// out[i] = sum_{j<i} in[j] for i in [0, n]; out has n+1 slots (out[n] = total).
void scan_excl_i64(Ctx* c, const i64* in, i64* out, i64 n);
void scan_excl_i32_to_i64(Ctx* c, const i32* in, i64* out, i64 n);
void scan_excl_i32(Ctx* c, const i32* in, i32* out, i64 n);  // caller guarantees the total fits i32
// Stable LSD radix sorts on the low `bits` bits of the key.
void sort_pairs_u32(Ctx* c, const u32* kin, u32* kout, const i32* vin, i32* vout, i64 n, int bits);
void sort_pairs_u64(Ctx* c, const u64* kin, u64* kout, const i32* vin, i32* vout, i64 n, int bits);
void sort_pairs_u32_u64(Ctx* c, const u32* kin, u32* kout, const u64* vin, u64* vout, i64 n, int bits);
void fill_i32(Ctx* c, i32* p, i32 v, i64 n);
// Sets up to kFillMax buffers to a 32-bit pattern in one launch (n in 32-bit
// words; entries with n <= 0 are skipped).
struct FillItem {
    void* p;
    i64 n;
    u32 v;
};
constexpr int kFillMax = 8;
struct FillList {
    FillItem it[kFillMax];
};
void fill_many(Ctx* c, std::initializer_list<FillItem> items);
void fill_i64(Ctx* c, i64* p, i64 v, i64 n);
void iota_i32(Ctx* c, i32* p, i64 n);
void gather_i32(Ctx* c, const i32* src, const i32* idx, i32* dst, i64 n);  // dst[i] = src[idx[i]]
// Reads `count` device i64 values into host memory (synchronises the stream).
void read_back(Ctx* c, const void* dev, i64* host, int count, int elem_bytes);
// Fails with HGP_E_DEVICE if a scan's look-back wait ran out since the state
// was allocated (synchronises the stream).
void check_scan_state(Ctx* c);
void release_scan_state(Ctx* c);

// ---------------------------------------------------------------------------
// Hypergraph launchers (k_graph.hip).
// ---------------------------------------------------------------------------
// Validates the input hypergraph; *errcode receives a bit mask (0 = valid) and
// sums[0..1] the weight totals.
void validate_graph(Ctx* c, i32 N, i32 E, const i64* he_off, const i32* he_nsrc, const i32* pins, const i32* hw,
                    const i32* nw, i64 P, i64* d_err_and_sums);
// Builds the incidence (node -> h-edges, inbound first, ascending ids) of L.
void build_incidence(Ctx* c, Level& L);
// Coarse pins of every h-edge through gamma, deduplicated, src' = gamma(src) \ dst'.
void contract_edges(Ctx* c, const Level& L, const i32* gamma, Level& out);
// Phi rows at the h-edge offsets: part / cnt / cnt_in, row length in len[E].
// Relabels pin roles in place for a constraint variant (delta_mode 1: each
// h-edge's sources and destinations swap blocks; 2: one sorted block of
// destinations, no sources).
void retarget_pins(Ctx* c, Level& L, int mode);
// Phi rows of every h-edge at its pin offset; with `single`, one byte per pin
// slot that is 1 when pins(rho(m), e) = 1 for the slot's pin m; with `part16`,
// a 16-bit copy of each row's partition id whose top bit marks pins(p,e) = 1
// (partition ids below 2^15).  With `elist`, only the *ecount h-edges it lists
// (a device count) are rebuilt; the other rows are left as they are.
void build_phi(Ctx* c, const Level& L, const i32* rho, i32* part, i32* cnt, i32* cnt_in, i32* len,
               unsigned char* single = nullptr, unsigned short* part16 = nullptr, const i32* elist = nullptr,
               const u32* ecount = nullptr);

// ---------------------------------------------------------------------------
// Coarsening launchers (k_coarsen.hip).
// ---------------------------------------------------------------------------
void coarsen_level(Ctx* c, int lv);
// Dense (MFMA) candidate proposal for small levels; see k_dense.hip.
bool dense_proposal_fits(i32 N, i32 E, u64 max_t);
bool prefer_dense_proposal(const Ctx* c, i32 N, i32 E, u64 max_t, u64 sum_card_sq);
void propose_dense(Ctx* c, const Level& L, int Pi, const unsigned long long* stats, int ib, u64 max_t, i32* cand,
                   u64* score);  // builds levels[lv+1] or leaves levels unchanged if no merge
// Dense (MFMA) in-isolation moves for small levels; see k_dense.hip.  `single`
// holds one byte per pin slot (pins(rho(m), e) = 1), `part` / `len` the Phi rows.
bool use_dense_gains(const Ctx* c, const Level& L, i32 nparts);
void gains_dense(Ctx* c, const Level& L, const i32* rho, i32 nparts, const i32* part, const i32* len,
                 const unsigned char* single, const i64* psize, i32* mdst_any, i64* mgain_any, i32* mdst_sa,
                 i64* mgain_sa);

// ---------------------------------------------------------------------------
// Refinement launchers (k_refine.hip).
// ---------------------------------------------------------------------------
struct RepInfo {
    i64 moves = 0, kstar = 0, gain = 0, links = 0;
};
// Host copies of one repetition's intermediate arrays (any pointer may be NULL).
struct RepTrace {
    i32* move_dst = nullptr;
    i64* move_gain = nullptr;
    i32* seq = nullptr;
    i32* seq_dst = nullptr;
    i64* gseq = nullptr;
    i64* prefix_gain = nullptr;
    i64* prefix_viol = nullptr;
};
// reuse = rho is unchanged since the previous call on this level (it applied
// no move), so its pins rows, sizes and moves are taken as they are.
// incr_k > 0 = the previous call on this level applied the first incr_k moves
// of its sequence: only the pins rows of their h-edges are rebuilt.
RepInfo refine_rep(Ctx* c, const Level& L, i32* rho, i32 nparts, int rep, int theta, RepTrace* trace = nullptr,
                   bool reuse = false, i64 incr_k = 0);
void project_rho(Ctx* c, const i32* rho_coarse, const i32* gamma, i32* rho_fine, i32 N);
void evaluate_dev(Ctx* c, const Level& L, const i32* rho, i32 nparts, hgp_eval* out);

// Static device workspace of the evaluation that allocates nothing: Phi rows,
// partition sizes and D(p), the range check of rho and the results.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
// Device address of that workspace on the current device; the symbol lookup
// runs once per device (later calls return the kept address).
void* noalloc_scratch_init(int device);
// Bytes of that workspace an evaluation of L with nparts partitions needs.
size_t noalloc_eval_bytes(const Level& L, i32 nparts);
// hgp_evaluate on a device-resident rho, with every buffer in the static
// workspace: no allocation, two host synchronisations (range check, results).
void evaluate_noalloc(Ctx* c, const Level& L, const i32* rho, i32 nparts, hgp_eval* out);

}  // namespace hgp
