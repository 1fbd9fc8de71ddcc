// Host driver and C ABI of the partitioner: context and memory, loading with
// on-device validation, the multilevel loop (Sec. III), the k-way adapter
// (Sec. VII-A), result export and profiling.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <set>
#include <vector>

#include "hgp_internal.h"

namespace hgp {

void phi_export(Ctx* c, const Level& L, const i32* rho, i32 nparts, i32** part, i32** cnt, i32** cin, i32** len);

[[noreturn]] void fail(hgp_status st, const std::string& msg) { throw Error{st, msg}; }

void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) fail(HGP_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

static const char* const kKfNames[KF_COUNT] = {
    "validate", "transpose", "radix_sort", "scan", "level_stats", "propose", "match", "isolated",
    "gamma", "contract_edges", "pack", "phi", "part_stats", "gains", "moves", "chains",
    "rank", "inseq", "events", "select", "apply", "project", "eval", "misc", "propose_dense", "dense_gemm",
    "gains_gemm"};

const char* kf_name(int kf) { return (kf >= 0 && kf < KF_COUNT) ? kKfNames[kf] : "?"; }

static hipEvent_t prof_event(Ctx* c) {
    Prof& P = c->prof;
    if (P.used < P.pool.size()) return P.pool[P.used++];
    hipEvent_t e;
    HIPC(hipEventCreate(&e));
    P.pool.push_back(e);
    P.used++;
    return e;
}

static void prof_flush(Ctx* c) {
    Prof& P = c->prof;
    if (P.open.empty()) return;
    HIPC(hipStreamSynchronize(c->stream));
    if (P.lv_ns.empty()) {
        P.lv_ns.assign((size_t)kProfLevels * KF_COUNT, 0);
        P.lv_launches.assign((size_t)kProfLevels * KF_COUNT, 0);
    }
    for (auto& o : P.open) {
        float ms = 0.f;
        HIPC(hipEventElapsedTime(&ms, o.begin, o.end));
        const i64 ns = (i64)((double)ms * 1e6);
        P.ns[o.kf] += ns;
        P.launches[o.kf] += 1;
        const size_t at = (size_t)o.level * KF_COUNT + o.kf;
        P.lv_ns[at] += ns;
        P.lv_launches[at] += 1;
    }
    P.open.clear();
    P.used = 0;
}

static bool prof_on(const Ctx* c, int kf) {
    return c->opt.profile && (c->opt.profile_families == 0 || ((c->opt.profile_families >> kf) & 1u));
}

void prof_begin(Ctx* c, int kf) {
    if (!prof_on(c, kf)) return;
    if (c->prof.open.size() > 8192) prof_flush(c);
    c->prof.cur_begin = prof_event(c);
    HIPC(hipEventRecord(c->prof.cur_begin, c->stream));
}

void prof_end(Ctx* c, int kf) {
    if (!prof_on(c, kf)) return;
    hipEvent_t e = prof_event(c);
    HIPC(hipEventRecord(e, c->stream));
    c->prof.open.push_back({kf, c->prof.level, c->prof.cur_begin, e});
}

void prof_add_work(Ctx* c, int kf, i64 units) {
    if (prof_on(c, kf)) c->prof.host_work[kf] += units;
}

void prof_level(Ctx* c, int lv) { c->prof.level = std::max(0, std::min(lv, kProfLevels - 1)); }

unsigned long long* prof_bytes(Ctx* c, int kf) {
    if (!prof_on(c, kf)) return nullptr;
    Prof& P = c->prof;
    if (!P.lv_bytes) {
        const size_t sz = sizeof(unsigned long long) * (size_t)kProfLevels * KF_COUNT;
        P.b_lv_bytes = c->alloc(sz);
        P.lv_bytes = (unsigned long long*)P.b_lv_bytes.p;
        HIPC(hipMemsetAsync(P.lv_bytes, 0, sz, c->stream));
    }
    return P.lv_bytes + (size_t)P.level * KF_COUNT + kf;
}

unsigned long long* prof_work(Ctx* c, int kf) {
    if (!prof_on(c, kf)) return nullptr;
    if (!c->prof.work) {
        c->prof.b_work = c->alloc(sizeof(unsigned long long) * KF_COUNT);
        c->prof.work = (unsigned long long*)c->prof.b_work.p;
        HIPC(hipMemsetAsync(c->prof.work, 0, sizeof(unsigned long long) * KF_COUNT, c->stream));
    }
    return c->prof.work + kf;
}

Buf Ctx::alloc(size_t bytes) {
    Buf b;
    if (bytes == 0) bytes = 16;
    bytes = (bytes + 255) & ~(size_t)255;
    if (opt.alloc) {
        b.p = opt.alloc(bytes, (void*)stream, opt.alloc_user);
    } else {
        hipError_t e = hipMallocAsync(&b.p, bytes, stream);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            b.p = nullptr;
            if (e != hipErrorOutOfMemory) HIPC(hipMalloc(&b.p, bytes));
        }
    }
    if (!b.p) fail(HGP_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    b.bytes = bytes;
    return b;
}

void Ctx::release(Buf& b) {
    if (!b.p) return;
    if (opt.free) opt.free(b.p, b.bytes, (void*)stream, opt.alloc_user);
    else (void)hipFreeAsync(b.p, stream);
    b.p = nullptr;
    b.bytes = 0;
}

void Ctx::free_level(Level& L) {
    for (Buf* b : {&L.b_he_off, &L.b_he_nsrc, &L.b_pins, &L.b_nw, &L.b_inc_off, &L.b_inc_nin, &L.b_inc, &L.b_inc_pos, &L.b_pins16, &L.b_gamma,
                   &L.b_cand, &L.b_score, &L.b_match})
        release(*b);
}

void* Ctx::ws_get(int slot, size_t bytes) {
    if ((size_t)slot >= ws.size()) ws.resize(slot + 1);
    Buf& b = ws[slot];
    if (b.bytes < bytes) {
        release(b);
        b = alloc(std::max(bytes, b.bytes + b.bytes / 2));
    }
    return b.p;
}

void Ctx::sync() { HIPC(hipStreamSynchronize(stream)); }

namespace {

// Frees every level above the input hypergraph, and the partition.
void drop_hierarchy(Ctx* c) {
    for (size_t i = 1; i < c->levels.size(); ++i) c->free_level(c->levels[i]);
    if (!c->levels.empty()) {
        Level& L0 = c->levels[0];
        c->release(L0.b_gamma);
        c->release(L0.b_cand);
        c->release(L0.b_score);
        c->release(L0.b_match);
        L0.pairs = 0;
        c->levels.resize(1);
    }
    c->release(c->b_rho);
    for (auto& e : c->level_ev_coarsen) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
    for (auto& e : c->level_ev_refine) {
        if (e.first) (void)hipEventDestroy(e.first);
        if (e.second) (void)hipEventDestroy(e.second);
    }
    c->level_ev_coarsen.clear();
    c->level_ev_refine.clear();
    c->coarsened = c->refined = false;
}

std::string describe_validation(i64 bits) {
    std::string s;
    auto add = [&](i64 b, const char* m) {
        if (bits & b) s += (s.empty() ? "" : "; ") + std::string(m);
    };
    add(1, "h-edge offsets not monotone or not covering the pins");
    add(2, "empty h-edge");
    add(4, "source count outside [0, |e|]");
    add(8, "pin id outside [0, N)");
    add(16, "source or destination block not strictly ascending");
    add(32, "a pin is both source and destination of one h-edge");
    add(64, "h-edge weight < 1");
    add(128, "h-edge with more than 4096 pins");
    add(256, "node weight < 1");
    return s;
}

std::pair<hipEvent_t, hipEvent_t> new_event_pair(Ctx* c) {
    hipEvent_t a, b;
    HIPC(hipEventCreate(&a));
    HIPC(hipEventCreate(&b));
    (void)c;
    return {a, b};
}

template <typename T>
void d2h(Ctx* c, T* host, const void* dev, size_t count) {
    if (count == 0) return;
    HIPC(hipMemcpyAsync(host, dev, count * sizeof(T), hipMemcpyDeviceToHost, c->stream));
    HIPC(hipStreamSynchronize(c->stream));
}

// Initial k-way partition of the coarsest nodes: by (size desc, id asc), each
// into the part of smallest (weight, id) that keeps size <= Omega and its
// distinct inbound h-edges <= Delta.
void kway_seat(Ctx* c, const Level& L, i32 k, std::vector<i32>& rho) {
    const i32 N = L.N;
    std::vector<i32> nw(N), nin(N);
    std::vector<i64> off(N + 1);
    std::vector<i32> inc((size_t)L.P);
    d2h(c, nw.data(), L.nw(), N);
    d2h(c, nin.data(), L.inc_nin(), N);
    d2h(c, off.data(), L.inc_off(), (size_t)N + 1);
    d2h(c, inc.data(), L.inc(), (size_t)L.P);
    std::vector<i32> order(N);
    for (i32 i = 0; i < N; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](i32 a, i32 b) { return nw[a] > nw[b]; });
    const size_t words = ((size_t)L.E + 63) / 64;
    std::vector<std::vector<u64>> bits(k, std::vector<u64>(words, 0));
    std::vector<i64> pw(k, 0), D(k, 0);
    std::set<std::pair<i64, i32>> by_weight;
    for (i32 p = 0; p < k; ++p) by_weight.insert({0, p});
    rho.assign(N, -1);
    for (i32 n : order) {
        i32 chosen = -1;
        for (const auto& wp : by_weight) {
            const i32 p = wp.second;
            if (pw[p] + nw[n] > c->omega) continue;
            i64 add = 0;
            for (i64 q = off[n]; q < off[n] + nin[n]; ++q) {
                const i32 e = inc[q];
                add += (bits[p][e >> 6] >> (e & 63)) & 1 ? 0 : 1;
            }
            if (D[p] + add > c->delta) continue;
            chosen = p;
            break;
        }
        if (chosen < 0) fail(HGP_E_INFEASIBLE, "k-way seating: no part can take coarse node " + std::to_string(n));
        by_weight.erase({pw[chosen], chosen});
        pw[chosen] += nw[n];
        by_weight.insert({pw[chosen], chosen});
        for (i64 q = off[n]; q < off[n] + nin[n]; ++q) {
            const i32 e = inc[q];
            u64& w = bits[chosen][e >> 6];
            if (!((w >> (e & 63)) & 1)) {
                w |= 1ull << (e & 63);
                D[chosen]++;
            }
        }
        rho[n] = chosen;
    }
}

void require(bool ok, hgp_status st, const char* msg) {
    if (!ok) fail(st, msg);
}

}  // namespace
}  // namespace hgp

using namespace hgp;

struct hgp_ctx {
    Ctx c;
};

#define API_BEGIN(ctx)        \
    if (!(ctx)) return HGP_E_INVALID; \
    Ctx* c = &(ctx)->c;       \
    c->err.clear();           \
    try {
#define API_END                                      \
    }                                                \
    catch (const Error& e) {                         \
        c->err = e.msg;                              \
        return e.st;                                 \
    }                                                \
    catch (const std::bad_alloc&) {                  \
        c->err = "host allocation failed";           \
        return HGP_E_NOMEM;                          \
    }                                                \
    catch (...) {                                    \
        c->err = "unexpected error";                 \
        return HGP_E_DEVICE;                         \
    }                                                \
    return HGP_OK;

extern "C" {

void hgp_default_options(hgp_options* opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->device = 0;
    opt->pi = 4;
    opt->theta = 16;
    opt->seed = 0;
}

hgp_status hgp_create(hgp_ctx** out, const hgp_options* opt) {
    if (!out) return HGP_E_INVALID;
    *out = nullptr;
    hgp_ctx* h = new (std::nothrow) hgp_ctx();
    if (!h) return HGP_E_NOMEM;
    Ctx* c = &h->c;
    hgp_default_options(&c->opt);
    if (opt) c->opt = *opt;
    const int t0 = c->opt.tune[0], t1 = c->opt.tune[1];
    if (c->opt.pi < 1 || c->opt.pi > 8 || c->opt.theta < 0 || c->opt.delta_mode < 0 || c->opt.delta_mode > 2 ||
        (t0 != 0 && (t0 < 10 || t0 > 13)) || t1 < 0 || t1 > 64 || c->opt.tune[2] != 0 || c->opt.tune[3] != 0) {
        delete h;
        return HGP_E_INVALID;
    }
    try {
        HIPC(hipSetDevice(c->opt.device));
        c->device = c->opt.device;
        hipDeviceProp_t prop;
        HIPC(hipGetDeviceProperties(&prop, c->device));
        c->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
        // device address of the static workspace (hgp_evaluate_noalloc), with the device current
        c->noalloc_scratch = noalloc_scratch_init(c->device);
        if (c->opt.stream) {
            c->stream = (hipStream_t)c->opt.stream;
        } else {
            HIPC(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
            c->own_stream = true;
        }
        HIPC(hipHostMalloc((void**)&c->host_scalars, 64 * sizeof(i64), hipHostMallocDefault));
        c->ws.resize(160);
        c->force_hash_propose = (c->opt.flags & 1) != 0;
    } catch (const Error& e) {
        std::fprintf(stderr, "hgp_create: %s\n", e.msg.c_str());
        delete h;
        return e.st;
    }
    *out = h;
    return HGP_OK;
}

void hgp_destroy(hgp_ctx* h) {
    if (!h) return;
    Ctx* c = &h->c;
    try {
        (void)hipSetDevice(c->device);
        drop_hierarchy(c);
        for (auto& L : c->levels) c->free_level(L);
        c->levels.clear();
        c->release(c->b_hw);
        for (auto& b : c->ws) c->release(b);
        release_scan_state(c);
        c->release(c->prof.b_work);
        c->release(c->prof.b_lv_bytes);
        (void)hipStreamSynchronize(c->stream);
        for (auto e : c->prof.pool) (void)hipEventDestroy(e);
        if (c->host_scalars) (void)hipHostFree(c->host_scalars);
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
    } catch (...) {
    }
    delete h;
}

hgp_status hgp_release(hgp_ctx* h, int32_t workspace_too) {
    API_BEGIN(h)
    HIPC(hipSetDevice(c->device));
    drop_hierarchy(c);
    for (auto& L : c->levels) c->free_level(L);
    c->levels.clear();
    c->release(c->b_hw);
    if (workspace_too) {
        for (auto& b : c->ws) c->release(b);
        release_scan_state(c);
    }
    c->loaded = c->limits_set = c->coarsened = c->refined = false;
    c->sync();  // the frees are stream-ordered: done when this returns
    API_END
}

const char* hgp_last_error(const hgp_ctx* h) { return h ? h->c.err.c_str() : "null context"; }

hgp_status hgp_load_csr(hgp_ctx* h, int32_t n_nodes, int32_t n_hedges, const int64_t* he_off,
                        const int32_t* he_nsrc, const int32_t* pins, const int32_t* hedge_w, const int32_t* node_w,
                        hgp_mem where) {
    API_BEGIN(h)
    require(n_nodes >= 1 && n_hedges >= 0 && he_off, HGP_E_INVALID, "need N >= 1, E >= 0 and he_off");
    require(n_hedges == 0 || (he_nsrc && pins), HGP_E_INVALID, "he_nsrc and pins are required when E > 0");
    require(where == HGP_MEM_HOST || where == HGP_MEM_DEVICE, HGP_E_INVALID, "bad memory kind");
    HIPC(hipSetDevice(c->device));
    drop_hierarchy(c);
    for (auto& L : c->levels) c->free_level(L);
    c->levels.clear();
    c->release(c->b_hw);
    c->loaded = c->limits_set = false;
    prof_level(c, 0);
    const hipMemcpyKind kind = where == HGP_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    i64 P = 0;
    if (where == HGP_MEM_HOST) {
        P = he_off[n_hedges];
    } else {
        HIPC(hipMemcpyAsync(c->host_scalars, he_off + n_hedges, sizeof(i64), hipMemcpyDeviceToHost, c->stream));
        c->sync();
        P = c->host_scalars[0];
    }
    require(P >= 0 && P < ((i64)1 << 40), HGP_E_INVALID, "he_off[E] out of range");
    require(n_hedges > 0 || P == 0, HGP_E_INVALID, "he_off[0] must be 0");
    Level L;
    L.N = n_nodes;
    L.E = n_hedges;
    L.P = P;
    L.b_he_off = c->alloc(sizeof(i64) * ((size_t)n_hedges + 1));
    L.b_he_nsrc = c->alloc(sizeof(i32) * (size_t)std::max(n_hedges, 1));
    L.b_pins = c->alloc(sizeof(i32) * (size_t)std::max<i64>(P, 1));
    L.b_nw = c->alloc(sizeof(i32) * (size_t)n_nodes);
    c->b_hw = c->alloc(sizeof(i32) * (size_t)std::max(n_hedges, 1));
    c->levels.push_back(L);
    Level& L0 = c->levels[0];
    HIPC(hipMemcpyAsync(L0.he_off(), he_off, sizeof(i64) * ((size_t)n_hedges + 1), kind, c->stream));
    if (n_hedges > 0) {
        HIPC(hipMemcpyAsync(L0.he_nsrc(), he_nsrc, sizeof(i32) * (size_t)n_hedges, kind, c->stream));
        if (P > 0) HIPC(hipMemcpyAsync(L0.pins(), pins, sizeof(i32) * (size_t)P, kind, c->stream));
        if (hedge_w) HIPC(hipMemcpyAsync((void*)c->hw(), hedge_w, sizeof(i32) * (size_t)n_hedges, kind, c->stream));
        else fill_i32(c, (i32*)c->hw(), 1, n_hedges);
    }
    if (node_w) HIPC(hipMemcpyAsync(L0.nw(), node_w, sizeof(i32) * (size_t)n_nodes, kind, c->stream));
    else fill_i32(c, L0.nw(), 1, n_nodes);
    i64* dres = (i64*)c->ws_get(0 + 150, 8 * sizeof(i64));
    validate_graph(c, n_nodes, n_hedges, L0.he_off(), L0.he_nsrc(), L0.pins(), c->hw(), L0.nw(), P, dres);
    i64 r[5];
    read_back(c, dres, r, 5, 8);
    if (r[0] != 0) {
        const hgp_status st = (r[0] == 128) ? HGP_E_UNSUPPORTED : HGP_E_INVALID;
        for (auto& X : c->levels) c->free_level(X);
        c->levels.clear();
        fail(st, "invalid hypergraph: " + describe_validation(r[0]));
    }
    if (r[1] >= ((i64)1 << 31) || r[2] >= ((i64)1 << 31)) {
        for (auto& X : c->levels) c->free_level(X);
        c->levels.clear();
        fail(HGP_E_INVALID, "weight totals must stay below 2^31");
    }
    c->total_hw = r[1];
    c->total_nw = r[2];
    c->max_card = (i32)std::max<i64>(1, r[3]);
    c->max_hw = std::max<i64>(1, r[4]);
    // Constraint variants: Delta counts the h-edges whose destination pins
    // touch a part, so relabelling the roles of the validated input selects
    // what it counts (sources: swap the blocks; any pin: one merged block).
    if (c->opt.delta_mode != HGP_DELTA_INBOUND) retarget_pins(c, L0, c->opt.delta_mode);
    build_incidence(c, L0);
    check_scan_state(c);
    c->loaded = true;
    API_END
}

hgp_status hgp_set_limits(hgp_ctx* h, int64_t omega, int64_t delta, int32_t k) {
    API_BEGIN(h)
    require(c->loaded, HGP_E_STATE, "load a hypergraph first");
    require(omega >= 1 && delta >= 0 && k >= 0, HGP_E_INVALID, "need omega >= 1, delta >= 0, k >= 0");
    HIPC(hipSetDevice(c->device));
    const Level& L0 = c->levels[0];
    std::vector<i32> nw(L0.N), nin(L0.N);
    d2h(c, nw.data(), L0.nw(), L0.N);
    d2h(c, nin.data(), L0.inc_nin(), L0.N);
    const i64 mw = *std::max_element(nw.begin(), nw.end());
    const i64 mi = *std::max_element(nin.begin(), nin.end());
    if (mw > omega) fail(HGP_E_INFEASIBLE, "a node is heavier than omega");
    if (mi > delta) fail(HGP_E_INFEASIBLE, "a node has more inbound h-edges than delta");
    if (k > 0 && (i64)k * omega < c->total_nw) fail(HGP_E_INFEASIBLE, "k * omega is below the total node weight");
    drop_hierarchy(c);
    c->omega = omega;
    c->delta = delta;
    c->k = k;
    c->limits_set = true;
    API_END
}

hgp_status hgp_set_kway_limits(hgp_ctx* h, int32_t k, int32_t eps_num, int32_t eps_den, int64_t delta,
                               int64_t* omega_out) {
    if (!h) return HGP_E_INVALID;
    Ctx* c = &h->c;
    if (!c->loaded) {
        c->err = "load a hypergraph first";
        return HGP_E_STATE;
    }
    if (k < 1 || eps_num < 0 || eps_den < 1) {
        c->err = "need k >= 1, eps_num >= 0, eps_den >= 1";
        return HGP_E_INVALID;
    }
    // Omega = (1 + eps) * W / k (Sec. VII-A), with W / k rounded up and the
    // product rounded down; W is the total node weight
    const i64 per = (c->total_nw + k - 1) / k;
    const i64 omega = ((i64)eps_den + eps_num) * per / eps_den;
    const hgp_status st = hgp_set_limits(h, omega, delta, k);
    if (st == HGP_OK && omega_out) *omega_out = omega;
    return st;
}

hgp_status hgp_coarsen(hgp_ctx* h, int32_t* n_levels_out) {
    API_BEGIN(h)
    require(c->loaded && c->limits_set, HGP_E_STATE, "load a hypergraph and set limits first");
    HIPC(hipSetDevice(c->device));
    drop_hierarchy(c);
    const i64 target = (c->total_nw + c->omega - 1) / c->omega;  // ceil(W / Omega)
    for (int lv = 0;; ++lv) {
        const i32 N = c->levels[lv].N;
        if (N <= target) break;
        if (c->k > 0 && N < 4096) break;
        auto ev = new_event_pair(c);
        HIPC(hipEventRecord(ev.first, c->stream));
        prof_level(c, lv);
        coarsen_level(c, lv);
        HIPC(hipEventRecord(ev.second, c->stream));
        c->level_ev_coarsen.push_back(ev);
        if ((int)c->levels.size() == lv + 1) break;  // no merge
    }
    check_scan_state(c);
    c->coarsened = true;
    if (n_levels_out) *n_levels_out = (int32_t)c->levels.size();
    API_END
}

static void refine_all(Ctx* c) {
    const int l = (int)c->levels.size() - 1;
    const Level& Lc = c->levels[l];
    const i32 N0 = c->levels[0].N;
    c->release(c->b_rho);
    c->b_rho = c->alloc(sizeof(i32) * (size_t)N0);
    Buf other = c->alloc(sizeof(i32) * (size_t)N0);
    i32* cur = (i32*)other.p;
    i32* nxt = (i32*)c->b_rho.p;
    // Ping-pong so that level 0 ends in b_rho.
    if (l % 2 == 1) std::swap(cur, nxt);
    if (c->k == 0) {
        c->nparts = Lc.N;
        iota_i32(c, cur, Lc.N);
    } else {
        c->nparts = c->k;
        std::vector<i32> r;
        kway_seat(c, Lc, c->k, r);
        HIPC(hipMemcpyAsync(cur, r.data(), sizeof(i32) * r.size(), hipMemcpyHostToDevice, c->stream));
        c->sync();
    }
    for (auto& e : c->level_ev_refine) {
        if (e.first) (void)hipEventDestroy(e.first);
        if (e.second) (void)hipEventDestroy(e.second);
    }
    c->level_ev_refine.assign(l + 1, {nullptr, nullptr});
    const int theta = c->opt.theta;
    for (int lv = l; lv >= 0; --lv) {
        const Level& L = c->levels[lv];
        auto ev = new_event_pair(c);
        HIPC(hipEventRecord(ev.first, c->stream));
        prof_level(c, lv);
        if (lv < l) {
            project_rho(c, cur, L.gamma(), nxt, L.N);
            std::swap(cur, nxt);
        }
        bool unchanged = false;  // rho as the previous repetition found it
        i64 applied = 0;         // moves the previous repetition applied (0: rows built in full)
        for (int rep = 0; rep < theta; ++rep) {
            RepInfo ri = refine_rep(c, L, cur, c->nparts, rep, theta, nullptr, unchanged, applied);
            unchanged = ri.kstar == 0;
            applied = ri.kstar;
            // A repetition that applies nothing leaves rho and the sizes as
            // they were, so the rest of its half would repeat it exactly.
            if (ri.kstar == 0) {
                if (rep < theta / 2) rep = theta / 2 - 1;
                else break;
            }
        }
        HIPC(hipEventRecord(ev.second, c->stream));
        c->level_ev_refine[lv] = ev;
    }
    if (cur != (i32*)c->b_rho.p) {
        HIPC(hipMemcpyAsync(c->b_rho.p, cur, sizeof(i32) * (size_t)N0, hipMemcpyDeviceToDevice, c->stream));
    }
    c->release(other);
    c->sync();
}

hgp_status hgp_refine(hgp_ctx* h) {
    API_BEGIN(h)
    require(c->coarsened, HGP_E_STATE, "coarsen first");
    HIPC(hipSetDevice(c->device));
    refine_all(c);
    check_scan_state(c);
    c->refined = true;
    API_END
}

hgp_status hgp_get_levels(hgp_ctx* h, int64_t* out, int64_t cap) {
    API_BEGIN(h)
    require(c->loaded, HGP_E_STATE, "nothing loaded");
    require(out && cap >= 4 * (i64)c->levels.size(), HGP_E_INVALID, "cap too small");
    for (size_t i = 0; i < c->levels.size(); ++i) {
        out[4 * i] = c->levels[i].N;
        out[4 * i + 1] = c->levels[i].E;
        out[4 * i + 2] = c->levels[i].P;
        out[4 * i + 3] = c->levels[i].pairs;
    }
    API_END
}

hgp_status hgp_get_cluster_map(hgp_ctx* h, int32_t level, int32_t* out, int64_t cap) {
    API_BEGIN(h)
    require(c->coarsened && level >= 0 && level + 1 < (int)c->levels.size(), HGP_E_INVALID, "no such level map");
    const Level& L = c->levels[level];
    require(out && cap >= L.N, HGP_E_INVALID, "cap too small");
    d2h(c, out, L.gamma(), L.N);
    API_END
}

hgp_status hgp_get_proposal(hgp_ctx* h, int32_t level, int32_t* cand, uint64_t* score, int32_t* match,
                            int64_t cap_nodes) {
    API_BEGIN(h)
    require(c->coarsened && level >= 0 && level < (int)c->levels.size(), HGP_E_INVALID, "no such level");
    const Level& L = c->levels[level];
    require(L.b_cand.p != nullptr, HGP_E_INVALID, "this level was not coarsened");
    require(cap_nodes >= L.N, HGP_E_INVALID, "cap too small");
    const int Pi = c->opt.pi;
    if (cand) d2h(c, cand, L.b_cand.p, (size_t)L.N * Pi);
    if (score) d2h(c, (u64*)score, L.b_score.p, (size_t)L.N * Pi);
    if (match) d2h(c, match, L.b_match.p, (size_t)L.N);
    API_END
}

hgp_status hgp_get_level_graph(hgp_ctx* h, int32_t level, int64_t* he_off, int32_t* he_nsrc, int32_t* pins,
                               int32_t* node_w) {
    API_BEGIN(h)
    require(c->loaded && level >= 0 && level < (int)c->levels.size(), HGP_E_INVALID, "no such level");
    const Level& L = c->levels[level];
    if (he_off) d2h(c, he_off, L.he_off(), (size_t)L.E + 1);
    if (he_nsrc) d2h(c, he_nsrc, L.he_nsrc(), (size_t)L.E);
    if (pins) d2h(c, pins, L.pins(), (size_t)L.P);
    if (node_w) d2h(c, node_w, L.nw(), (size_t)L.N);
    API_END
}

hgp_status hgp_get_partition(hgp_ctx* h, int32_t* rho_out, int64_t cap, int32_t* n_parts_out) {
    API_BEGIN(h)
    require(c->refined, HGP_E_STATE, "refine first");
    require(rho_out && cap >= c->levels[0].N, HGP_E_INVALID, "cap too small");
    d2h(c, rho_out, c->b_rho.p, (size_t)c->levels[0].N);
    if (n_parts_out) *n_parts_out = c->nparts;
    API_END
}

hgp_status hgp_get_phi(hgp_ctx* h, int64_t* row_off, int32_t* part, int32_t* cnt, int32_t* cnt_in, int64_t cap,
                       int64_t* needed) {
    API_BEGIN(h)
    require(c->refined, HGP_E_STATE, "refine first");
    HIPC(hipSetDevice(c->device));
    const Level& L = c->levels[0];
    i32 *dp, *dc, *di, *dl;
    phi_export(c, L, (const i32*)c->b_rho.p, c->nparts, &dp, &dc, &di, &dl);
    std::vector<i32> len(L.E);
    std::vector<i64> off(L.E + 1);
    d2h(c, len.data(), dl, L.E);
    d2h(c, off.data(), L.he_off(), (size_t)L.E + 1);
    i64 total = 0;
    for (i32 e = 0; e < L.E; ++e) total += len[e];
    if (needed) *needed = total;
    if (!part || cap < total) return HGP_OK;
    std::vector<i32> hp((size_t)L.P), hc((size_t)L.P), hi((size_t)L.P);
    d2h(c, hp.data(), dp, (size_t)L.P);
    d2h(c, hc.data(), dc, (size_t)L.P);
    d2h(c, hi.data(), di, (size_t)L.P);
    i64 w = 0;
    for (i32 e = 0; e < L.E; ++e) {
        if (row_off) row_off[e] = w;
        for (i32 r = 0; r < len[e]; ++r, ++w) {
            part[w] = hp[off[e] + r];
            if (cnt) cnt[w] = hc[off[e] + r];
            if (cnt_in) cnt_in[w] = hi[off[e] + r];
        }
    }
    if (row_off) row_off[L.E] = w;
    API_END
}

hgp_status hgp_evaluate(hgp_ctx* h, const int32_t* rho, int32_t n_parts, hgp_eval* out) {
    API_BEGIN(h)
    require(c->loaded && c->limits_set && out, HGP_E_STATE, "load and set limits first");
    HIPC(hipSetDevice(c->device));
    const Level& L = c->levels[0];
    if (!rho) {
        require(c->refined, HGP_E_STATE, "no current partition");
        evaluate_dev(c, L, (const i32*)c->b_rho.p, c->nparts, out);
    } else {
        require(n_parts >= 1, HGP_E_INVALID, "n_parts >= 1");
        for (i32 n = 0; n < L.N; ++n)
            if (rho[n] < 0 || rho[n] >= n_parts) fail(HGP_E_INVALID, "rho out of range");
        i32* d = (i32*)c->ws_get(151, sizeof(i32) * (size_t)L.N);
        HIPC(hipMemcpyAsync(d, rho, sizeof(i32) * (size_t)L.N, hipMemcpyHostToDevice, c->stream));
        evaluate_dev(c, L, d, n_parts, out);
    }
    API_END
}

hgp_status hgp_evaluate_noalloc(hgp_ctx* h, const int32_t* rho, int32_t n_parts, hgp_eval* out) {
    API_BEGIN(h)
    require(c->loaded && c->limits_set, HGP_E_STATE, "load and set limits first");
    require(rho != nullptr && out != nullptr && n_parts >= 1, HGP_E_INVALID, "rho, out and n_parts >= 1 required");
    HIPC(hipSetDevice(c->device));
    evaluate_noalloc(c, c->levels[0], (const i32*)rho, n_parts, out);
    API_END
}

hgp_status hgp_refine_rep(hgp_ctx* h, int32_t* rho, int32_t n_parts, int32_t rep, int64_t* info,
                          int32_t* move_dst, int64_t* move_gain, int32_t* seq, int32_t* seq_dst, int64_t* gseq,
                          int64_t* prefix_gain, int64_t* prefix_viol) {
    API_BEGIN(h)
    require(c->loaded && c->limits_set, HGP_E_STATE, "load and set limits first");
    require(rho && n_parts >= 1 && rep >= 0, HGP_E_INVALID, "bad arguments");
    HIPC(hipSetDevice(c->device));
    const Level& L = c->levels[0];
    for (i32 n = 0; n < L.N; ++n)
        if (rho[n] < 0 || rho[n] >= n_parts) fail(HGP_E_INVALID, "rho out of range");
    i32* d = (i32*)c->ws_get(152, sizeof(i32) * (size_t)L.N);
    HIPC(hipMemcpyAsync(d, rho, sizeof(i32) * (size_t)L.N, hipMemcpyHostToDevice, c->stream));
    RepTrace tr;
    tr.move_dst = move_dst;
    tr.move_gain = move_gain;
    tr.seq = seq;
    tr.seq_dst = seq_dst;
    tr.gseq = gseq;
    tr.prefix_gain = prefix_gain;
    tr.prefix_viol = prefix_viol;
    RepInfo ri = refine_rep(c, L, d, n_parts, rep, c->opt.theta, &tr);
    check_scan_state(c);
    d2h(c, rho, d, (size_t)L.N);
    if (info) {
        info[0] = ri.moves;
        info[1] = ri.kstar;
        info[2] = ri.gain;
        info[3] = ri.links;
    }
    API_END
}

hgp_status hgp_kernel_stats(hgp_ctx* h, const char** names, int64_t* launches, int64_t* total_ns, int32_t* count) {
    API_BEGIN(h)
    prof_flush(c);
    if (count) *count = KF_COUNT;
    for (int i = 0; i < KF_COUNT; ++i) {
        if (names) names[i] = kf_name(i);
        if (launches) launches[i] = c->prof.launches[i];
        if (total_ns) total_ns[i] = c->prof.ns[i];
    }
    API_END
}

hgp_status hgp_reset_kernel_stats(hgp_ctx* h) {
    API_BEGIN(h)
    prof_flush(c);
    for (int i = 0; i < KF_COUNT; ++i) c->prof.launches[i] = c->prof.ns[i] = c->prof.host_work[i] = 0;
    if (c->prof.work) HIPC(hipMemsetAsync(c->prof.work, 0, sizeof(unsigned long long) * KF_COUNT, c->stream));
    std::fill(c->prof.lv_ns.begin(), c->prof.lv_ns.end(), 0);
    std::fill(c->prof.lv_launches.begin(), c->prof.lv_launches.end(), 0);
    if (c->prof.lv_bytes)
        HIPC(hipMemsetAsync(c->prof.lv_bytes, 0, sizeof(unsigned long long) * (size_t)kProfLevels * KF_COUNT,
                            c->stream));
    API_END
}

hgp_status hgp_kernel_work(hgp_ctx* h, int64_t* work, int32_t* count) {
    API_BEGIN(h)
    if (count) *count = KF_COUNT;
    if (work) {
        unsigned long long w[KF_COUNT] = {0};
        if (c->prof.work) {
            HIPC(hipMemcpyAsync(w, c->prof.work, sizeof(w), hipMemcpyDeviceToHost, c->stream));
            HIPC(hipStreamSynchronize(c->stream));
        }
        for (int i = 0; i < KF_COUNT; ++i) work[i] = (int64_t)w[i] + c->prof.host_work[i];
    }
    API_END
}

hgp_status hgp_kernel_level_stats(hgp_ctx* h, int64_t* out, int64_t cap, int32_t* n_levels_out) {
    API_BEGIN(h)
    const i64 L = std::min<i64>((i64)c->levels.size(), kProfLevels);
    if (n_levels_out) *n_levels_out = (int32_t)L;
    if (out) {
        require(cap >= L * KF_COUNT * 3, HGP_E_INVALID, "cap too small");
        prof_flush(c);
        std::vector<unsigned long long> b((size_t)L * KF_COUNT, 0);
        if (c->prof.lv_bytes && L > 0) {
            HIPC(hipMemcpyAsync(b.data(), c->prof.lv_bytes, sizeof(unsigned long long) * b.size(),
                                hipMemcpyDeviceToHost, c->stream));
            HIPC(hipStreamSynchronize(c->stream));
        }
        for (i64 i = 0; i < L * KF_COUNT; ++i) {
            const bool any = !c->prof.lv_ns.empty();
            out[3 * i] = any ? c->prof.lv_launches[i] : 0;
            out[3 * i + 1] = any ? c->prof.lv_ns[i] : 0;
            out[3 * i + 2] = (int64_t)b[i];
        }
    }
    API_END
}

hgp_status hgp_level_times(hgp_ctx* h, int64_t* out, int64_t cap) {
    API_BEGIN(h)
    const size_t L = c->levels.size();
    require(out && cap >= 2 * (i64)L, HGP_E_INVALID, "cap too small");
    c->sync();
    for (size_t i = 0; i < L; ++i) {
        out[2 * i] = out[2 * i + 1] = 0;
        float ms = 0.f;
        if (i < c->level_ev_coarsen.size() &&
            hipEventElapsedTime(&ms, c->level_ev_coarsen[i].first, c->level_ev_coarsen[i].second) == hipSuccess)
            out[2 * i] = (i64)((double)ms * 1e6);
        if (i < c->level_ev_refine.size() && c->level_ev_refine[i].first &&
            hipEventElapsedTime(&ms, c->level_ev_refine[i].first, c->level_ev_refine[i].second) == hipSuccess)
            out[2 * i + 1] = (i64)((double)ms * 1e6);
    }
    API_END
}

}  // extern "C"
