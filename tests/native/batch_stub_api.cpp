// Stand-in for the partitioner's context calls, for running the batch
// scheduler (hgp_batch.cpp) on the CPU under ThreadSanitizer and
// AddressSanitizer.  Each context copies its inputs like the library does,
// spends time in proportion to the job's pins, and returns a result that is a
// fixed function of the input (rho[n] = (n * 7 + P) % 13, conn = P), so the
// driver can check every job's outputs.  A job whose delta is kOomDelta runs
// out of device memory in coarsening when another job was in progress at its
// load or is at that moment, as a deep hierarchy can beside other jobs.  Contexts share no
// state except the counters of live contexts and of jobs in progress.
#include <atomic>
#include <chrono>
#include <cstring>
#include <thread>
#include <vector>

#include "../../include/hgp.h"

std::atomic<int> g_live_contexts{0};
std::atomic<int> g_in_job{0};  // contexts between load and the end of their job
std::atomic<int> g_oom_returns{0};
constexpr int64_t kOomDelta = (1 << 20) + 1;

struct hgp_ctx {
    hgp_options opt;
    std::vector<int64_t> he_off;
    std::vector<int32_t> he_nsrc, pins, hw, nw;
    int32_t N = 0, E = 0;
    int64_t omega = 0, delta = 0;
    int32_t k = 0;
    bool loaded = false, limited = false, coarsened = false, refined = false, in_job = false;
    bool crowded = false;  // another job was in progress when this one was loaded
    std::vector<int32_t> rho;
};

extern "C" {

void hgp_default_options(hgp_options* opt) {
    std::memset(opt, 0, sizeof(*opt));
    opt->pi = 4;
    opt->theta = 16;
}

hgp_status hgp_create(hgp_ctx** out, const hgp_options* opt) {
    hgp_ctx* c = new hgp_ctx();
    c->opt = *opt;
    *out = c;
    g_live_contexts++;
    return HGP_OK;
}

void hgp_destroy(hgp_ctx* c) {
    if (!c) return;
    if (c->in_job) g_in_job--;
    g_live_contexts--;
    delete c;
}

hgp_status hgp_load_csr(hgp_ctx* c, int32_t n, int32_t e, const int64_t* he_off, const int32_t* he_nsrc,
                        const int32_t* pins, const int32_t* hedge_w, const int32_t* node_w, hgp_mem where) {
    if (!c || where != HGP_MEM_HOST || n < 1 || e < 0) return HGP_E_INVALID;
    c->N = n;
    c->E = e;
    c->he_off.assign(he_off, he_off + e + 1);
    c->he_nsrc.assign(he_nsrc, he_nsrc + e);
    c->pins.assign(pins, pins + he_off[e]);
    c->hw = hedge_w ? std::vector<int32_t>(hedge_w, hedge_w + e) : std::vector<int32_t>(e, 1);
    c->nw = node_w ? std::vector<int32_t>(node_w, node_w + n) : std::vector<int32_t>(n, 1);
    c->loaded = true;
    c->limited = c->coarsened = c->refined = false;
    if (!c->in_job) c->crowded = ++g_in_job > 1;
    c->in_job = true;
    return HGP_OK;
}

hgp_status hgp_set_limits(hgp_ctx* c, int64_t omega, int64_t delta, int32_t k) {
    if (!c->loaded) return HGP_E_STATE;
    if (omega < 1 || delta < 0 || k < 0) return HGP_E_INVALID;
    c->omega = omega;
    c->delta = delta;
    c->k = k;
    c->limited = true;
    return HGP_OK;
}

hgp_status hgp_coarsen(hgp_ctx* c, int32_t* nl) {
    if (!c->limited) return HGP_E_STATE;
    std::this_thread::sleep_for(std::chrono::microseconds(c->pins.size() / 64));
    if (c->delta == kOomDelta && (c->crowded || g_in_job.load() > 1)) {
        c->in_job = false;
        g_in_job--;
        g_oom_returns++;
        return HGP_E_NOMEM;
    }
    *nl = 3;
    c->coarsened = true;
    return HGP_OK;
}

hgp_status hgp_refine(hgp_ctx* c) {
    if (!c->coarsened) return HGP_E_STATE;
    std::this_thread::sleep_for(std::chrono::microseconds(c->pins.size() / 128));
    const int64_t P = (int64_t)c->pins.size();
    c->rho.resize(c->N);
    for (int32_t n = 0; n < c->N; ++n) c->rho[n] = (int32_t)(((int64_t)n * 7 + P) % 13);
    c->refined = true;
    return HGP_OK;
}

hgp_status hgp_get_partition(hgp_ctx* c, int32_t* rho, int64_t cap, int32_t* np) {
    if (!c->refined) return HGP_E_STATE;
    if (cap < c->N) return HGP_E_INVALID;
    std::memcpy(rho, c->rho.data(), sizeof(int32_t) * c->N);
    if (np) *np = 13;
    return HGP_OK;
}

hgp_status hgp_evaluate(hgp_ctx* c, const int32_t* rho, int32_t, hgp_eval* out) {
    if (!c->refined || rho) return HGP_E_STATE;
    std::memset(out, 0, sizeof(*out));
    out->conn = (int64_t)c->pins.size();
    out->n_parts = 13;
    if (c->in_job) g_in_job--;
    c->in_job = false;
    return HGP_OK;
}

hgp_status hgp_release(hgp_ctx* c, int32_t) {
    if (!c) return HGP_E_INVALID;
    if (c->in_job) g_in_job--;
    c->in_job = false;
    c->he_off.clear();
    c->he_nsrc.clear();
    c->pins.clear();
    c->hw.clear();
    c->nw.clear();
    c->rho.clear();
    c->loaded = c->limited = c->coarsened = c->refined = false;
    return HGP_OK;
}

}  // extern "C"
