// Batched execution of many partitioning jobs on one GPU.
//
// Small and mid-size jobs leave most of the chip idle: their levels are a few
// thousand nodes, their kernels are short, and every level has host round
// trips.  Here several worker threads each own a context with its own HIP
// stream and run whole jobs; the streams overlap on the device.  Jobs are
// admitted in arrival order, when a worker is free and their estimated device
// footprint fits the budget next to the jobs in flight.  The footprint is an
// estimate: a hierarchy's depth is known only once it is built, and a deep one
// (hundreds of levels) can outgrow it.  A job that runs out of device memory
// while other jobs are in flight is put back and run again alone, once every
// other job has finished; only a job that fails alone reports HGP_E_NOMEM.
// A worker frees its job's hierarchy as soon as the results are on the host,
// so idle workers keep only their scratch buffers.
// One worker gives the plain one-at-a-time baseline with the same code path.
// Each job's result is that of a lone run (the method is deterministic;
// contexts share nothing).
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/hgp.h"

namespace {

// Device bytes a job may hold at once: the input CSR and incidence, a
// hierarchy whose levels together hold up to about kLevelCopies times the
// input's pins (pins, incidence, pin positions and 16-bit copies, 14 B per
// pin; 72 B per node for sizes, offsets, candidates, scores, matching, cluster
// map), and the refinement and sort scratch (about 40 B per pin at the largest
// level).  Contraction shrinks pins slowly where h-edges span many clusters:
// all levels together held 5.5 times the input's pins on a convolutional
// graph, 8.5 on a netlist, 18 to 33 on uniform random and layered graphs.
constexpr int64_t kLevelCopies = 32;
int64_t footprint(const hgp_job& j) {
    const int64_t P = j.he_off ? j.he_off[j.n_hedges] : 0;
    const int64_t level = 14 * P + 72 * (int64_t)j.n_nodes + 12 * (int64_t)j.n_hedges;
    return kLevelCopies * level + 40 * P + (int64_t)(16 << 20);
}

double seconds_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

hgp_status run_one(hgp_ctx* ctx, hgp_job& j) {
    hgp_status st = hgp_load_csr(ctx, j.n_nodes, j.n_hedges, j.he_off, j.he_nsrc, j.pins, j.hedge_w, j.node_w,
                                 HGP_MEM_HOST);
    if (st != HGP_OK) return st;
    if ((st = hgp_set_limits(ctx, j.omega, j.delta, j.k)) != HGP_OK) return st;
    int32_t nl = 0;
    if ((st = hgp_coarsen(ctx, &nl)) != HGP_OK) return st;
    if ((st = hgp_refine(ctx)) != HGP_OK) return st;
    j.n_levels = nl;
    int32_t np = 0;
    if (j.rho) {
        if ((st = hgp_get_partition(ctx, j.rho, j.n_nodes, &np)) != HGP_OK) return st;
    }
    hgp_eval ev;
    if ((st = hgp_evaluate(ctx, nullptr, 0, &ev)) != HGP_OK) return st;
    j.n_parts = (int32_t)ev.n_parts;
    j.conn = ev.conn;
    j.violations = ev.violations;
    // an idle worker holds no hierarchy: a deep one can be tens of GB, which
    // the jobs still running (or a lone rerun) may need
    return hgp_release(ctx, 0);
}

}  // namespace

extern "C" hgp_status hgp_run_jobs(const hgp_options* opt, hgp_job* jobs, int64_t n_jobs, int32_t workers,
                                   int64_t hbm_budget) {
    if (n_jobs < 0 || (n_jobs > 0 && !jobs) || workers < 1 || workers > 64) return HGP_E_INVALID;
    hgp_options o;
    hgp_default_options(&o);
    if (opt) o = *opt;
    if (o.stream || o.alloc || o.free) return HGP_E_INVALID;  // every worker owns its stream and pool memory
    for (int64_t i = 0; i < n_jobs; ++i) {
        jobs[i].status = HGP_E_STATE;
        jobs[i].start_s = jobs[i].end_s = -1.0;
        jobs[i].footprint = footprint(jobs[i]);
        jobs[i].reruns = 0;
        if (i > 0 && jobs[i].arrival_s < jobs[i - 1].arrival_s) return HGP_E_INVALID;
    }
    if (hipSetDevice(o.device) != hipSuccess) return HGP_E_DEVICE;
    if (hbm_budget <= 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) return HGP_E_DEVICE;
        hbm_budget = (int64_t)(fr / 10 * 6);
    }

    std::mutex mu;
    std::condition_variable cv;
    int64_t next = 0, inflight = 0;
    int64_t admissions = 0;  // jobs started so far, lone reruns included
    int running = 0;
    bool exclusive = false;         // a job put back for lack of memory is running alone
    std::vector<int64_t> put_back;  // such jobs, waiting for the device to empty
    hgp_status setup = HGP_OK;
    const auto t0 = std::chrono::steady_clock::now();

    auto worker = [&]() {
        (void)hipSetDevice(o.device);
        hgp_ctx* ctx = nullptr;
        const hgp_status cs = hgp_create(&ctx, &o);
        if (cs != HGP_OK) {
            std::lock_guard<std::mutex> lk(mu);
            setup = cs;
            return;
        }
        for (;;) {
            int64_t i;
            int concurrent = 0;  // jobs in progress, this one included, when it started
            int64_t seen = 0;    // admissions, this one included, when it started
            bool alone = false;  // this run is a put-back job's lone rerun
            {
                std::unique_lock<std::mutex> lk(mu);
                for (;;) {
                    if (exclusive) {  // a lone rerun holds the device
                        cv.wait(lk);
                        continue;
                    }
                    if (!put_back.empty()) {
                        if (running > 0) {
                            cv.wait(lk);
                            continue;
                        }
                        alone = true;
                        break;
                    }
                    if (next >= n_jobs) break;
                    const hgp_job& j = jobs[next];
                    const auto due = t0 + std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                                              std::chrono::duration<double>(j.arrival_s));
                    if (std::chrono::steady_clock::now() < due) {
                        cv.wait_until(lk, due);
                        continue;
                    }
                    if (running > 0 && inflight + j.footprint > hbm_budget) {
                        cv.wait(lk);
                        continue;
                    }
                    break;
                }
                if (alone) {
                    i = put_back.back();
                    put_back.pop_back();
                    exclusive = true;
                } else {
                    if (next >= n_jobs) break;
                    i = next++;
                    jobs[i].start_s = seconds_since(t0);  // under the lock: starts follow admission order
                }
                ++running;
                inflight += jobs[i].footprint;
                concurrent = running;
                seen = ++admissions;
            }
            hgp_job& j = jobs[i];
            j.status = run_one(ctx, j);
            j.end_s = seconds_since(t0);
            // Out of memory beside other jobs: free what this job holds and
            // put it back for a lone rerun.  Another job overlapped this one if
            // it was in progress at this one's start or started since.
            bool again = false;
            {
                std::lock_guard<std::mutex> lk(mu);
                if (j.status == HGP_E_NOMEM && !alone && (concurrent > 1 || admissions != seen)) {
                    put_back.push_back(i);
                    j.reruns = 1;
                    again = true;
                }
                --running;
                inflight -= j.footprint;
                if (alone) exclusive = false;
            }
            if (again) {
                // a fresh context: the partial hierarchy and the workspace go
                hgp_destroy(ctx);
                ctx = nullptr;
                const hgp_status rs = hgp_create(&ctx, &o);
                if (rs != HGP_OK) {
                    std::lock_guard<std::mutex> lk(mu);
                    setup = rs;
                    cv.notify_all();
                    return;
                }
            }
            cv.notify_all();
        }
        hgp_destroy(ctx);
        cv.notify_all();
    };

    std::vector<std::thread> pool;
    pool.reserve(workers);
    for (int w = 0; w < workers; ++w) pool.emplace_back(worker);
    for (auto& t : pool) t.join();
    return setup;
}
