// Runs the batch scheduler (hgp_run_jobs) on the CPU against the stand-in
// context calls with many workers and jobs, arrivals spread over time, and a
// tight memory budget, then checks every job: status, outputs, admission
// after arrival, and that jobs running at once never exceeded the budget
// unless one ran alone.  Every 17th job runs out of device memory whenever
// another job is in progress (the stand-in's kOomDelta): it must be put back,
// rerun alone and end with status OK.  Built and run under the sanitizers by
// tests/test_native_sanitizers.py.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../include/hgp.h"

#include <atomic>
extern std::atomic<int> g_oom_returns;  // the stand-in's out-of-memory returns

int main(int argc, char** argv) {
    const int n_jobs = argc > 1 ? std::atoi(argv[1]) : 200;
    const int workers = argc > 2 ? std::atoi(argv[2]) : 8;
    uint64_t s = 12345;
    auto rnd = [&]() {
        s = s * 6364136223846793005ull + 1442695040888963407ull;
        return (uint32_t)(s >> 33);
    };
    struct Input {
        std::vector<int64_t> he_off;
        std::vector<int32_t> nsrc, pins, hw, nw, rho;
    };
    std::vector<Input> in(n_jobs);
    std::vector<hgp_job> jobs(n_jobs);
    double t = 0;
    for (int i = 0; i < n_jobs; ++i) {
        const int N = 64 + (int)(rnd() % 4000), E = N, card = 2 + (int)(rnd() % 30);
        Input& x = in[i];
        x.he_off.push_back(0);
        for (int e = 0; e < E; ++e) {
            x.nsrc.push_back(1);
            for (int q = 0; q < card; ++q) x.pins.push_back((e + q) % N);
            x.he_off.push_back((int64_t)x.pins.size());
        }
        x.hw.assign(E, 1);
        x.nw.assign(N, 1);
        x.rho.assign(N, -1);
        hgp_job& j = jobs[i];
        j = hgp_job{};
        j.n_nodes = N;
        j.n_hedges = E;
        j.he_off = x.he_off.data();
        j.he_nsrc = x.nsrc.data();
        j.pins = x.pins.data();
        j.hedge_w = (i % 3) ? x.hw.data() : nullptr;
        j.node_w = (i % 5) ? x.nw.data() : nullptr;
        j.omega = 64;
        j.delta = (i % 17 == 5) ? (1 << 20) + 1 : 1 << 20;  // (1 << 20) + 1: out of memory beside others
        if (i % 17 == 5 && i > 0) j.arrival_s = jobs[i - 1].arrival_s;
        j.k = 0;
        t += (rnd() % 4 == 0) ? 0.0 : 0.0005 * (rnd() % 4);
        j.arrival_s = t;  // (a job that runs out of memory beside others arrives with its predecessor)
        j.rho = x.rho.data();
    }
    // budget: room for about three average jobs at once, by the scheduler's
    // footprint estimate (32 level copies of 14 B per pin, 72 B per node and
    // 12 B per h-edge, 40 B per pin of scratch, 16 MiB)
    hgp_options opt;
    hgp_default_options(&opt);
    int64_t budget = 0;
    {
        int64_t tot = 0;
        for (auto& j : jobs) {
            const int64_t P = j.he_off[j.n_hedges];
            tot += 32 * (14 * P + 72 * (int64_t)j.n_nodes + 12 * (int64_t)j.n_hedges) + 40 * P + (16 << 20);
        }
        budget = 3 * tot / n_jobs;
    }
    hgp_status st = hgp_run_jobs(&opt, jobs.data(), n_jobs, workers, budget);
    if (st != HGP_OK) {
        std::printf("hgp_run_jobs returned %d\n", (int)st);
        return 1;
    }
    int bad = 0;
    for (int i = 0; i < n_jobs; ++i) {
        const hgp_job& j = jobs[i];
        const int64_t P = j.he_off[j.n_hedges];
        if (j.status != HGP_OK) { std::printf("job %d status %d\n", i, (int)j.status); bad++; continue; }
        if (j.conn != P || j.n_parts != 13 || j.n_levels != 3) { std::printf("job %d outputs\n", i); bad++; }
        for (int n = 0; n < j.n_nodes; ++n)
            if (in[i].rho[n] != (int32_t)(((int64_t)n * 7 + P) % 13)) { std::printf("job %d rho\n", i); bad++; break; }
        if (j.start_s + 1e-9 < j.arrival_s || j.end_s < j.start_s) { std::printf("job %d times\n", i); bad++; }
        if (i > 0 && j.start_s + 1e-9 < jobs[i - 1].start_s) { std::printf("job %d admitted out of order\n", i); bad++; }
    }
    // at each admission no more jobs are in flight than workers (a put-back
    // job's span covers its first attempt and its lone rerun, so those spans
    // are left out)
    auto put_back = [&](int q) { return jobs[q].delta == (1 << 20) + 1; };
    for (int i = 0; i < n_jobs; ++i) {
        if (put_back(i)) continue;
        int cnt = 0;
        for (int q = 0; q < n_jobs; ++q)
            if (!put_back(q) && jobs[q].start_s <= jobs[i].start_s && jobs[q].end_s > jobs[i].start_s) cnt++;
        if (cnt > workers) { std::printf("more jobs in flight than workers at job %d\n", i); bad++; }
    }
    // every out-of-memory return beside other jobs is one recorded rerun
    int reruns = 0;
    for (int i = 0; i < n_jobs; ++i) {
        reruns += jobs[i].reruns;
        if (jobs[i].reruns && !put_back(i)) { std::printf("job %d rerun without running out of memory\n", i); bad++; }
    }
    if (reruns != g_oom_returns.load()) { std::printf("reruns %d, out-of-memory returns %d\n", reruns, g_oom_returns.load()); bad++; }
    std::printf("jobs %d workers %d budget %lld put back %d bad %d\n", n_jobs, workers, (long long)budget,
                g_oom_returns.load(), bad);
    return bad ? 1 : 0;
}
