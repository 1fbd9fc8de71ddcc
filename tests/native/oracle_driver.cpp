// Exercises the serial oracle through its C entry points on many small
// random hypergraphs (partitioning in both modes, single repetitions, explicit
// move sequences, evaluation, Phi rows, k-way seating), for the
// AddressSanitizer / UndefinedBehaviorSanitizer build made by
// tests/test_native_sanitizers.py.  Checks a few invariants on the way.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../oracle/hgp_oracle.cpp"

int main() {
    uint64_t s = 99;
    auto rnd = [&](uint32_t m) {
        s = s * 6364136223846793005ull + 1442695040888963407ull;
        return (int32_t)((s >> 33) % m);
    };
    int bad = 0;
    for (int it = 0; it < 60; ++it) {
        const int N = 8 + rnd(120), E = 4 + rnd(140), maxc = 2 + rnd(12);
        std::vector<int64_t> off(1, 0);
        std::vector<int32_t> nsrc, pins, hw, nw(N);
        std::vector<char> used(N);
        for (int e = 0; e < E; ++e) {
            const int c = 1 + rnd(std::min(maxc, N));
            std::vector<int32_t> mem;
            while ((int)mem.size() < c) {
                int32_t m = rnd(N);
                if (!used[m]) { used[m] = 1; mem.push_back(m); }
            }
            for (int32_t m : mem) used[m] = 0;
            const int ns = rnd(std::min(3, c) + 1);
            std::sort(mem.begin(), mem.begin() + ns);
            std::sort(mem.begin() + ns, mem.end());
            nsrc.push_back(ns);
            pins.insert(pins.end(), mem.begin(), mem.end());
            off.push_back((int64_t)pins.size());
            hw.push_back(1 + rnd(3));
        }
        for (int n = 0; n < N; ++n) nw[n] = 1 + rnd(3);
        void* g = nullptr;
        char err[256];
        if (hgpo_graph_new(N, E, off.data(), nsrc.data(), pins.data(), hw.data(), nw.data(), &g, err, 256) != 0) {
            std::printf("graph_new: %s\n", err);
            return 1;
        }
        const int64_t omega = 3 + rnd(20), delta = 2 + rnd(40);
        for (int k : {0, 2 + rnd(6)}) {
            void* r = nullptr;
            const int64_t om = k ? 1 << 20 : omega;
            if (hgpo_partition(g, om, delta + (k ? 1000 : 0), k, 1 + rnd(6), rnd(5), (uint64_t)it, it & 1, &r, err,
                               256) == 0) {
                std::vector<int32_t> rho(N);
                hgpo_result_rho(r, 0, rho.data());
                int64_t ev[6];
                const int32_t P = hgpo_result_nparts(r);
                if (hgpo_evaluate(g, rho.data(), P, om, delta + (k ? 1000 : 0), ev, nullptr, nullptr) != 0) bad++;
                hgpo_result_free(r);
            }
        }
        const int32_t P = 2 + rnd(9);
        std::vector<int32_t> rho(N), seq(N), spd(N), cl(N), dst(N);
        std::vector<int64_t> gseq(N), C(N + 1), V(N + 1), gain(N), info(6);
        for (int n = 0; n < N; ++n) rho[n] = rnd(P);
        hgpo_moves(g, rho.data(), P, rnd(16), 16, omega, dst.data(), gain.data());
        hgpo_refine_rep(g, rho.data(), P, rnd(16), 16, 1 << 20, 1 << 20, seq.data(), spd.data(), gseq.data(),
                        C.data(), V.data(), cl.data(), info.data());
        std::vector<int64_t> roff(E + 1);
        const int64_t L = hgpo_phi(g, rho.data(), nullptr, nullptr, nullptr, nullptr);
        std::vector<int32_t> part(L + 1), cnt(L + 1), cin(L + 1);
        hgpo_phi(g, rho.data(), roff.data(), part.data(), cnt.data(), cin.data());
        std::vector<int64_t> nw64(nw.begin(), nw.end());
        std::vector<int32_t> nin(N, 0), mn, mps, mpd;
        std::vector<int64_t> mg;
        for (int n = 0; n < N; ++n)
            if (dst[n] >= 0) { mn.push_back(n); mps.push_back(rho[n]); mpd.push_back(dst[n]); mg.push_back(gain[n]); }
        int64_t sinfo[3];
        std::vector<int32_t> sq(mn.size() + 1), scl(mn.size() + 1);
        if (hgpo_sequence(N, nw64.data(), nin.data(), (int64_t)mn.size(), mn.data(), mps.data(), mpd.data(),
                          mg.data(), 16, sq.data(), scl.data(), sinfo) != 0)
            bad++;
        std::vector<int32_t> kr(N);
        hgpo_kway_initial(g, 3, 1 << 20, 1 << 20, kr.data(), err, 256);
        hgpo_graph_free(g);
    }
    std::printf("oracle driver: bad %d\n", bad);
    return bad ? 1 : 0;
}
