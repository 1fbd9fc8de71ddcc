"""Parity of the HIP path with the oracle, element by element, on seeded
inputs: every level's proposal (candidates, scores, matching), cluster map
and coarse hypergraph, the final partition, connectivity and the pins(p,e)
rows.  Everything is integer, so the bar is bit-exact equality."""
import numpy as np
import pytest

import oracle
from paper_2605_20497_amd import workloads as W

pytestmark = pytest.mark.gpu


def _gpu(Pi=4, theta=16, seed=0, profile=False, sparse=False, dense=None, dense_gains=None):
    from paper_2605_20497_amd import Partitioner
    return Partitioner(pi=Pi, theta=theta, seed=seed, profile=profile, sparse_proposal=sparse,
                       dense_proposal=dense, dense_gains=dense_gains)


def _compare_runs(hg, omega, delta, k=0, Pi=4, theta=16, seed=0, label="", sparse=False, dense=None,
                  dense_gains=None):
    print("case", label, "N", hg.n_nodes, "E", hg.n_hedges, "P", hg.n_pins, "omega", omega, "delta", delta,
          "k", k, "sparse", sparse, "dense", dense, "dense_gains", dense_gains, flush=True)
    og = oracle.Graph(hg)
    res = og.partition(omega, delta, k=k, Pi=Pi, theta=theta, seed=seed)
    g = _gpu(Pi, theta, seed, sparse=sparse, dense=dense, dense_gains=dense_gains)
    g.load(hg)
    g.hgp_set_limits(omega, delta, k)
    nl = g.hgp_coarsen()
    g.hgp_refine()
    assert nl == res.nlevels, (nl, res.nlevels)
    levels = g.hgp_get_levels()
    for lv in range(nl):
        o = res.levels[lv]
        assert (levels[lv, 0], levels[lv, 1], levels[lv, 2]) == (o["N"], o["E"], o["P"]), lv
        he_off, nsrc, pins, nw = g.hgp_get_level_graph(lv)
        ooff, onsrc, opins, ohw, onw = res.graph(lv).csr()
        assert np.array_equal(he_off, ooff) and np.array_equal(nsrc, onsrc), lv
        assert np.array_equal(pins, opins) and np.array_equal(nw, onw), lv
    for lv in range(res.ncoarsened):
        cand, score, match = g.hgp_get_proposal(lv)
        ocand, oscore, omatch = res.proposal(lv)
        assert np.array_equal(cand, ocand), ("cand", lv)
        assert np.array_equal(score, oscore), ("score", lv)
        assert np.array_equal(match, omatch), ("match", lv)
    for lv in range(nl - 1):
        assert np.array_equal(g.hgp_get_cluster_map(lv), res.gamma(lv)), ("gamma", lv)
    rho, nparts = g.hgp_get_partition()
    assert nparts == res.nparts
    assert np.array_equal(rho, res.rho(0))
    ev = g.hgp_evaluate()
    oev = og.evaluate(rho, nparts, omega, delta)
    for key in ("conn", "cutnet", "max_size", "max_inbound", "violations"):
        assert ev[key] == oev[key], key
    assert ev["n_parts"] == oev["nonempty"]
    assert ev["violations"] == 0
    off, part, cnt, cin = g.hgp_get_phi()
    ooff, opart, ocnt, ocin = og.phi(rho)
    assert np.array_equal(off, ooff) and np.array_equal(part, opart)
    assert np.array_equal(cnt, ocnt) and np.array_equal(cin, ocin)
    g.close()
    return res


SMALL_CASES = [
    # (n, e, max_card, seed, max_src, max_hw, max_nw, omega, delta)
    (60, 50, 6, 1, 1, 1, 1, 8, 40),
    (120, 100, 9, 2, 3, 4, 3, 12, 60),
    (200, 260, 12, 3, 1, 2, 1, 16, 90),
    (300, 200, 30, 4, 2, 1, 2, 40, 300),
    (150, 400, 5, 5, 0, 3, 1, 10, 1000),
    (500, 450, 20, 6, 1, 1, 4, 64, 200),
]


@pytest.mark.parametrize("case", SMALL_CASES, ids=lambda c: "n%d-e%d-s%d" % (c[0], c[1], c[3]))
def test_small_random_full_pipeline(case):
    n, e, card, seed, msrc, mhw, mnw, omega, delta = case
    hg = W.random_small(n, e, card, seed, max_src=msrc, max_hw=mhw, max_nw=mnw)
    _compare_runs(hg, omega, delta, label="small-%d" % seed)


@pytest.mark.parametrize("case", SMALL_CASES[:4], ids=lambda c: "n%d-e%d-s%d" % (c[0], c[1], c[3]))
def test_small_random_sparse_proposal(case):
    n, e, card, seed, msrc, mhw, mnw, omega, delta = case
    hg = W.random_small(n, e, card, seed, max_src=msrc, max_hw=mhw, max_nw=mnw)
    _compare_runs(hg, omega, delta, label="sparse-%d" % seed, sparse=True)


@pytest.mark.parametrize("case", SMALL_CASES, ids=lambda c: "n%d-e%d-s%d" % (c[0], c[1], c[3]))
def test_small_random_dense_proposal(case):
    # every level's proposal through the MFMA products
    n, e, card, seed, msrc, mhw, mnw, omega, delta = case
    hg = W.random_small(n, e, card, seed, max_src=msrc, max_hw=mhw, max_nw=mnw)
    _compare_runs(hg, omega, delta, label="dense-%d" % seed, dense=True)


def test_dense_proposal_snn_and_rand_4k_e32():
    hg = W.random_snn(1024, 15, 3)
    _compare_runs(hg, 64, 256, label="snn-1k-dense", dense=True)
    hg = W.random_snn(4096, 95, 6)
    _compare_runs(hg, 256, 1024, label="snn-4k-e96-dense", dense=True)
    hg = W.layered_snn(4, 512, 31, 128, 0.8, seed=1)
    _compare_runs(hg, 64, 512, label="layered-2k-dense", dense=True)
    hg = W.rand_4k_e32()
    _compare_runs(hg, hg.omega, hg.delta, label="rand-4k-e32-dense", dense=True)


def test_sparse_proposal_with_passes():
    # Neighbourhoods (~7,000) above half the 4,096-slot table force several
    # hashed passes per node.
    hg = W.random_snn(8192, 95, 6)
    _compare_runs(hg, 512, 2048, label="snn-8k-sparse", sparse=True)


def test_snn_shaped_small():
    hg = W.random_snn(1024, 15, 3)
    _compare_runs(hg, 64, 256, label="snn-1k")


def test_layered_small():
    hg = W.layered_snn(4, 512, 31, 128, 0.8, seed=1)
    _compare_runs(hg, 64, 512, label="layered-2k")


def test_pi_and_theta_variants():
    hg = W.random_snn(700, 11, 9)
    _compare_runs(hg, 48, 200, Pi=1, theta=4, label="pi1")
    _compare_runs(hg, 48, 200, Pi=8, theta=6, seed=5, label="pi8")


def test_rand_4k_e32_full():
    hg = W.rand_4k_e32()
    _compare_runs(hg, hg.omega, hg.delta, label="rand-4k-e32")


def test_edge_cases():
    # no h-edges at all: every node isolated, pairing by size only
    nw = np.array([3, 1, 6, 2, 5, 4, 1, 7, 2, 2], np.int32)
    hg = W.Hypergraph(10, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32),
                      np.zeros(0, np.int32), nw)
    _compare_runs(hg, 8, 5, label="no-edges")
    # single node
    hg = W.Hypergraph(1, np.array([0, 1], np.int64), np.array([1], np.int32), np.array([0], np.int32),
                      np.ones(1, np.int32), np.ones(1, np.int32))
    _compare_runs(hg, 1, 0, label="one-node")
    # single-pin h-edges, zero-source h-edges, caps so loose that one part remains
    hg = W.random_small(80, 90, 4, 17, max_src=0, max_hw=5)
    _compare_runs(hg, 80, 90, label="one-part")
    hg = W.random_small(64, 64, 1, 18, max_src=1)
    _compare_runs(hg, 4, 64, label="singletons")


def test_kway_small_netlist():
    hg = W.netlist(6000, 6600, 2, 80, 2.827, 256, 0.9, 8, seed=2, k=8, delta=1 << 15)
    _compare_runs(hg, hg.omega, hg.delta, k=8, label="netlist-6k-k8")


@pytest.mark.parametrize("rep", [0, 11])
def test_refine_rep_step(rep):
    hg = W.random_small(400, 380, 10, 33, max_src=2, max_hw=3, max_nw=2)
    og = oracle.Graph(hg)
    rng = np.random.default_rng(rep)
    P = 9
    rho0 = rng.integers(0, P, size=400).astype(np.int32)
    ev = og.evaluate(rho0, P)
    omega, delta = int(ev["max_size"]) + 2, int(ev["max_inbound"]) + 1
    g = _gpu()
    g.load(hg)
    g.hgp_set_limits(omega, delta, 0)
    rho = rho0
    for it in range(3):
        orho, od = og.refine_rep(rho, P, rep, 16, omega, delta)
        odst, ogain = og.moves(rho, P, rep, 16, omega)
        grho, gd = g.hgp_refine_rep(rho, P, rep)
        assert np.array_equal(gd["move_dst"], odst) and np.array_equal(gd["move_gain"], ogain)
        assert gd["moves"] == od["M"] and gd["kstar"] == od["kstar"] and gd["gain"] == od["applied_gain"]
        assert gd["links"] == od["links"]
        for key in ("seq", "seq_pd", "gseq", "C", "V"):
            assert np.array_equal(gd[key], od[key]), key
        assert np.array_equal(grho, orho)
        rho = orho


def test_evaluate_arbitrary_rho():
    hg = W.random_small(250, 300, 12, 44, max_src=2, max_hw=6, max_nw=3)
    og = oracle.Graph(hg)
    g = _gpu()
    g.load(hg)
    g.hgp_set_limits(30, 40, 0)
    rng = np.random.default_rng(0)
    for P in (1, 5, 250):
        rho = rng.integers(0, P, size=250).astype(np.int32)
        ev = g.hgp_evaluate(rho, P)
        oev = og.evaluate(rho, P, 30, 40)
        for key in ("conn", "cutnet", "max_size", "max_inbound", "violations"):
            assert ev[key] == oev[key]


def test_deterministic_across_runs():
    hg = W.random_snn(2048, 23, 4)
    outs = []
    for _ in range(2):
        g = _gpu()
        outs.append(g.partition(hg, 96, 400)[0])
        g.close()
    assert np.array_equal(outs[0], outs[1])


def test_error_paths():
    from paper_2605_20497_amd import HgpError, HGP_E_INVALID, HGP_E_INFEASIBLE, HGP_E_STATE
    g = _gpu()
    with pytest.raises(HgpError) as ei:  # a pin both source and destination
        g.hgp_load_csr(4, np.array([0, 3]), np.array([1], np.int32), np.array([1, 1, 2], np.int32))
    assert ei.value.status == HGP_E_INVALID
    with pytest.raises(HgpError) as ei:  # unsorted destinations
        g.hgp_load_csr(4, np.array([0, 3]), np.array([1], np.int32), np.array([0, 3, 2], np.int32))
    assert ei.value.status == HGP_E_INVALID
    with pytest.raises(HgpError) as ei:  # pin out of range
        g.hgp_load_csr(4, np.array([0, 2]), np.array([1], np.int32), np.array([0, 4], np.int32))
    assert ei.value.status == HGP_E_INVALID
    with pytest.raises(HgpError) as ei:
        g.hgp_coarsen()
    assert ei.value.status == HGP_E_STATE
    hg = W.random_small(30, 20, 5, 1, max_nw=5)
    g.load(hg)
    with pytest.raises(HgpError) as ei:  # a node heavier than omega
        g.hgp_set_limits(2, 100, 0)
    assert ei.value.status == HGP_E_INFEASIBLE
    g.hgp_set_limits(10, 100, 0)  # the context stays usable
    g.hgp_coarsen()
    g.hgp_refine()
    g.close()


def test_profile_family_mask():
    from paper_2605_20497_amd import KERNEL_FAMILIES, Partitioner
    hg = W.random_snn(1024, 15, 3)
    g = Partitioner(profile=True, profile_families=("propose",))
    g.partition(hg, 64, 256)
    st = g.hgp_kernel_stats()
    assert list(st) == KERNEL_FAMILIES
    assert st["propose"][0] > 0
    assert all(v[0] == 0 for k, v in st.items() if k != "propose")
    g.close()


def test_large_hedges_both_inseq_kernels():
    # h-edges up to 420 pins: the in-sequence outcome comes from the event-list
    # kernel for h-edges of at most 256 pins and from the all-pairs kernel above
    hg = W.random_small(1200, 260, 420, 7, max_src=2, max_hw=3, max_nw=2, min_card=40)
    assert int(np.diff(hg.he_off).max()) > 256
    _compare_runs(hg, 64, 400, label="large-hedges")


def test_gains_work_counter():
    # the profiled gains sweep counts the Phi row entries it reads:
    # sum over n and e in I(n) of lambda(e) = sum over e of |e| lambda(e)
    from paper_2605_20497_amd import Partitioner
    hg = W.random_small(400, 380, 10, 33, max_src=2, max_hw=3, max_nw=2)
    rho0 = np.random.default_rng(5).integers(0, 9, size=400).astype(np.int32)
    g = Partitioner(profile=True, profile_families=("gains",))
    g.load(hg)
    g.hgp_set_limits(10 ** 6, 10 ** 6, 0)
    g.hgp_reset_kernel_stats()
    g.hgp_refine_rep(rho0, 9, 0)
    work = g.hgp_kernel_work()
    card = np.diff(hg.he_off)
    lam = np.array([len(set(rho0[hg.pins[hg.he_off[e]:hg.he_off[e + 1]]].tolist())) for e in range(hg.n_hedges)])
    assert work["gains"] == int((card * lam).sum())
    assert all(v == 0 for k, v in work.items() if k != "gains")
    g.close()


@pytest.mark.parametrize("case", SMALL_CASES, ids=lambda c: "n%d-e%d-s%d" % (c[0], c[1], c[3]))
def test_small_random_dense_gains(case):
    # every level's in-isolation moves through the MFMA product (weights up to 4)
    n, e, card, seed, msrc, mhw, mnw, omega, delta = case
    hg = W.random_small(n, e, card, seed, max_src=msrc, max_hw=mhw, max_nw=mnw)
    _compare_runs(hg, omega, delta, label="dense-gains-%d" % seed, dense_gains=True)


def test_dense_gains_snn_netlist_large_weights():
    hg = W.random_snn(4096, 95, 6)
    _compare_runs(hg, 128, 1024, label="snn-4k-dense-gains", dense_gains=True)
    hg = W.netlist(6000, 6600, 2, 300, 2.827, 256, 0.9, 8, seed=9, k=8, delta=1 << 15)
    _compare_runs(hg, hg.omega, hg.delta, k=8, label="netlist-6k-k8-dense-gains", dense_gains=True)
    # h-edge weights up to 300,000: three 7-bit digit planes
    hg = W.random_small(700, 800, 40, 21, max_src=2, max_hw=300000, max_nw=3)
    _compare_runs(hg, 48, 400, label="heavy-weights-dense-gains", dense_gains=True)


def test_dense_gains_rep_step():
    # one repetition with an arbitrary partition: moves equal the oracle's
    hg = W.random_small(400, 380, 10, 33, max_src=2, max_hw=3, max_nw=2)
    og = oracle.Graph(hg)
    rho0 = np.random.default_rng(2).integers(0, 9, size=400).astype(np.int32)
    ev = og.evaluate(rho0, 9)
    omega, delta = int(ev["max_size"]) + 2, int(ev["max_inbound"]) + 1
    g = _gpu(dense_gains=True)
    g.load(hg)
    g.hgp_set_limits(omega, delta, 0)
    for rep in (0, 11):
        odst, ogain = og.moves(rho0, 9, rep, 16, omega)
        grho, gd = g.hgp_refine_rep(rho0, 9, rep)
        assert np.array_equal(gd["move_dst"], odst) and np.array_equal(gd["move_gain"], ogain)
    g.close()


@pytest.mark.parametrize("mode", [1, 2])
def test_delta_variants_full_pipeline(mode):
    # outbound (1) and incident (2) Delta: the library relabels pin roles on
    # the device at load; the oracle relabels the same input on the host
    from paper_2605_20497_amd import Partitioner
    for hg, omega, delta in ((W.random_small(300, 260, 14, 8, max_src=2, max_hw=2), 24, 40),
                             (W.random_snn(2048, 23, 4), 64, 300)):
        print("case delta_mode", mode, "N", hg.n_nodes, "P", hg.n_pins, flush=True)
        og = oracle.Graph(hg, delta_mode=mode)
        res = og.partition(omega, delta, Pi=4, theta=16, seed=0)
        g = Partitioner(delta_mode=mode)
        g.load(hg)
        g.hgp_set_limits(omega, delta, 0)
        assert g.hgp_coarsen() == res.nlevels
        g.hgp_refine()
        rho, _ = g.hgp_get_partition()
        assert np.array_equal(rho, res.rho(0))
        ev = g.hgp_evaluate()
        assert ev["conn"] == res.conn and ev["violations"] == 0
        # evaluation of an arbitrary partition under the variant
        r2 = np.random.default_rng(mode).integers(0, 7, size=hg.n_nodes).astype(np.int32)
        e2, o2 = g.hgp_evaluate(r2, 7), og.evaluate(r2, 7)
        assert (e2["conn"], e2["max_inbound"]) == (o2["conn"], o2["max_inbound"])
        g.close()


def test_no_chains_ablation():
    from paper_2605_20497_amd import Partitioner
    for hg, omega, delta in ((W.random_snn(1024, 15, 3), 64, 256), (W.random_snn(4096, 95, 6), 128, 1024)):
        print("case no-chains N", hg.n_nodes, flush=True)
        res = oracle.Graph(hg).partition(omega, delta, Pi=4, theta=16, seed=0, chains=False)
        g = Partitioner(no_chains=True)
        g.load(hg)
        g.hgp_set_limits(omega, delta, 0)
        assert g.hgp_coarsen() == res.nlevels
        g.hgp_refine()
        rho, _ = g.hgp_get_partition()
        assert np.array_equal(rho, res.rho(0))
        assert g.hgp_evaluate()["conn"] == res.conn
        g.close()


def test_greedy_matching_ablation():
    # greedy matching rounds against the oracle's, every level's matching and
    # the final partition; the 20,000-node case takes the per-depth kernels,
    # the others the single-workgroup matching
    from paper_2605_20497_amd import Partitioner
    cases = ((W.random_snn(1024, 15, 3), 64, 256), (W.random_snn(4096, 95, 6), 128, 1024),
             (W.random_snn(20000, 11, 8), 256, 1024))
    for hg, omega, delta in cases:
        print("case greedy N", hg.n_nodes, flush=True)
        res = oracle.Graph(hg).partition(omega, delta, Pi=4, theta=16, seed=0, greedy=True)
        g = Partitioner(greedy_matching=True)
        g.load(hg)
        g.hgp_set_limits(omega, delta, 0)
        assert g.hgp_coarsen() == res.nlevels
        for lv in range(res.ncoarsened):
            oc, os_, om = res.proposal(lv)
            gc, gs, gm = g.hgp_get_proposal(lv)
            assert np.array_equal(gm, om), lv
        g.hgp_refine()
        rho, _ = g.hgp_get_partition()
        assert np.array_equal(rho, res.rho(0))
        assert g.hgp_evaluate()["conn"] == res.conn
        g.close()


def test_dense_work_counters():
    # the multiply-adds the library reports for the two dense products equal
    # the padded-size formulas: (planes + 1) x 128^2 x tile pairs x Epad for
    # the proposal, planes x Npad x Ppad x Epad for the moves
    from paper_2605_20497_amd import Partitioner
    hg = W.random_snn(1024, 15, 3)
    g = Partitioner(profile=True, profile_families=("dense_gemm", "gains_gemm"), dense_proposal=True,
                    dense_gains=True)
    g.load(hg)
    g.hgp_set_limits(64, 256, 0)
    nl = g.hgp_coarsen()
    g.hgp_refine()
    work = g.hgp_kernel_work()
    st = g.hgp_kernel_stats()
    levels = g.hgp_get_levels()
    hw = hg.hedge_w.astype(np.int64)
    exp_p = 0
    for lv in range(st["dense_gemm"][0]):
        N, E = int(levels[lv, 0]), int(levels[lv, 1])
        card = np.maximum(np.diff(g.hgp_get_level_graph(lv, what=("he_off",))[0]), 1)
        t = np.maximum(1, (hw[:E] << 16) // card)
        planes = 1
        while planes <= 3 and (int(t.max()) >> (7 * planes)) != 0:
            planes += 1
        nt = (N + 127) // 128
        epad = (((E + 31) // 32 + 3) // 4 * 4) * 32
        exp_p += nt * (nt + 1) // 2 * 128 * 128 * epad * (planes + 1)
    assert st["dense_gemm"][0] == nl or st["dense_gemm"][0] == nl - 1
    assert work["dense_gemm"] == exp_p
    nparts = int(levels[nl - 1, 0])
    ppad = (nparts + 127) // 128 * 128
    assert st["gains_gemm"][0] >= nl  # at least one repetition per level
    per_level = [(int(levels[lv, 0]) + 127) // 128 * 128 * ppad *
                 ((((int(levels[lv, 1]) + 31) // 32 + 3) // 4 * 4) * 32) for lv in range(nl)]
    assert work["gains_gemm"] % 1 == 0 and work["gains_gemm"] >= sum(per_level)
    g.close()


@pytest.mark.parametrize("theta", [2, 4])
def test_early_exit_with_second_half_commit(theta):
    # A graph whose level-0 first-half repetitions apply nothing while a
    # second-half (size-aware) one applies a move (Reading R25): the library's
    # early exit must still run the second half.
    hg = W.random_small(14, 16, 4, 1, max_src=1, max_hw=3, max_nw=3)
    _compare_runs(hg, 7, 10 ** 6, theta=theta, label="r25-theta%d" % theta)
