"""Pins of the oracle's coarsening (Sec. V): histogram, inter, validity,
top-Pi candidates, the pseudo-forest matching DP, isolated pairing and
coarse hypergraph construction."""
import numpy as np
import pytest

from paper_2605_20497_amd import workloads as W
from tests import _routes


def _tvec(g, hg):
    return np.array([g.tnorm(e) for e in range(hg.n_hedges)], dtype=np.uint64)


def test_tnorm_fixed_point_values(oracle_mod):
    # omega/|e| in 16-bit fixed point, floored, at least 1 (reading of Eq. neighbors_histogram)
    hg = W._assemble(5, [[0], [0], [1]], [[1], [1, 2, 3], [0, 2, 3, 4]], hedge_w=[1, 3, 1])
    g = oracle_mod.Graph(hg)
    assert g.tnorm(0) == 65536 // 2
    assert g.tnorm(1) == 3 * 65536 // 4
    assert g.tnorm(2) == 65536 // 5
    # noise cap: 10% of the mean over h-edges with >= 2 pins, floored
    assert g.noise_cap() == (32768 + 49152 + 13107) // 30


@pytest.mark.parametrize("seed", range(4))
def test_histogram_and_inter_match_matrix_products(oracle_mod, seed):
    hg = W.random_small(30, 40, 8, seed, max_src=2, max_hw=4)
    g = oracle_mod.Graph(hg)
    H, Hd = _routes.incidence_matrices(hg)
    t = _tvec(g, hg).astype(np.int64)
    eta = H.T @ (t[:, None] * H)         # eta(n,m) = sum_e [n in e][m in e] t(e)
    inter = Hd.T @ Hd                    # |in(n) ∩ in(m)|
    assert np.array_equal(eta, eta.T)
    for n in range(hg.n_nodes):
        for m in range(hg.n_nodes):
            if n == m:
                continue
            e_nm, i_nm = g.pair(n, m)
            assert e_nm == eta[n, m] and i_nm == inter[n, m]
            assert g.pair(m, n) == (e_nm, i_nm)


@pytest.mark.parametrize("seed", range(5))
def test_top_pi_candidates_by_sorting(oracle_mod, seed):
    hg = W.random_small(45, 60, 7, 20 + seed, max_src=2, max_hw=3, max_nw=3)
    omega, delta, Pi, nseed = 5, 9, 4, 7 + seed
    g = oracle_mod.Graph(hg)
    H, Hd = _routes.incidence_matrices(hg)
    t = _tvec(g, hg).astype(np.int64)
    eta = H.T @ (t[:, None] * H)
    inter = Hd.T @ Hd
    nin = Hd.sum(axis=0)
    cap = g.noise_cap()
    cand, score = g.propose(omega, delta, nseed, Pi)
    for n in range(hg.n_nodes):
        rows = []
        for m in range(hg.n_nodes):
            if m == n or eta[n, m] == 0:
                continue
            ok = hg.node_w[n] + hg.node_w[m] <= omega and nin[n] + nin[m] - inter[n, m] <= delta
            if ok:
                rows.append((int(eta[n, m]) + oracle_mod.noise(nseed, n, m, cap), m))
        rows.sort(key=lambda x: (-x[0], -x[1]))
        exp = rows[:Pi] + [(0, -1)] * (Pi - len(rows[:Pi]))
        assert [c for _, c in exp] == list(cand[n])
        assert [s for s, _ in exp] == [int(x) for x in score[n]]


def test_noise_symmetric_and_capped(oracle_mod):
    rng = np.random.default_rng(3)
    for _ in range(200):
        a, b = rng.integers(0, 1 << 31, size=2)
        cap = int(rng.integers(0, 5000))
        v = oracle_mod.noise(11, int(a), int(b), cap)
        assert v == oracle_mod.noise(11, int(b), int(a), cap)
        assert 0 <= v <= cap
    assert oracle_mod.noise(11, 3, 4, 0) == 0


def _random_proposal_graph(rng, n, p_edge=0.35, p_inactive=0.1):
    """Symmetric random weights on a random graph; each active node targets its
    max-id argmax (the construction of Eq. proposal_graph)."""
    w = np.zeros((n, n), np.int64)
    for a in range(n):
        for b in range(a + 1, n):
            if rng.random() < p_edge:
                w[a, b] = w[b, a] = int(rng.integers(1, 6))
    active = (rng.random(n) > p_inactive).astype(np.int8)
    target = np.full(n, -1, np.int32)
    score = np.zeros(n, np.uint64)
    for a in range(n):
        if not active[a]:
            continue
        best = None
        for b in range(n):
            if b != a and active[b] and w[a, b] > 0:
                if best is None or (w[a, b], b) > (w[a, best], best):
                    best = b
        if best is not None:
            target[a] = best
            score[a] = w[a, best]
    return active, target, score


@pytest.mark.parametrize("seed", range(40))
def test_match_round_is_maximum_weight(oracle_mod, seed):
    import ctypes as C
    rng = np.random.default_rng(seed)
    n = int(rng.integers(4, 15))
    active, target, score = _random_proposal_graph(rng, n)
    match = np.zeros(n, np.int32)
    err = C.create_string_buffer(256)
    rc = oracle_mod.lib().hgpo_match_round(n, oracle_mod._p(active), oracle_mod._p(target),
                                          oracle_mod._p(score), oracle_mod._p(match), err, 256)
    assert rc == 0, err.value
    edges = {}
    for a in range(n):
        if active[a] and target[a] >= 0:
            key = (min(a, target[a]), max(a, target[a]))
            edges[key] = int(score[a])
    total = 0
    for a in range(n):
        if match[a] >= 0:
            assert match[match[a]] == a
            key = (min(a, match[a]), max(a, match[a]))
            assert key in edges             # only proposal edges are matched
            if a < match[a]:
                total += edges[key]
    assert total == _routes.max_weight_matching_brute([(a, b, w) for (a, b), w in edges.items()])
    # maximal: no proposal edge with both ends free (scores are positive)
    for (a, b) in edges:
        assert match[a] >= 0 or match[b] >= 0


def test_match_round_rejects_long_cycle(oracle_mod):
    import ctypes as C
    active = np.ones(3, np.int8)
    target = np.array([1, 2, 0], np.int32)
    score = np.array([5, 5, 5], np.uint64)
    match = np.zeros(3, np.int32)
    err = C.create_string_buffer(256)
    rc = oracle_mod.lib().hgpo_match_round(3, oracle_mod._p(active), oracle_mod._p(target),
                                          oracle_mod._p(score), oracle_mod._p(match), err, 256)
    assert rc != 0 and b"cycle" in err.value


@pytest.mark.parametrize("seed", range(4))
def test_level_matching_rounds_properties(oracle_mod, seed):
    hg = W.random_small(80, 70, 6, 40 + seed, max_src=1, max_nw=2)
    omega, delta = 4, 12
    g = oracle_mod.Graph(hg)
    cand, score = g.propose(omega, delta, 0, 4)
    match, rp = g.match(omega, delta, cand, score)
    H, Hd = _routes.incidence_matrices(hg)
    nin = Hd.sum(axis=0)
    inter = Hd.T @ Hd
    assert rp.sum() == int((match > np.arange(80)).sum())
    for a in range(80):
        b = match[a]
        if b < 0:
            continue
        assert match[b] == a
        assert hg.node_w[a] + hg.node_w[b] <= omega
        if cand[a, 0] >= 0:           # matched in a round: a valid candidate pair
            assert any(cand[a, r] == b or cand[b, r] == a for r in range(4))  # same round
            assert nin[a] + nin[b] - inter[a, b] <= delta
        else:                         # isolated pairing uses the |in|+|in| over-estimate
            assert cand[b, 0] < 0 and nin[a] + nin[b] <= delta
    # every round's matching was maximal: a node left unmatched has no unmatched
    # candidate among the ones it proposed
    for a in range(80):
        if match[a] < 0:
            for c in cand[a]:
                if c >= 0:
                    assert match[c] >= 0


def test_isolated_pairing_two_pointer(oracle_mod):
    # No h-edges: every node is isolated; sizes 1..6, Omega 7.
    nw = np.array([3, 1, 6, 2, 5, 4, 1], np.int32)
    g = oracle_mod.Graph(n_nodes=7, he_off=np.zeros(1, np.int64), he_nsrc=np.zeros(0, np.int32),
                         pins=np.zeros(0, np.int32), node_w=nw)
    cand, score = g.propose(7, 10, 0, 4)
    assert (cand == -1).all()
    match, rp = g.match(7, 10, cand, score)
    pairs = {tuple(sorted((a, int(match[a])))) for a in range(7) if match[a] >= 0}
    # sorted by (size, id): 1(1) 6(1) 3(2) 0(3) 5(4) 4(5) 2(6); smallest with the
    # largest that fits: 1+2, 6+4, 3+5; node 0 is left.
    assert pairs == {(1, 2), (4, 6), (3, 5)}
    assert rp[4] == 3


@pytest.mark.parametrize("seed", range(5))
def test_contraction_invariants(oracle_mod, seed):
    hg = W.random_small(60, 50, 7, 60 + seed, max_src=3, max_hw=4, max_nw=3)
    omega, delta = 8, 40
    g = oracle_mod.Graph(hg)
    cand, score = g.propose(omega, delta, 0, 4)
    match, rp = g.match(omega, delta, cand, score)
    gamma, gc = g.contract(match)
    pairs = int((match > np.arange(60)).sum())
    assert gc.N == 60 - pairs and gc.E == hg.n_hedges
    he_off, nsrc, pins, hw, nw = gc.csr()
    assert nw.sum() == hg.node_w.sum()
    # coarse ids ordered by smallest member
    reps = [min(a, int(match[a])) if match[a] >= 0 else a for a in range(60)]
    assert np.array_equal(np.argsort(np.unique(reps)), np.arange(gc.N))
    # duality: Score(gamma) + Conn(gamma) = sum_e w(e) (|e| - 1)
    card0 = np.diff(hg.he_off)
    card1 = np.diff(he_off)
    score_g = int((hg.hedge_w.astype(np.int64) * (card0 - card1)).sum())
    conn_g = g.evaluate(gamma, gc.N)["conn"]
    assert score_g + conn_g == int((hg.hedge_w.astype(np.int64) * (card0 - 1)).sum())
    # level invariance of Conn, cut-net, sizes and D under rho = rho' o gamma
    rng = np.random.default_rng(seed)
    for _ in range(5):
        rho_c = rng.integers(0, 6, size=gc.N).astype(np.int32)
        a = g.evaluate(rho_c[gamma], 6, omega, delta)
        b = gc.evaluate(rho_c, 6, omega, delta)
        for k in ("conn", "cutnet", "violations"):
            assert a[k] == b[k]
        assert np.array_equal(a["part_size"], b["part_size"])
        assert np.array_equal(a["part_inbound"], b["part_inbound"])
    # in(n') = in(a) ∪ in(b); out(n') = (out(a) ∪ out(b)) \ in(n')
    off0, nin0, inc0 = g.incidence()
    off1, nin1, inc1 = gc.incidence()
    members = {}
    for a in range(60):
        members.setdefault(int(gamma[a]), []).append(a)
    for c, ms in members.items():
        ins = set()
        outs = set()
        for a in ms:
            ins |= set(inc0[off0[a]:off0[a] + nin0[a]].tolist())
            outs |= set(inc0[off0[a] + nin0[a]:off0[a + 1]].tolist())
        assert inc1[off1[c]:off1[c] + nin1[c]].tolist() == sorted(ins)
        assert inc1[off1[c] + nin1[c]:off1[c + 1]].tolist() == sorted(outs - ins)
