"""Pins of the oracle's refinement (Sec. VI): gains, moves, the sequence of
chains, in-sequence gains, the event-based validity of every prefix and the
applied prefix."""
import numpy as np
import pytest

from paper_2605_20497_amd import workloads as W


def _setup(oracle_mod, seed, n=60, e=70, card=6, nparts=8, omega=None, delta=None):
    hg = W.random_small(n, e, card, 200 + seed, max_src=2, max_hw=3, max_nw=2)
    g = oracle_mod.Graph(hg)
    rng = np.random.default_rng(seed)
    rho = rng.integers(0, nparts, size=n).astype(np.int32)
    ev = g.evaluate(rho, nparts)
    if omega is None:
        omega = int(ev["max_size"]) + 2
    if delta is None:
        delta = int(ev["max_inbound"]) + 1
    return hg, g, rho, nparts, omega, delta


@pytest.mark.parametrize("seed", range(6))
def test_gain_is_connectivity_difference(oracle_mod, seed):
    hg, g, rho, P, omega, delta = _setup(oracle_mod, seed)
    base = g.evaluate(rho, P)["conn"]
    for n in range(0, hg.n_nodes, 3):
        for p in range(P):
            if p == rho[n]:
                continue
            r2 = rho.copy()
            r2[n] = p
            assert g.gain(rho, n, p) == base - g.evaluate(r2, P)["conn"]


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("rep", [0, 12])
def test_moves_are_best_improving(oracle_mod, seed, rep):
    hg, g, rho, P, omega, delta = _setup(oracle_mod, seed)
    theta = 16
    dst, gain = g.moves(rho, P, rep, theta, omega)
    base = g.evaluate(rho, P)
    size = base["part_size"]
    for n in range(hg.n_nodes):
        best = None
        for p in range(P):
            if p == rho[n]:
                continue
            if rep >= theta // 2 and hg.node_w[n] + size[p] > omega:
                continue
            r2 = rho.copy()
            r2[n] = p
            gp = base["conn"] - g.evaluate(r2, P)["conn"]
            if gp > 0 and (best is None or (gp, p) > best):
                best = (gp, p)
        if best is None:
            assert dst[n] == -1
        else:
            assert (int(gain[n]), int(dst[n])) == best


def _apply(rho, seq, seq_pd, k):
    r = rho.copy()
    r[seq[:k]] = seq_pd[:k]
    return r


@pytest.mark.parametrize("seed", range(10))
@pytest.mark.parametrize("rep", [0, 9])
def test_sequence_prefix_gains_and_violations(oracle_mod, seed, rep):
    """C_k (cumulative in-sequence gain) equals Conn(rho_0) - Conn(rho_k) and V_k
    equals the from-scratch violated-partition count, for every prefix k."""
    hg, g, rho, P, omega, delta = _setup(oracle_mod, seed, omega=None, delta=None)
    # tight caps so that some prefixes are invalid
    omega = max(int(hg.node_w.max()), int(g.evaluate(rho, P)["max_size"]))
    delta = int(g.evaluate(rho, P)["max_inbound"])
    new_rho, d = g.refine_rep(rho, P, rep, 16, omega, delta)
    M = d["M"]
    base = g.evaluate(rho, P, omega, delta)
    assert d["C"][0] == 0 and d["V"][0] == base["violations"]
    for k in range(M + 1):
        rk = _apply(rho, d["seq"], d["seq_pd"], k)
        ev = g.evaluate(rk, P, omega, delta)
        assert d["C"][k] == base["conn"] - ev["conn"]
        assert d["V"][k] == ev["violations"]
    # k* = shortest valid prefix of maximal cumulative gain (k = 0 allowed)
    cands = [k for k in range(M + 1) if k == 0 or d["V"][k] == 0]
    best = max(d["C"][k] for k in cands)
    assert d["kstar"] == min(k for k in cands if d["C"][k] == best)
    assert np.array_equal(new_rho, _apply(rho, d["seq"], d["seq_pd"], d["kstar"]))
    ev = g.evaluate(new_rho, P, omega, delta)
    assert ev["conn"] <= base["conn"]
    assert ev["violations"] <= base["violations"] or d["kstar"] == 0


@pytest.mark.parametrize("seed", range(8))
def test_sequence_is_ranked_chains(oracle_mod, seed):
    hg, g, rho, P, omega, delta = _setup(oracle_mod, seed, n=120, e=150, nparts=6)
    dst, gain = g.moves(rho, P, 0, 16, omega)
    new_rho, d = g.refine_rep(rho, P, 0, 16, omega, delta)
    movers = np.nonzero(dst >= 0)[0]
    assert sorted(d["seq"].tolist()) == movers.tolist()          # a permutation of the movers
    assert np.array_equal(d["seq_pd"], dst[d["seq"]])
    cl = d["chain_len"]
    assert cl.sum() == d["M"]
    pos = 0
    totals = []
    for L in cl:
        items = d["seq"][pos:pos + L]
        for a, b in zip(items[:-1], items[1:]):
            assert rho[b] == dst[a]                               # p_s of next = p_d of previous
        totals.append((int(gain[items].sum()), int(items[0])))
        pos += L
    assert totals == sorted(totals, key=lambda t: (-t[0], t[1]))   # ranked by total gain


def test_rep_keeps_valid_state(oracle_mod):
    hg = W.random_small(200, 220, 6, 5, max_src=1, max_nw=3)
    g = oracle_mod.Graph(hg)
    P = 10
    rho = (np.arange(200) % P).astype(np.int32)
    ev = g.evaluate(rho, P)
    omega, delta = int(ev["max_size"]) + 3, int(ev["max_inbound"]) + 2
    conn = ev["conn"]
    for rep in range(16):
        rho, d = g.refine_rep(rho, P, rep, 16, omega, delta)
        ev = g.evaluate(rho, P, omega, delta)
        assert ev["violations"] == 0
        assert ev["conn"] == conn - d["applied_gain"]
        assert ev["conn"] <= conn
        conn = ev["conn"]
