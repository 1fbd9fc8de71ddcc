"""Pins of the oracle's evaluator (Sec. II-B): pins(p,e), pins_in(p,e), sizes,
distinct inbound h-edges D(p), connectivity and cut-net."""
import os

import numpy as np
import pytest

from paper_2605_20497_amd import workloads as W
from tests import _routes

HERE = os.path.dirname(os.path.abspath(__file__))


def test_splitmix64_published_vectors(oracle_mod):
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "splitmix64.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for a, b in rows:
        assert oracle_mod.mix64(int(a, 16)) == int(b, 16)


@pytest.mark.parametrize("seed", range(6))
def test_eval_matches_incidence_products(oracle_mod, seed):
    hg = W.random_small(40, 30, 9, seed, max_src=3, max_hw=5, max_nw=4)
    g = oracle_mod.Graph(hg)
    rng = np.random.default_rng(100 + seed)
    nparts = 7
    rho = rng.integers(0, nparts, size=hg.n_nodes).astype(np.int32)
    ev = g.evaluate(rho, nparts, omega=12, delta=9)
    ref = _routes.eval_by_products(hg, rho, nparts)
    assert ev["conn"] == ref["conn"]
    assert ev["cutnet"] == ref["cutnet"]
    assert np.array_equal(ev["part_size"], ref["size"])
    assert np.array_equal(ev["part_inbound"], ref["D"])
    assert ev["violations"] == int(((ref["size"] > 12) | (ref["D"] > 9)).sum())
    # Sparse Phi rows against the dense products.
    off, part, cnt, cin = g.phi(rho)
    dense = np.zeros((hg.n_hedges, nparts), np.int64)
    dense_in = np.zeros_like(dense)
    for e in range(hg.n_hedges):
        sl = slice(off[e], off[e + 1])
        assert np.all(np.diff(part[sl]) > 0)
        dense[e, part[sl]] = cnt[sl]
        dense_in[e, part[sl]] = cin[sl]
    assert np.array_equal(dense, ref["Phi"])
    assert np.array_equal(dense_in, ref["Phi_in"])


def test_phi_row_sums(oracle_mod):
    hg = W.random_small(60, 50, 12, 7, max_src=4)
    g = oracle_mod.Graph(hg)
    rho = np.random.default_rng(1).integers(0, 5, size=60).astype(np.int32)
    off, part, cnt, cin = g.phi(rho)
    for e in range(hg.n_hedges):
        s, d = hg.edge(e)
        assert cnt[off[e]:off[e + 1]].sum() == len(s) + len(d)   # sum_p Phi(e,p) = |e|
        assert cin[off[e]:off[e + 1]].sum() == len(d)            # sum_p Phi_in(e,p) = |dst(e)|


def test_eval_special_cases(oracle_mod):
    hg = W.random_small(30, 25, 8, 3, max_src=2, max_hw=7)
    g = oracle_mod.Graph(hg)
    one = np.zeros(30, np.int32)
    ev = g.evaluate(one, 1)
    assert ev["conn"] == 0 and ev["cutnet"] == 0
    assert ev["part_inbound"][0] == sum(1 for e in range(hg.n_hedges) if len(hg.edge(e)[1]) > 0)
    single = np.arange(30, dtype=np.int32)
    ev = g.evaluate(single, 30)
    card = np.diff(hg.he_off)
    assert ev["conn"] == int((hg.hedge_w.astype(np.int64) * (card - 1)).sum())
    assert ev["cutnet"] == int(hg.hedge_w[card > 1].astype(np.int64).sum())
    for n in range(30):  # each singleton's D is |in(n)|
        assert ev["part_inbound"][n] == sum(1 for e in range(hg.n_hedges) if n in hg.edge(e)[1])


def test_two_pin_edges_give_graph_cut(oracle_mod):
    hg = W.random_small(20, 40, 2, 5, max_src=1, max_hw=3, min_card=2)
    g = oracle_mod.Graph(hg)
    rho = np.random.default_rng(2).integers(0, 3, size=20).astype(np.int32)
    ev = g.evaluate(rho, 3)
    cut = 0
    for e in range(hg.n_hedges):
        s, d = hg.edge(e)
        a, b = np.concatenate([s, d])
        cut += int(hg.hedge_w[e]) * int(rho[a] != rho[b])
    assert ev["conn"] == cut == ev["cutnet"]


def test_bruteforce_all_partitions_conn(oracle_mod):
    """Every partition of a 10-node graph: Conn from the oracle equals the
    enumeration's on a sample, and the enumeration's per-partition validity
    agrees with the oracle's violation count."""
    hg = W.random_small(10, 8, 5, 11, max_src=2, max_hw=3, max_nw=2)
    g = oracle_mod.Graph(hg)
    R, conn, valid = _routes.brute_force_all(hg, omega=5, delta=4)
    assert R.shape[0] == 115975  # Bell(10)
    rng = np.random.default_rng(0)
    for i in rng.choice(R.shape[0], 400, replace=False):
        rho = R[i].astype(np.int32)
        ev = g.evaluate(rho, 10, omega=5, delta=4)
        assert ev["conn"] == conn[i]
        assert (ev["violations"] == 0) == bool(valid[i])


def test_validation_rejects_malformed(oracle_mod):
    ok = W.random_small(8, 5, 4, 1)
    with pytest.raises(oracle_mod.OracleError):  # source also a destination
        oracle_mod.Graph(n_nodes=4, he_off=np.array([0, 3]), he_nsrc=np.array([1], np.int32),
                         pins=np.array([1, 1, 2], np.int32))
    with pytest.raises(oracle_mod.OracleError):  # unsorted destination block
        oracle_mod.Graph(n_nodes=4, he_off=np.array([0, 3]), he_nsrc=np.array([1], np.int32),
                         pins=np.array([0, 3, 2], np.int32))
    with pytest.raises(oracle_mod.OracleError):  # pin out of range
        oracle_mod.Graph(n_nodes=4, he_off=np.array([0, 2]), he_nsrc=np.array([1], np.int32),
                         pins=np.array([0, 4], np.int32))
    with pytest.raises(oracle_mod.OracleError):  # empty h-edge
        oracle_mod.Graph(n_nodes=4, he_off=np.array([0, 0]), he_nsrc=np.array([0], np.int32),
                         pins=np.array([], np.int32))
    oracle_mod.Graph(ok)
