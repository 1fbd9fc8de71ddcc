"""Pins of the oracle's multilevel driver (Sec. III) and k-way adapter
(Sec. VII-A): validity, optimality bound by exhaustive enumeration, special
cases and level invariants."""
import numpy as np
import pytest

from paper_2605_20497_amd import workloads as W
from tests import _routes


@pytest.mark.parametrize("seed", range(4))
def test_tiny_graphs_valid_and_above_bruteforce_optimum(oracle_mod, seed):
    hg = W.random_small(11, 9, 5, 300 + seed, max_src=2, max_hw=3, max_nw=2)
    omega, delta = 5, 5
    R, conn, valid = _routes.brute_force_all(hg, omega, delta)
    opt = int(conn[valid].min())
    g = oracle_mod.Graph(hg)
    res = g.partition(omega, delta, Pi=4, theta=16)
    rho = res.rho(0)
    ev = g.evaluate(rho, res.nparts, omega, delta)
    assert ev["violations"] == 0
    assert ev["conn"] == res.conn >= opt


def test_bell_12_enumeration_size():
    assert _routes.all_rgs(12).shape[0] == 4213597


def test_twelve_node_graph_against_all_partitions(oracle_mod):
    hg = W.random_small(12, 10, 5, 77, max_src=2, max_hw=2, max_nw=2)
    omega, delta = 6, 6
    R, conn, valid = _routes.brute_force_all(hg, omega, delta)
    assert R.shape[0] == 4213597
    g = oracle_mod.Graph(hg)
    res = g.partition(omega, delta)
    ev = g.evaluate(res.rho(0), res.nparts, omega, delta)
    assert ev["violations"] == 0 and ev["conn"] >= int(conn[valid].min())


def test_loose_caps_give_one_partition(oracle_mod):
    hg = W.random_small(50, 40, 6, 9, max_src=2, max_hw=3, max_nw=3)
    W_ = int(hg.node_w.sum())
    g = oracle_mod.Graph(hg)
    res = g.partition(W_, hg.n_hedges)
    rho = res.rho(0)
    assert len(np.unique(rho)) == 1
    assert res.conn == 0


def test_levels_conn_monotone_and_gamma_sizes(oracle_mod):
    hg = W.random_snn(512, 15, 4, omega=32, delta=160)
    g = oracle_mod.Graph(hg)
    res = g.partition(hg.omega, hg.delta)
    # projection keeps Conn; refinement never raises it
    for lv in range(res.nlevels - 1):
        assert res.levels[lv]["conn_after"] <= res.levels[lv + 1]["conn_after"]
        gam = res.gamma(lv)
        assert gam.max() + 1 == res.levels[lv + 1]["N"]
        assert res.levels[lv + 1]["N"] == res.levels[lv]["N"] - sum(res.levels[lv]["pairs"])
    ev = g.evaluate(res.rho(0), res.nparts, hg.omega, hg.delta)
    assert ev["violations"] == 0 and ev["conn"] == res.conn


def test_early_exit_is_result_neutral(oracle_mod):
    hg = W.random_snn(600, 20, 8, omega=40, delta=250)
    g = oracle_mod.Graph(hg)
    a = g.partition(hg.omega, hg.delta, early_exit=True)
    b = g.partition(hg.omega, hg.delta, early_exit=False)
    assert np.array_equal(a.rho(0), b.rho(0)) and a.conn == b.conn


def test_kway_initial_partition(oracle_mod):
    hg = W.netlist(3000, 3300, 2, 60, 2.827, 64, 0.9, 8, seed=1, k=8, delta=1 << 15)
    g = oracle_mod.Graph(hg)
    rho = g.kway_initial(8, hg.omega, hg.delta)
    ev = g.evaluate(rho, 8, hg.omega, hg.delta)
    assert ev["violations"] == 0
    res = g.partition(hg.omega, hg.delta, k=8)
    ev = g.evaluate(res.rho(0), 8, hg.omega, hg.delta)
    assert res.nparts == 8 and ev["violations"] == 0
