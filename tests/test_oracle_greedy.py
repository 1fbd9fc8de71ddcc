"""Pins of the oracle's greedy matching, the prototype heuristic that the
ablation of Sec. VII-D swaps in for the exact matching (Reading R28: every
two-cycle of the proposal graph is matched, and each node that its parent
leaves unmatched, or each root without a partner, takes the child proposing
to it with the highest score, ties to the larger id).  Expected matchings
are worked out by hand from that reading."""
import ctypes as C

import numpy as np
import pytest


def _greedy(oracle_mod, target, score, active=None):
    n = len(target)
    t = np.asarray(target, np.int32)
    s = np.asarray(score, np.uint64)
    a = np.ones(n, np.int8) if active is None else np.asarray(active, np.int8)
    m = np.zeros(n, np.int32)
    err = C.create_string_buffer(256)
    rc = oracle_mod.lib().hgpo_match_round_greedy(n, oracle_mod._p(a), oracle_mod._p(t), oracle_mod._p(s),
                                                  oracle_mod._p(m), err, 256)
    return rc, m, err.value.decode()


def _exact(oracle_mod, target, score):
    n = len(target)
    t = np.asarray(target, np.int32)
    s = np.asarray(score, np.uint64)
    a = np.ones(n, np.int8)
    m = np.zeros(n, np.int32)
    err = C.create_string_buffer(256)
    rc = oracle_mod.lib().hgpo_match_round(n, oracle_mod._p(a), oracle_mod._p(t), oracle_mod._p(s),
                                           oracle_mod._p(m), err, 256)
    assert rc == 0
    return m


def test_root_pair_forced_where_the_exact_matching_declines(oracle_mod):
    # 0 <-> 1 (score 5); 2 -> 0 and 3 -> 1 (score 4 each).  The exact matching
    # prefers {0,2} and {1,3} (8 > 5); the greedy one always takes the root
    # pair, which leaves 2 and 3 without partners.
    target = [1, 0, 0, 1]
    score = [5, 5, 4, 4]
    rc, m, _ = _greedy(oracle_mod, target, score)
    assert rc == 0
    assert m.tolist() == [1, 0, -1, -1]
    assert _exact(oracle_mod, target, score).tolist() == [2, 3, 0, 1]


def test_decisions_carried_down_with_ties_to_the_larger_id(oracle_mod):
    # 0 <-> 1 (6); 2 -> 1 (4); 3 -> 2 (3); 4 -> 2 (3); 5 -> 3 (2).
    # {0,1} matched; 2 is free and takes its best child: 3 and 4 tie at 3, the
    # larger id 4 wins; 3 is then free and takes 5.
    target = [1, 0, 1, 2, 2, 3]
    score = [6, 6, 4, 3, 3, 2]
    rc, m, _ = _greedy(oracle_mod, target, score)
    assert rc == 0
    assert m.tolist() == [1, 0, 4, 5, 2, 3]


def test_root_without_partner_and_score_order(oracle_mod):
    # 0 has no target; 1 -> 0 (2), 2 -> 0 (9), 3 -> 1 (1), 4 -> 2 (8).
    # 0 takes 2 (score 9 beats 2); 1 is free and takes 3; 4 stays unmatched
    # because its target 2 is taken.
    target = [-1, 0, 0, 1, 2]
    score = [0, 2, 9, 1, 8]
    rc, m, _ = _greedy(oracle_mod, target, score)
    assert rc == 0
    assert m.tolist() == [2, 3, 0, 1, -1]


def test_inactive_nodes_take_no_part(oracle_mod):
    # node 2 matched in an earlier round: inactive, and nobody targets it
    target = [1, 0, -1, 0]
    score = [5, 5, 0, 4]
    rc, m, _ = _greedy(oracle_mod, target, score, active=[1, 1, 0, 1])
    assert rc == 0
    assert m.tolist() == [1, 0, -1, -1]


def test_long_cycle_rejected(oracle_mod):
    rc, _, err = _greedy(oracle_mod, [1, 2, 0], [3, 3, 3])
    assert rc != 0 and "cycle" in err


def test_greedy_partition_is_valid(oracle_mod):
    from paper_2605_20497_amd import workloads as W
    hg = W.random_snn(600, 11, seed=4)
    g = oracle_mod.Graph(hg)
    res = g.partition(48, 200, greedy=True)
    ev = g.evaluate(res.rho(0), res.nparts, 48, 200)
    assert ev["violations"] == 0
    exact = g.partition(48, 200)
    # every level's matching is symmetric
    assert res.nlevels >= 2 and exact.nlevels >= 2
    for lv in range(res.ncoarsened):
        _, _, match = res.proposal(lv)
        for n, mm in enumerate(match.tolist()):
            if mm >= 0:
                assert match[mm] == n
