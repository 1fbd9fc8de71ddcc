"""Hand-worked pins of the oracle's readings of silent or ambiguous passages.

Each case is small enough that its expected outcome is derived by hand in the
comments from the reading alone (Sec. V-C, V-D, VI-C, VI-D, VII-A and
Readings R3, R8, R15-R17, R21, R25), so a plausible slip in the oracle (a
flipped sign, a wrong window, a reversed tie-break, the wrong pointer moved)
changes the result.  tests/test_oracle_mutants.py builds such slips into
copies of the oracle and checks that these cases catch every one of them.
"""
import numpy as np
import pytest

from paper_2605_20497_amd import workloads as W

G7 = 10_000_000  # the integer grade is 10^7 x the paper's grade (Reading R16)


def seq_of(oracle_mod, moves, n, node_w=None, n_in=None, rounds=16):
    nw = np.ones(n, np.int64) if node_w is None else np.asarray(node_w, np.int64)
    nin = np.zeros(n, np.int32) if n_in is None else np.asarray(n_in, np.int32)
    return oracle_mod.sequence(nw, nin, moves, rounds)


# ---------------------------------------------------------------------------
# Chain rounds (Sec. VI-C, Reading R16): the grade and its penalty terms
# ---------------------------------------------------------------------------

def test_grade_penalises_size_difference(oracle_mod):
    # Move 0: part 0 -> 1, gain 5.  Two moves leave part 1 with equal gain 3:
    # node 1 (size 1) and node 2 (size 4).  Grade from node 0 (size 1):
    #   node 1: 3*10^7 - 10*|1-1| = 3*10^7
    #   node 2: 3*10^7 - 10*|1-4| = 3*10^7 - 30
    # so node 0 links to node 1 (a sign slip would pick node 2, the larger id).
    # Chains: [0, 1] total 8, [2] total 3  ->  sequence 0, 1, 2.
    seq, cl, links, rounds = seq_of(oracle_mod, [(0, 0, 1, 5), (1, 1, 2, 3), (2, 1, 3, 3)], 3,
                                    node_w=[1, 1, 4])
    assert seq == [0, 1, 2] and cl == [2, 1] and links == 1 and rounds == 2


def test_grade_penalises_inbound_difference(oracle_mod):
    # As above with equal sizes; |in| = 0, 2, 0.  Grades from node 0:
    #   node 1: 3*10^7 - |0-2| = 3*10^7 - 2;  node 2: 3*10^7.  -> node 2.
    # Chains: [0, 2] total 8, [1] total 3  ->  0, 2, 1.
    seq, cl, _, _ = seq_of(oracle_mod, [(0, 0, 1, 5), (1, 1, 2, 3), (2, 1, 3, 3)], 3, n_in=[0, 2, 0])
    assert seq == [0, 2, 1] and cl == [2, 1]


def test_grade_weights_size_ten_times_inbound(oracle_mod):
    # Node 1 differs from node 0 by 1 in size (penalty 10), node 2 by 9 in |in|
    # (penalty 9): node 2 scores higher.  Swapping the two weights (size x1,
    # |in| x10) would give penalties 1 and 90 and pick node 1.
    seq, cl, _, _ = seq_of(oracle_mod, [(0, 0, 1, 5), (1, 1, 2, 3), (2, 1, 3, 3)], 3,
                           node_w=[1, 2, 1], n_in=[0, 0, 9])
    assert seq == [0, 2, 1] and cl == [2, 1]


def test_gain_dominates_the_penalty(oracle_mod):
    # Node 1 has gain 4 but a size gap of 100 (penalty 1000); node 2 gain 3 and
    # no gap.  4*10^7 - 1000 > 3*10^7, so node 0 links to node 1.
    # Chains: [0, 1] total 9, [2] total 3.
    seq, cl, _, _ = seq_of(oracle_mod, [(0, 0, 1, 5), (1, 1, 2, 4), (2, 1, 3, 3)], 3,
                           node_w=[1, 101, 1])
    assert seq == [0, 1, 2] and cl == [2, 1]


def test_window_reaches_beyond_the_first_candidate(oracle_mod):
    # Part 1 is left by node 1 (gain 5, size 3) and node 2 (gain 5, size 1), in
    # that sort order (equal gain, id ascending).  From node 0 (size 1) node 2
    # grades higher (no size gap); a window of one move would only see node 1.
    seq, cl, _, _ = seq_of(oracle_mod, [(0, 0, 1, 9), (1, 1, 2, 5), (2, 1, 3, 5)], 3, node_w=[1, 3, 1])
    assert seq == [0, 2, 1] and cl == [2, 1]


def test_window_is_the_first_256_predecessor_less_moves(oracle_mod):
    # Node 0 moves 0 -> 1 (gain 10); nodes 1..257 all move 1 -> 2 with gain 1,
    # unit sizes.  The moves sort puts them in id order (equal p_s and gain,
    # Reading R15), so the window holds nodes 1..256 and every grade is
    # 10^7: the tie goes to the largest id in the window, node 256; node 257
    # is outside it.  Nothing leaves part 2, so no other link forms.
    # Chains: [0, 256] total 11, then 256 single moves of gain 1 by id.
    moves = [(0, 0, 1, 10)] + [(i, 1, 2, 1) for i in range(1, 258)]
    seq, cl, links, rounds = seq_of(oracle_mod, moves, 258)
    assert seq == [0, 256] + list(range(1, 256)) + [257]
    assert cl == [2] + [1] * 256 and links == 1 and rounds == 2


def test_successor_tie_goes_to_larger_node_id(oracle_mod):
    # Two moves leave part 1 with equal gain and no penalty: nodes 1 and 2.
    # The proposer takes the lexicographic max (grade, id): node 2.
    seq, cl, _, _ = seq_of(oracle_mod, [(0, 0, 1, 5), (1, 1, 2, 3), (2, 1, 3, 3)], 3)
    assert seq == [0, 2, 1] and cl == [2, 1]


# ---------------------------------------------------------------------------
# Acceptance (Reading R16): the successor keeps the max (grade, proposer id)
# ---------------------------------------------------------------------------

def test_acceptance_tie_goes_to_larger_proposer(oracle_mod):
    # Nodes 1 (0 -> 2) and 3 (1 -> 2), gain 5 each, both propose node 5
    # (2 -> 4, gain 2) with grade 2*10^7.  Node 5 accepts proposer 3.  In round
    # 2 node 1 finds no predecessor-less move leaving part 2 and stops.
    # Chains: [3, 5] total 7, [1] total 5  ->  3, 5, 1.
    seq, cl, links, rounds = seq_of(oracle_mod, [(1, 0, 2, 5), (3, 1, 2, 5), (5, 2, 4, 2)], 6)
    assert seq == [3, 5, 1] and cl == [2, 1] and links == 1 and rounds == 2


def test_acceptance_prefers_higher_grade_over_id(oracle_mod):
    # As above, but node 3 has size 2: its grade for node 5 (size 1) is
    # 2*10^7 - 10 < 2*10^7, so node 5 accepts node 1.  Chains: [1, 5] total 7,
    # [3] total 5.
    seq, cl, _, _ = seq_of(oracle_mod, [(1, 0, 2, 5), (3, 1, 2, 5), (5, 2, 4, 2)], 6,
                           node_w=[1, 1, 1, 2, 1, 1])
    assert seq == [1, 5, 3] and cl == [2, 1]


def test_rejected_proposer_retries_next_round(oracle_mod):
    # Part 2 is left by node 5 (gain 2) and node 6 (gain 1).  Round 1: nodes 1
    # and 3 both prefer node 5 (grade 2*10^7 vs 10^7); node 5 accepts node 3.
    # Round 2: node 1's window now skips node 5 (it has a predecessor) and it
    # links to node 6.  Round 3 adds nothing (nothing leaves parts 4 or 8).
    # Chains: [3, 5] total 7, [1, 6] total 6.
    moves = [(1, 0, 2, 5), (3, 1, 2, 5), (5, 2, 4, 2), (6, 2, 8, 1)]
    seq, cl, links, rounds = seq_of(oracle_mod, moves, 7)
    assert seq == [3, 5, 1, 6] and cl == [2, 2] and links == 2 and rounds == 3


def test_rounds_limit(oracle_mod):
    # Rounds = 0 is the ablation without chaining: every move is its own chain
    # and the sequence orders moves by (gain desc, id asc).
    moves = [(1, 0, 2, 5), (3, 1, 2, 5), (5, 2, 4, 2), (6, 2, 8, 1)]
    seq, cl, links, rounds = seq_of(oracle_mod, moves, 7, rounds=0)
    assert seq == [1, 3, 5, 6] and cl == [1, 1, 1, 1] and links == 0 and rounds == 0
    # One round: only round 1's link (3 -> 5) forms.
    seq, cl, links, rounds = seq_of(oracle_mod, moves, 7, rounds=1)
    assert seq == [3, 5, 1, 6] and cl == [2, 1, 1] and links == 1 and rounds == 1


# ---------------------------------------------------------------------------
# Chain linearisation and ranking (Reading R17)
# ---------------------------------------------------------------------------

def test_cycles_start_at_smallest_node_and_rank_by_gain_then_first_id(oracle_mod):
    # A 3-cycle 7 (0->1) -> 4 (1->2) -> 9 (2->0), gains 3 each: every move has
    # exactly one candidate successor, so all three links form in round 1.
    # It is linearised from its smallest node: 4, 9, 7 (total 9).
    # Node 2 (3 -> 5, gain 9) is a chain of its own with the same total 9 and
    # a smaller first id, so it comes first.
    # A 2-cycle 10 (6->7), 11 (7->6), gains 1: 10, 11 (total 2), last.
    moves = [(7, 0, 1, 3), (4, 1, 2, 3), (9, 2, 0, 3), (2, 3, 5, 9), (10, 6, 7, 1), (11, 7, 6, 1)]
    seq, cl, links, rounds = seq_of(oracle_mod, moves, 12)
    assert seq == [2, 4, 9, 7, 10, 11] and cl == [1, 3, 2] and links == 5 and rounds == 2


def test_paths_run_head_to_tail(oracle_mod):
    # 8 (0->1, gain 1) -> 2 (1->2, gain 1) -> 5 (2->3, gain 1): one path,
    # head first, all links in round 1.  Node 0 (4 -> 5, gain 2) ranks
    # after it (total 2 < 3).
    moves = [(8, 0, 1, 1), (2, 1, 2, 1), (5, 2, 3, 1), (0, 4, 5, 2)]
    seq, cl, _, _ = seq_of(oracle_mod, moves, 9)
    assert seq == [8, 2, 5, 0] and cl == [3, 1]


# ---------------------------------------------------------------------------
# Isolated pairing (Sec. V-C, Reading R8): the skip step moves the large end
# ---------------------------------------------------------------------------

def _graph(oracle_mod, n, edges, node_w=None, hedge_w=None):
    srcs = [e[0] for e in edges]
    dsts = [e[1] for e in edges]
    hg = W._assemble(n, srcs, dsts, hedge_w=hedge_w, node_w=node_w)
    return oracle_mod.Graph(hg)


def test_isolated_pairing_skips_the_largest_on_size(oracle_mod):
    # Every node isolated.  Sorted (size, id): 0(1) 1(1) 2(3) 3(6); Omega 6.
    # i=0, j=3: 1+6 > 6, so j moves to 2: 1+3 <= 6 pairs {0, 2}; then i=1,
    # j=1 stops.  Moving i instead of j would pair nothing.
    g = _graph(oracle_mod, 4, [], node_w=[1, 1, 3, 6])
    cand = -np.ones((4, 4), np.int32)
    match, rp = g.match(6, 100, cand, np.zeros((4, 4), np.uint64))
    assert match.tolist() == [2, -1, 0, -1] and rp[4] == 1


def test_isolated_pairing_skips_on_inbound(oracle_mod):
    # Unit sizes; |in| = 3, 0, 1, 2 (h-edges into nodes 0, 0, 0, 3, 3, 2).
    # Delta 4: i=0, j=3: 3+2 > 4, j -> 2: 3+1 <= 4 pairs {0, 2}; i=1, j=1 stops.
    edges = [([1], [0]), ([1], [0]), ([1], [0]), ([0], [3]), ([0], [3]), ([0], [2])]
    g = _graph(oracle_mod, 4, edges)
    _, nin, _ = g.incidence()
    assert nin.tolist() == [3, 0, 1, 2]
    cand = -np.ones((4, 4), np.int32)
    match, rp = g.match(10, 4, cand, np.zeros((4, 4), np.uint64))
    assert match.tolist() == [2, -1, 0, -1] and rp[4] == 1


# ---------------------------------------------------------------------------
# Noise cap (Sec. V-C, Reading R3): h-edges with one pin are left out
# ---------------------------------------------------------------------------

def test_noise_cap_ignores_single_pin_hedges(oracle_mod):
    # e0: 1 pin (w 1); e1: 2 pins (w 1), t = 2^16/2 = 32768; e2: 4 pins (w 3),
    # t = 3*2^16/4 = 49152; e3: 1 pin (w 5).  Over the h-edges with >= 2 pins:
    # cap = floor((32768 + 49152) / (10 * 2)) = 4096.  Counting e0 and e3 too
    # would give floor((81920 + 65536 + 327680) / 40) = 11878.
    edges = [([], [0]), ([0], [1]), ([1], [2, 3, 4]), ([], [5])]
    g = _graph(oracle_mod, 6, edges, hedge_w=[1, 1, 3, 5])
    assert [g.tnorm(e) for e in range(4)] == [65536, 32768, 49152, 327680]
    assert g.noise_cap() == 4096


def test_noise_cap_of_only_single_pin_hedges_is_zero(oracle_mod):
    g = _graph(oracle_mod, 3, [([], [0]), ([1], [])])
    assert g.noise_cap() == 0


# ---------------------------------------------------------------------------
# k-way seating (Sec. VII-A, Reading R21): the lightest part first
# ---------------------------------------------------------------------------

def test_kway_seats_into_lightest_part(oracle_mod):
    # Sizes 3, 2, 2, 1; k = 2; loose caps.  Order (size desc, id asc): 0 1 2 3.
    # 0 -> part 0 (both empty: smaller id); 1 -> part 1 (0 < 3); 2 -> part 1
    # (2 < 3); 3 -> part 0 (3 < 4).  Weights end 4 / 4.  Seating into the
    # heaviest part would put every node in part 0.
    g = _graph(oracle_mod, 4, [([0], [1])], node_w=[3, 2, 2, 1])
    assert g.kway_initial(2, 10, 100).tolist() == [0, 1, 1, 0]


def test_kway_seating_order_is_size_then_id(oracle_mod):
    # Sizes 1, 2, 2, 3; order (size desc, id asc): 3 1 2 0.
    # 3 -> part 0; 1 -> part 1; 2 -> part 1 (2 < 3); 0 -> part 0 (3 < 4).
    g = _graph(oracle_mod, 4, [([0], [1])], node_w=[1, 2, 2, 3])
    assert g.kway_initial(2, 10, 100).tolist() == [0, 1, 1, 0]


def test_kway_respects_delta(oracle_mod):
    # Node 0 (size 2) is the source of e0 -> 1 and e1 -> 2; |in| of 1 and 2 is 1.
    # Delta 1.  0 -> part 0; 1 -> part 1 (D 1); 2 -> part 1 is lighter but
    # would reach D = 2, so part 0 (D 1).
    g = _graph(oracle_mod, 3, [([0], [1]), ([0], [2])], node_w=[2, 1, 1])
    assert g.kway_initial(2, 10, 1).tolist() == [0, 1, 0]


# ---------------------------------------------------------------------------
# Early exit of repetitions (Reading R25)
# ---------------------------------------------------------------------------

def _replay_kstar(res, omega, delta, theta):
    """k* of every repetition at every level, replayed without the early
    exit (repetitions are deterministic, so the replay is the driver's)."""
    L = res.nlevels
    rho = np.arange(res.levels[L - 1]["N"], dtype=np.int32)
    out = {}
    for lv in range(L - 1, -1, -1):
        g = res.graph(lv)
        if lv < L - 1:
            rho = rho[res.gamma(lv)]
        ks = []
        for rep in range(theta):
            rho, d = g.refine_rep(rho, res.nparts, rep, theta, omega, delta)
            ks.append(d["kstar"])
        out[lv] = ks
    return out


@pytest.mark.parametrize("theta", [2, 4])
def test_early_exit_still_runs_the_second_half(oracle_mod, theta):
    # On this graph the level-0 repetitions of the first half apply nothing
    # while one of the second half (size-aware, Sec. VI-B) applies a move.
    # The early exit may skip only the rest of the half it is in, so the run
    # with it must equal the run of all theta repetitions at every level.
    hg = W.random_small(14, 16, 4, 1, max_src=1, max_hw=3, max_nw=3)
    omega, delta = 7, 10 ** 6
    g = oracle_mod.Graph(hg)
    full = g.partition(omega, delta, theta=theta, early_exit=False)
    ks = _replay_kstar(full, omega, delta, theta)
    h = theta // 2
    assert all(k == 0 for k in ks[0][:h]) and any(k > 0 for k in ks[0][h:])
    fast = g.partition(omega, delta, theta=theta, early_exit=True)
    assert fast.nlevels == full.nlevels
    for lv in range(full.nlevels):
        assert np.array_equal(fast.rho(lv), full.rho(lv))
    assert fast.levels[0]["moves_applied"] == full.levels[0]["moves_applied"] > 0
