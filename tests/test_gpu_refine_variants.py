"""Single refinement repetitions (Sec. VI) of the HIP path against the
oracle, on inputs that route the in-isolation gains through each of the
library's gains kernels, and at full size against stored oracle digests.

Compared bit for bit: every node's in-isolation move and gain (Eq.
refinement_move_selection), the sequence and its destinations (Sec. VI-C),
the in-sequence gains, C_k and V_k after every prefix (Sec. VI-D), the counts
and the partition after the applied prefix."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from tests import _refine_cases as RC

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


@pytest.mark.parametrize("rep", [0, 9])
@pytest.mark.parametrize("name", sorted(RC.GAINS_VARIANTS))
def test_gains_kernel_variants(name, rep):
    from paper_2605_20497_amd import Partitioner
    hg, rho, P = RC.gains_variant(name)
    og = oracle.Graph(hg)
    ev = og.evaluate(rho, P)
    # first half: Omega two above the largest part; size-aware half: Omega at
    # the largest part, so moves into full parts are excluded
    omega = int(ev["max_size"]) + (2 if rep == 0 else 0)
    delta = int(ev["max_inbound"]) + 1
    print("case", name, "rep", rep, "N", hg.n_nodes, "P", hg.n_pins, "parts", P, "omega", omega, "delta", delta,
          flush=True)
    g = Partitioner(dense_gains=False)
    g.load(hg)
    g.hgp_set_limits(omega, delta, 0)
    cur = rho
    for it in range(2):
        odst, ogain = og.moves(cur, P, rep, 16, omega)
        orho, od = og.refine_rep(cur, P, rep, 16, omega, delta)
        grho, gd = g.hgp_refine_rep(cur, P, rep)
        assert np.array_equal(gd["move_dst"], odst), ("move_dst", it)
        assert np.array_equal(gd["move_gain"], ogain), ("move_gain", it)
        assert (gd["moves"], gd["kstar"], gd["gain"], gd["links"]) == (od["M"], od["kstar"], od["applied_gain"],
                                                                        od["links"]), it
        for key in ("seq", "seq_pd", "gseq", "C", "V"):
            assert np.array_equal(gd[key], od[key]), (key, it)
        assert np.array_equal(grho, orho), it
        cur = orho
    assert od["M"] > 0
    g.close()


@pytest.mark.parametrize("seed", [0, 1])
def test_inseq_size_classes_against_oracle(seed):
    """H-edges of every in-sequence size class (one lane each up to 8 pins,
    16-lane groups up to 64, whole waves up to 256, all pairs beyond) mixed in
    one input, so that windows hold a few h-edges of a class and lane groups
    stay idle: the repetition matches the oracle, and two runs of it on the
    device match each other."""
    from paper_2605_20497_amd import Partitioner
    hg, rho, P = RC.mixed_size_case(seed)
    og = oracle.Graph(hg)
    ev = og.evaluate(rho, P)
    omega = int(ev["max_size"]) + 2
    delta = int(ev["max_inbound"]) + 1
    print("case mixed seed", seed, "N", hg.n_nodes, "P", hg.n_pins, "omega", omega, "delta", delta, flush=True)
    g = Partitioner()
    g.load(hg)
    g.hgp_set_limits(omega, delta, 0)
    orho, od = og.refine_rep(rho, P, 0, 16, omega, delta)
    runs = [g.hgp_refine_rep(rho, P, 0) for _ in range(2)]
    for grho, gd in runs:
        assert gd["moves"] == od["M"] and gd["kstar"] == od["kstar"]
        for key in ("seq", "seq_pd", "gseq", "C", "V"):
            assert np.array_equal(gd[key], od[key]), key
        assert np.array_equal(grho, orho)
    assert od["M"] > 100
    g.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name", sorted(RC.FULL))
def test_full_size_refine_rep_against_oracle_digests(name):
    from paper_2605_20497_amd import Partitioner
    gold = json.load(open(os.path.join(HERE, "golden", "refine_rep.json")))[name]
    hg, rho, P, delta, reps = RC.full_case(name)
    print("case", name, "N", hg.n_nodes, "P", hg.n_pins, "parts", P, flush=True)
    assert (hg.n_nodes, hg.n_pins, P, delta) == (gold["nodes"], gold["pins"], gold["nparts"], gold["delta"])
    # the 8k-node case forces the dense (MFMA) in-isolation moves; the
    # 65,536-node case is beyond them and takes the sparse sweep
    g = Partitioner(dense_gains=True if name.startswith("dense") else None)
    g.load(hg)
    for (rep, omega), run in zip(reps, gold["runs"]):
        assert (rep, omega) == (run["rep"], run["omega"])
        g.hgp_set_limits(omega, delta, 0)
        grho, gd = g.hgp_refine_rep(rho, P, rep)
        assert (gd["moves"], gd["kstar"], gd["gain"], gd["links"]) == (run["moves"], run["kstar"], run["gain"],
                                                                        run["links"]), rep
        assert run["kstar"] > 0
        assert _digest(gd["move_dst"].astype(np.int32)) == run["move_dst"], rep
        assert _digest(gd["move_gain"].astype(np.int64)) == run["move_gain"], rep
        for key in ("seq", "seq_pd"):
            assert _digest(gd[key].astype(np.int32)) == run[key], (key, rep)
        for key in ("gseq", "C", "V"):
            assert _digest(gd[key].astype(np.int64)) == run[key], (key, rep)
        assert _digest(grho.astype(np.int32)) == run["rho"], rep
    g.close()
