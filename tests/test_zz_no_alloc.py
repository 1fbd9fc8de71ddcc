"""hgp_evaluate_noalloc (the evaluation that allocates no device memory)
against hgp_evaluate and the oracle, through the C ABI.

Everything compared is an integer (Eq. connectivity, Eq. cut-net, the largest
partition size and D(p) of Sec. II-B, the violation count and the non-empty
partitions), so the bar is equality.  Two calls in a row on one context, the
second on a smaller hypergraph with fewer partitions, show that what the static
workspace keeps from the previous call does not leak into the next; a third
context on the same device shares that workspace."""
import numpy as np
import pytest

import oracle
from paper_2605_20497_amd import workloads as W
from tests import _refine_cases as RC

pytestmark = pytest.mark.gpu


def _case(n, fanout, nparts, seed):
    hg = RC._weighted(W.random_snn(n, fanout, seed=seed), seed)
    rho = RC.random_partition(n, nparts, seed)
    return hg, rho


def _check(part, hg, rho, nparts, omega, delta):
    import torch
    part.hgp_set_limits(omega, delta, 0)
    ref = part.hgp_evaluate(rho, nparts)
    dev = torch.from_numpy(rho).to("cuda")
    got = part.hgp_evaluate_noalloc(dev, nparts)
    assert got == ref
    ev = oracle.Graph(hg).evaluate(rho, nparts, omega, delta)
    for key in ("conn", "cutnet", "max_size", "max_inbound", "violations"):
        assert got[key] == ev[key], key
    assert got["n_parts"] == ev["nonempty"]
    return got


def test_noalloc_matches_evaluate_twice_then_smaller():
    from paper_2605_20497_amd import Partitioner
    big, rho_big = _case(20000, 63, 700, 31)
    small, rho_small = _case(3000, 15, 50, 32)
    print("case noalloc big N", big.n_nodes, "P", big.n_pins, "then small N", small.n_nodes, "P", small.n_pins,
          flush=True)
    g = Partitioner()
    g.load(big)
    a = _check(g, big, rho_big, 700, 40, 1500)
    # tight caps: violations counted, then loose caps on the same rows
    b = _check(g, big, rho_big, 700, 20, 900)
    assert b["violations"] > 0 and a["conn"] == b["conn"]
    g.load(small)
    _check(g, small, rho_small, 50, 80, 600)
    g.close()
    # a second context on the device reuses the same workspace
    h = Partitioner()
    h.load(small)
    _check(h, small, rho_small[::-1].copy(), 50, 80, 600)
    h.close()


def test_noalloc_errors_leave_context_usable():
    import torch
    from paper_2605_20497_amd import HGP_E_INVALID, HGP_E_UNSUPPORTED, HgpError, Partitioner
    small, rho = _case(3000, 15, 50, 33)
    print("case noalloc errors", flush=True)
    g = Partitioner()
    g.load(small)
    g.hgp_set_limits(80, 600, 0)
    bad = rho.copy()
    bad[1234] = 50
    with pytest.raises(HgpError) as ei:
        g.hgp_evaluate_noalloc(torch.from_numpy(bad).to("cuda"), 50)
    assert ei.value.status == HGP_E_INVALID
    _check(g, small, rho, 50, 80, 600)
    # 5.9 M pins: the rows alone need 71 MB, beyond the 64 MiB workspace
    large = W.random_snn(31000, 189, seed=34)
    g.load(large)
    g.hgp_set_limits(1 << 20, 1 << 20, 0)
    rl = RC.random_partition(large.n_nodes, 100, 35)
    with pytest.raises(HgpError) as ei:
        g.hgp_evaluate_noalloc(torch.from_numpy(rl).to("cuda"), 100)
    assert ei.value.status == HGP_E_UNSUPPORTED
    g.load(small)
    _check(g, small, rho, 50, 80, 600)
    g.close()
