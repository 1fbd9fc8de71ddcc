"""Seeded inputs of the single-repetition refinement checks: a hypergraph, a
partition and the caps.  Input generation only; no step of the method.

Each case is chosen so that one in-isolation gains kernel of the library
serves it (the partition count and the mean incidence degree decide which),
or, for the full-size cases, so that refinement commits moves at a size the
library meets in real runs.
"""
import numpy as np

from paper_2605_20497_amd import workloads as W


def _weighted(hg, seed, max_hw=3, max_nw=2):
    rng = np.random.default_rng(1000 + seed)
    hg.hedge_w = rng.integers(1, max_hw + 1, size=hg.n_hedges).astype(np.int32)
    hg.node_w = rng.integers(1, max_nw + 1, size=hg.n_nodes).astype(np.int32)
    return hg


def many_sources_hypergraph(n, e, fanout, seed):
    """e h-edges over n nodes: a uniform source and `fanout` distinct uniform
    destinations other than it (so nodes sit in e*(fanout+1)/n h-edges)."""
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, size=e, dtype=np.int64)
    dst = W.sample_distinct(rng, e, fanout, n, exclude=src)
    return W._assemble_uniform(n, src, dst)


def random_partition(n, nparts, seed):
    return np.random.default_rng(seed).integers(0, nparts, size=n).astype(np.int32)


def loose_caps(hg, rho, nparts):
    """Omega two above the largest part's weight."""
    size = np.bincount(rho, weights=hg.node_w, minlength=nparts).astype(np.int64)
    return int(size.max()) + 2


# name -> (hypergraph builder, partitions, partition seed, weighted)
GAINS_VARIANTS = {
    # few partitions, mean degree above 256: the block-per-node 16-bit sweep
    "p3000-deg300": (lambda: many_sources_hypergraph(2000, 2000, 300, 11), 3000, 1, True),
    # more than 4,096 partitions: the block-per-node 16-bit sweep, one pass
    "p6000-deg30": (lambda: W.random_snn(8000, 29, seed=12), 6000, 2, True),
    # more than 16,384 partitions: the 16-bit sweep over id ranges
    "p20000-deg21": (lambda: W.random_snn(30000, 20, seed=13), 20000, 3, True),
    # more than 32,767 partitions: the 32-bit rows
    "p40000-deg17": (lambda: W.random_snn(50000, 16, seed=14), 40000, 4, True),
    # at most 4,096 partitions and mean degree at most 256: one wave per node
    "p2872-deg192": (lambda: W.random_snn(12000, 191, seed=15), 2872, 5, True),
}


def mixed_size_hypergraph(n, e, seed):
    """e h-edges over n nodes with sizes cycling through 2-8, 9-64, 65-256
    and 257-400 pins in a seeded random order, so that each size class of the
    in-sequence kernels meets windows of 64 h-edges where it holds only a few
    (and lane groups that stay idle in a window's last round).  One or two
    sources per h-edge."""
    rng = np.random.default_rng(seed)
    bounds = [(2, 8), (9, 64), (65, 256), (257, 400)]
    weights = np.array([0.55, 0.3, 0.12, 0.03])
    cls = rng.choice(4, size=e, p=weights)
    srcs, dsts = [], []
    for c in cls:
        lo, hi = bounds[c]
        card = int(rng.integers(lo, hi + 1))
        ids = rng.choice(n, size=card, replace=False)
        ns = 1 + int(rng.integers(0, 2))
        srcs.append(ids[:ns])
        dsts.append(ids[ns:])
    return W._assemble(n, srcs, dsts)


def mixed_size_case(seed):
    hg = _weighted(mixed_size_hypergraph(3000, 6000, 40 + seed), seed)
    rho = random_partition(hg.n_nodes, 64, seed)
    return hg, rho, 64


def gains_variant(name):
    build, nparts, pseed, weighted = GAINS_VARIANTS[name]
    hg = build()
    if weighted:
        hg = _weighted(hg, pseed)
    rho = random_partition(hg.n_nodes, nparts, pseed)
    return hg, rho, nparts


# Full-size single repetitions stored as oracle digests
# (tests/golden/refine_rep.json, written by tests/golden/make_refine_golden.py).
FULL = {
    # the 65,536-node random SNN workload with a random partition over 2,872
    # parts and a Delta loose enough that refinement commits
    "rand-64k-e192-rho2872": dict(hg=lambda: W.rand_64k_e192(), nparts=2872, seed=7, delta=1 << 20),
    # 8,192 nodes in 65,536 h-edges of 64 pins: every node meets ~512 h-edges
    # and the in-isolation moves fit the dense product
    "dense-8k-e65k-rho1024": dict(hg=lambda: many_sources_hypergraph(8192, 65536, 63, 21), nparts=1024, seed=8,
                                  delta=1 << 20),
}


def full_case(name):
    """(hypergraph, partition, partitions, delta, [(rep, omega), ...]): a
    first-half repetition with Omega two above the largest part and a
    size-aware one with Omega equal to it, so that full parts take no move."""
    d = FULL[name]
    hg = d["hg"]()
    rho = random_partition(hg.n_nodes, d["nparts"], d["seed"])
    big = loose_caps(hg, rho, d["nparts"]) - 2
    return hg, rho, d["nparts"], d["delta"], [(0, big + 2), (9, big)]
