"""Independent computation routes used to pin the oracle.

Nothing here calls into the oracle.  Quantities are computed through a
different route than the oracle's loops: incidence-matrix products for the
pin counts, histogram and intersections, and exhaustive enumeration for
optima.  A mistake in the oracle (a dropped term, a wrong sign or index, a
swapped source/destination) shows up as a disagreement with these.
"""
from __future__ import annotations

import itertools

import numpy as np


def incidence_matrices(hg):
    """H[e, n] = 1 if n in e; Hd[e, n] = 1 if n in dst(e) (dense, int64)."""
    E, N = hg.n_hedges, hg.n_nodes
    H = np.zeros((E, N), np.int64)
    Hd = np.zeros((E, N), np.int64)
    for e in range(E):
        s, d = hg.edge(e)
        H[e, s] = 1
        H[e, d] = 1
        Hd[e, d] = 1
    return H, Hd


def eval_by_products(hg, rho, nparts):
    """Phi = H X, Phi_in = Hd X for the one-hot assignment X (N x |P|)."""
    H, Hd = incidence_matrices(hg)
    X = np.zeros((hg.n_nodes, nparts), np.int64)
    X[np.arange(hg.n_nodes), rho] = 1
    Phi = H @ X
    Phi_in = Hd @ X
    lam = (Phi > 0).sum(axis=1)
    w = hg.hedge_w.astype(np.int64)
    conn = int((w * (lam - 1)).sum())
    cutnet = int((w * (lam > 1)).sum())
    size = X.T @ hg.node_w.astype(np.int64)
    D = (Phi_in > 0).sum(axis=0)
    return dict(Phi=Phi, Phi_in=Phi_in, conn=conn, cutnet=cutnet, size=size, D=D)


def all_rgs(n: int) -> np.ndarray:
    """Every set partition of n elements as a restricted growth string
    (rows), Bell(n) rows."""
    cur = np.zeros((1, 1), np.int8)
    mx = np.zeros(1, np.int8)
    for _ in range(1, n):
        reps = (mx + 2).astype(np.int64)
        idx = np.repeat(np.arange(cur.shape[0]), reps)
        base = np.concatenate([[0], np.cumsum(reps)[:-1]])
        lab = (np.arange(idx.shape[0]) - np.repeat(base, reps)).astype(np.int8)
        cur = np.concatenate([cur[idx], lab[:, None]], axis=1)
        mx = np.maximum(mx[idx], lab)
    return cur


def brute_force_all(hg, omega, delta):
    """Conn, validity of every partition of a tiny hypergraph (vectorised
    over all Bell(N) restricted growth strings)."""
    R = all_rgs(hg.n_nodes).astype(np.int64)
    B = R.shape[0]
    conn = np.zeros(B, np.int64)
    D = np.zeros((B, hg.n_nodes), np.int64)
    for e in range(hg.n_hedges):
        s, d = hg.edge(e)
        members = np.concatenate([s, d])
        lab = np.sort(R[:, members], axis=1)
        lam = 1 + (lab[:, 1:] != lab[:, :-1]).sum(axis=1)
        conn += int(hg.hedge_w[e]) * (lam - 1)
        if len(d):
            hit = np.zeros((B, hg.n_nodes), bool)
            for m in d:
                hit[np.arange(B), R[:, m]] = True
            D += hit
    size = np.zeros((B, hg.n_nodes), np.int64)
    for n in range(hg.n_nodes):
        size[np.arange(B), R[:, n]] += int(hg.node_w[n])
    valid = (size <= omega).all(axis=1) & (D <= delta).all(axis=1)
    return R, conn, valid


def max_weight_matching_brute(edges):
    """edges: list of (a, b, w).  Exhaustive maximum total weight over all
    sets of pairwise disjoint edges."""
    best = 0
    m = len(edges)

    def rec(i, used, tot):
        nonlocal best
        if i == m:
            best = max(best, tot)
            return
        rec(i + 1, used, tot)
        a, b, w = edges[i]
        if a not in used and b not in used:
            rec(i + 1, used | {a, b}, tot + w)

    rec(0, frozenset(), 0)
    return best
