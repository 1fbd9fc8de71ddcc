"""Seeded synthetic hypergraph generators.

This module only draws random structure; it holds none of the partitioning
method's arithmetic.  Both the serial checker and the HIP library consume the
arrays it returns, so input parity between the two never has to be argued.

Every generator returns a :class:`Hypergraph` in the dual-CSR input layout of
the paper's data-structure section (Sec. IV-B): h-edge offsets (int64), the
number of source pins per h-edge, and the pin array with each h-edge's sources
first and destinations after, each block sorted ascending.  Ids are zero-based
int32.  Weights are int32.

The shapes stand in for the paper's benchmark suites (Table I: spiking neural
network hypergraphs; Table II: ISPD98 netlists augmented 16x), which are not
available here.  Only their sizes, cardinalities and constraint pairs are used;
no item of either suite is reproduced.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Hypergraph:
    n_nodes: int
    he_off: np.ndarray   # int64 [E+1]
    he_nsrc: np.ndarray  # int32 [E]
    pins: np.ndarray     # int32 [P], per h-edge: sources (sorted) then destinations (sorted)
    hedge_w: np.ndarray  # int32 [E]
    node_w: np.ndarray   # int32 [N]
    omega: int = 0       # partition size cap (node-weight sum)
    delta: int = 0       # cap on distinct inbound h-edges per partition
    k: int = 0           # 0 = constrained method; >0 = k-way balanced mode
    name: str = ""

    @property
    def n_hedges(self) -> int:
        return int(self.he_nsrc.shape[0])

    @property
    def n_pins(self) -> int:
        return int(self.pins.shape[0])

    def edge(self, e: int):
        a, b = int(self.he_off[e]), int(self.he_off[e + 1])
        s = int(self.he_nsrc[e])
        return self.pins[a:a + s], self.pins[a + s:b]


def _assemble(n_nodes, srcs, dsts, hedge_w=None, node_w=None, **kw) -> Hypergraph:
    """srcs/dsts: lists (or 2-D arrays) of per-h-edge id arrays."""
    E = len(srcs)
    sizes = np.fromiter((len(s) + len(d) for s, d in zip(srcs, dsts)), dtype=np.int64, count=E)
    he_off = np.zeros(E + 1, dtype=np.int64)
    np.cumsum(sizes, out=he_off[1:])
    he_nsrc = np.fromiter((len(s) for s in srcs), dtype=np.int32, count=E)
    parts = []
    for s, d in zip(srcs, dsts):
        parts.append(np.sort(np.asarray(s, dtype=np.int32)))
        parts.append(np.sort(np.asarray(d, dtype=np.int32)))
    pins = np.concatenate(parts).astype(np.int32) if parts else np.zeros(0, np.int32)
    if hedge_w is None:
        hedge_w = np.ones(E, dtype=np.int32)
    if node_w is None:
        node_w = np.ones(n_nodes, dtype=np.int32)
    return Hypergraph(n_nodes, he_off, he_nsrc, pins,
                      np.asarray(hedge_w, np.int32), np.asarray(node_w, np.int32), **kw)


def _assemble_uniform(n_nodes, src: np.ndarray, dst: np.ndarray, **kw) -> Hypergraph:
    """Fast path: every h-edge has one source (src[E]) and dst.shape[1] destinations."""
    E, k = dst.shape
    dst = np.sort(dst, axis=1)
    pins = np.empty((E, k + 1), dtype=np.int32)
    pins[:, 0] = src
    pins[:, 1:] = dst
    he_off = np.arange(E + 1, dtype=np.int64) * (k + 1)
    he_nsrc = np.ones(E, dtype=np.int32)
    return Hypergraph(n_nodes, he_off, he_nsrc, pins.reshape(-1),
                      np.ones(E, np.int32), np.ones(n_nodes, np.int32), **kw)


def sample_distinct(rng: np.random.Generator, rows: int, k: int, M: int,
                    exclude: np.ndarray | None = None) -> np.ndarray:
    """rows x k array; row r holds k distinct values drawn uniformly from
    [0, M) minus {exclude[r]} (when given).  Draw order is kept, so taking the
    first k distinct values of an i.i.d. stream gives a uniform k-subset."""
    Meff = M - (1 if exclude is not None else 0)
    if k > Meff:
        raise ValueError("cannot draw %d distinct values from %d" % (k, Meff))
    out = np.empty((rows, k), dtype=np.int64)
    if k == 0 or rows == 0:
        return out
    if 4 * k > Meff:  # dense draw: per-row permutation prefix
        for r in range(rows):
            v = rng.permutation(Meff)[:k]
            if exclude is not None:
                v = v + (v >= exclude[r])
            out[r] = v
        return out
    todo = np.arange(rows)
    extra = max(8, int(3 * k * k / Meff) + 8)
    while todo.size:
        draws = rng.integers(0, Meff, size=(todo.size, k + extra), dtype=np.int64)
        if exclude is not None:
            draws += draws >= np.asarray(exclude, np.int64)[todo, None]
        order = np.argsort(draws, axis=1, kind="stable")
        sd = np.take_along_axis(draws, order, 1)
        dup = np.zeros(sd.shape, dtype=bool)
        dup[:, 1:] = sd[:, 1:] == sd[:, :-1]
        first = np.empty_like(dup)
        np.put_along_axis(first, order, ~dup, 1)
        cnt = np.cumsum(first, axis=1)
        ok = cnt[:, -1] >= k
        sel = first & (cnt <= k)
        okr = np.nonzero(ok)[0]
        if okr.size:
            out[todo[okr]] = draws[okr][sel[okr]].reshape(-1, k)
        todo = todo[~ok]
        extra *= 2
    return out


# ---------------------------------------------------------------------------
# Random SNN-shaped hypergraphs (Table I "-rand" shapes)
# ---------------------------------------------------------------------------

def random_snn(n: int, fanout: int, seed: int = 0, omega: int = 0, delta: int = 0,
               name: str = "") -> Hypergraph:
    """One h-edge per node: source i plus `fanout` distinct uniform destinations."""
    rng = np.random.default_rng(seed)
    src = np.arange(n, dtype=np.int64)
    dst = sample_distinct(rng, n, fanout, n, exclude=src)
    return _assemble_uniform(n, src, dst, omega=omega, delta=delta, name=name)


def rand_4k_e32(seed: int = 0) -> Hypergraph:
    """4,096 nodes, 4,096 h-edges of size 32 (131,072 pins), Omega=256, Delta=1,024."""
    return random_snn(4096, 31, seed, omega=256, delta=1024, name="rand-4k-e32")


def rand_64k_e192(seed: int = 0) -> Hypergraph:
    """65,536 nodes, 65,536 h-edges of size 192 (12,582,912 pins), Omega=2^10, Delta=2^12."""
    return random_snn(65536, 191, seed, omega=1 << 10, delta=1 << 12, name="rand-64k-e192")


# ---------------------------------------------------------------------------
# Layered feed-forward SNN (Table I "-model" shapes)
# ---------------------------------------------------------------------------

def layered_snn(layers: int, width: int, fanout: int, window: int, local_frac: float,
                seed: int = 0, omega: int = 0, delta: int = 0, name: str = "") -> Hypergraph:
    """Node (l, j) drives `fanout` distinct destinations in layer (l+1) mod layers:
    round(local_frac*fanout) inside the window of `window` positions centred on j
    (wrapping), the rest uniform over the remaining positions of that layer."""
    rng = np.random.default_rng(seed)
    n = layers * width
    n_loc = int(round(local_frac * fanout))
    n_far = fanout - n_loc
    window = min(window, width)
    half = window // 2
    j = np.tile(np.arange(width, dtype=np.int64), layers)
    lay = np.repeat(np.arange(layers, dtype=np.int64), width)
    loc = sample_distinct(rng, n, n_loc, window)            # offsets in [0, window)
    pos_loc = (j[:, None] - half + loc) % width
    far = sample_distinct(rng, n, n_far, width - window)    # positions outside the window
    pos_far = (j[:, None] - half + window + far) % width
    nxt = ((lay + 1) % layers)[:, None] * width
    dst = np.concatenate([pos_loc, pos_far], axis=1) + nxt
    return _assemble_uniform(n, np.arange(n, dtype=np.int64), dst,
                             omega=omega, delta=delta, name=name)


def layered_256k_e256(seed: int = 0) -> Hypergraph:
    """8 layers x 32,768 nodes, |e|=256 (204 local in a 2,048 window + 51 uniform): 67M pins."""
    return layered_snn(8, 32768, 255, 2048, 0.8, seed, omega=1 << 12, delta=1 << 16,
                       name="layered-256k-e256")


# ---------------------------------------------------------------------------
# Conv-like SNN (Table I mobilenet shape)
# ---------------------------------------------------------------------------

def conv_snn(layers: int, hw: int, channels: int, mean_fanout: float, seed: int = 0,
             omega: int = 0, delta: int = 0, name: str = "", progress=None, threads: int = 0) -> Hypergraph:
    """Node (l, y, x, c) drives clamp(Poisson(mean), 1, |W|) distinct destinations in
    layer (l+1) mod layers at |y'-y|<=1, |x'-x|<=1, any channel (|W| <= 9*channels).
    `progress(done, total)` is called after each block of rows when given.

    The random draws are taken in one fixed order on the calling thread (the
    fan-outs, then one block of uniform keys per block of rows); turning a
    block's keys into destination ids runs on `threads` worker threads (0 =
    up to 16 by the host's CPUs), which changes nothing in the output."""
    import concurrent.futures as cf
    import os

    rng = np.random.default_rng(seed)
    per_layer = hw * hw * channels
    n = layers * per_layer
    ids_all = np.arange(n, dtype=np.int64)
    l = ids_all // per_layer
    rem = ids_all % per_layer
    y = rem // (hw * channels)
    x = (rem // channels) % hw
    y0 = np.maximum(y - 1, 0)
    x0 = np.maximum(x - 1, 0)
    wy = np.minimum(y + 1, hw - 1) - y0 + 1
    wx = np.minimum(x + 1, hw - 1) - x0 + 1
    wsize = wy * wx * channels
    k = np.clip(rng.poisson(mean_fanout, size=n), 1, wsize).astype(np.int64)
    base = ((l + 1) % layers) * per_layer
    he_off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(k + 1, out=he_off[1:])
    pins = np.empty(int(he_off[-1]), dtype=np.int32)
    chunk = 1 << 15

    def rows_to_pins(c0, c1, keys):
        rows = c1 - c0
        ws = wsize[c0:c1]
        wmax = keys.shape[1]
        keys[np.arange(wmax)[None, :] >= ws[:, None]] = 2.0
        kk = k[c0:c1]
        kmax = int(kk.max())
        sel = np.argsort(keys, axis=1, kind="stable")[:, :kmax]
        valid = np.arange(kmax)[None, :] < kk[:, None]
        cc = sel % channels
        t = sel // channels
        wxx = wx[c0:c1, None]
        yy = y0[c0:c1, None] + t // wxx
        xx = x0[c0:c1, None] + t % wxx
        ids = base[c0:c1, None] + (yy * hw + xx) * channels + cc
        ids = np.where(valid, ids, np.int64(1) << 40)
        ids.sort(axis=1)
        row_pins = np.empty((rows, kmax + 1), dtype=np.int64)
        row_pins[:, 0] = ids_all[c0:c1]
        row_pins[:, 1:] = ids
        m = np.concatenate([np.ones((rows, 1), bool), valid], axis=1)
        pins[he_off[c0]:he_off[c1]] = row_pins[m].astype(np.int32)

    if threads <= 0:
        threads = max(1, min(16, os.cpu_count() or 1))
    pending = []
    with cf.ThreadPoolExecutor(threads) as ex:
        for c0 in range(0, n, chunk):
            c1 = min(n, c0 + chunk)
            keys = rng.random((c1 - c0, int(wsize[c0:c1].max())))
            pending.append(ex.submit(rows_to_pins, c0, c1, keys))
            if len(pending) >= 2 * threads:  # bounds the keys held at once
                pending.pop(0).result()
            if progress is not None and (c1 == n or (c1 // chunk) % 32 == 0):
                progress(c1, n)
        for f in pending:
            f.result()
    return Hypergraph(n, he_off, np.ones(n, np.int32), pins, np.ones(n, np.int32),
                      np.ones(n, np.int32), omega=omega, delta=delta, name=name)


def conv_6_9m(seed: int = 0, progress=None) -> Hypergraph:
    """7 layers of 176x176x32 (6,938,624 nodes), Poisson(82) fanout: ~577M pins."""
    return conv_snn(7, 176, 32, 82.0, seed, omega=1 << 12, delta=1 << 16, name="conv-6.9m", progress=progress)


# ---------------------------------------------------------------------------
# Circuit-netlist shape (Table II, ISPD98 x16)
# ---------------------------------------------------------------------------

def netlist(n: int, n_nets: int, smin: int, smax: int, alpha: float, local: int,
            local_frac: float, wmax: int, seed: int = 0, k: int = 64,
            eps_pct: int = 3, delta: int = 1 << 15, name: str = "") -> Hypergraph:
    """Nets with power-law sizes P(s) ~ s^-alpha on [smin, smax]; pin 0 is a uniform
    driver (the source), the other s-1 pins are distinct sinks, each local (within
    +-local ids of the driver, wrapping) with probability local_frac, else uniform.
    Node weights uniform in [1, wmax].  Omega = floor((100+eps)*ceil(W/k)/100)."""
    rng = np.random.default_rng(seed)
    s_vals = np.arange(smin, smax + 1, dtype=np.float64)
    p = s_vals ** (-alpha)
    p /= p.sum()
    sizes = rng.choice(np.arange(smin, smax + 1), size=n_nets, p=p).astype(np.int64)
    sizes = np.minimum(sizes, n)
    driver = rng.integers(0, n, size=n_nets, dtype=np.int64)
    srcs, dsts = [], []
    nsink = sizes - 1
    tot = int(nsink.sum())
    # oversample sink draws, keep first distinct non-driver values per net
    net_of = np.repeat(np.arange(n_nets, dtype=np.int64), nsink)
    need = nsink.copy()
    sinks = [[] for _ in range(n_nets)]
    pending = np.arange(n_nets)[need > 0]
    rounds = 0
    chosen = {}
    while pending.size:
        reps = need[pending] + 2 + rounds
        ids = np.repeat(pending, reps)
        m = ids.size
        is_loc = rng.random(m) < local_frac
        off = rng.integers(-local, local + 1, size=m)
        uni = rng.integers(0, n, size=m)
        v = np.where(is_loc, (driver[ids] + off) % n, uni)
        start = 0
        nxt = []
        for idx, net in enumerate(pending):
            r = int(reps[idx])
            cand = v[start:start + r]
            start += r
            lst = sinks[net]
            seen = chosen.setdefault(net, {int(driver[net])})
            for c in cand:
                c = int(c)
                if len(lst) >= nsink[net]:
                    break
                if c not in seen:
                    seen.add(c)
                    lst.append(c)
            if len(lst) < nsink[net]:
                need[net] = nsink[net] - len(lst)
                nxt.append(net)
        pending = np.asarray(nxt, dtype=np.int64)
        rounds += 1
    srcs = [np.asarray([driver[e]], np.int32) for e in range(n_nets)]
    dsts = [np.asarray(sinks[e], np.int32) for e in range(n_nets)]
    node_w = rng.integers(1, wmax + 1, size=n).astype(np.int32)
    W = int(node_w.sum())
    omega = ((100 + eps_pct) * ((W + k - 1) // k)) // 100
    return _assemble(n, srcs, dsts, node_w=node_w, omega=omega, delta=delta, k=k, name=name)


def netlist_500k(seed: int = 0) -> Hypergraph:
    """500k cells, 550k nets, sizes ~ s^-2.827 on [2, 2000], weights in [1, 8], k=64, eps=3%."""
    return netlist(500_000, 550_000, 2, 2000, 2.827, 2048, 0.9, 8, seed, k=64,
                   name="netlist-500k")


# ---------------------------------------------------------------------------
# Small random hypergraphs for tests
# ---------------------------------------------------------------------------

def random_small(n: int, e: int, max_card: int, seed: int, max_src: int = 1,
                 max_hw: int = 1, max_nw: int = 1, omega: int = 0, delta: int = 0,
                 min_card: int = 1) -> Hypergraph:
    """Arbitrary small directed hypergraph: |e| uniform in [min_card, max_card],
    0..max_src sources (never more than |e|), random integer weights."""
    rng = np.random.default_rng(seed)
    srcs, dsts = [], []
    for _ in range(e):
        c = int(rng.integers(min_card, min(max_card, n) + 1))
        members = rng.permutation(n)[:c]
        s = int(rng.integers(0, min(max_src, c) + 1))
        srcs.append(members[:s])
        dsts.append(members[s:])
    hw = rng.integers(1, max_hw + 1, size=e)
    nw = rng.integers(1, max_nw + 1, size=n)
    return _assemble(n, srcs, dsts, hedge_w=hw, node_w=nw, omega=omega, delta=delta,
                     name="small-%d" % seed)


# ---------------------------------------------------------------------------
# Job stream for batched and served runs
# ---------------------------------------------------------------------------

def job_specs(n_jobs: int = 256, min_nodes: int = 2048, max_nodes: int = 262144, seed: int = 0):
    """(sizes, kinds) of the job stream: log-uniform node counts in
    [min_nodes, max_nodes] and a family index 0..4 per job."""
    rng = np.random.default_rng(seed)
    sizes = np.floor(np.exp(rng.uniform(np.log(min_nodes), np.log(max_nodes), size=n_jobs))).astype(np.int64)
    kinds = rng.integers(0, 5, size=n_jobs)
    return sizes, kinds


def make_job(i: int, sizes, kinds, seed: int = 0) -> Hypergraph:
    """Job i of a stream: family kinds[i] (|e| = 32 and 192 random SNN,
    layered, conv, netlist) on sizes[i] nodes, seeded with seed + i.
    Omega_i = min(family Omega, 2^floor(log2(N_i / 16))), Delta_i = 4 Omega_i
    (random) or 16 Omega_i (layered, conv); netlist jobs are k-way with
    k_i = 2^clamp(round(log2(N_i / 8000)), 1, 6)."""
    n = int(sizes[i])
    kind = int(kinds[i])
    s = seed + i
    pow_om = 1 << max(1, int(np.floor(np.log2(max(n // 16, 2)))))
    if kind == 0:
        om = min(1 << 8, pow_om)
        return random_snn(n, 31, s, omega=om, delta=4 * om, name="job%d-rand-e32" % i)
    if kind == 1:
        om = min(1 << 10, pow_om)
        return random_snn(n, min(191, n - 1), s, omega=om, delta=4 * om, name="job%d-rand-e192" % i)
    if kind == 2:
        width = max(64, n // 8)
        window = max(16, min(2048, width // 4))
        om = min(1 << 12, pow_om)
        return layered_snn(8, width, min(255, window), window, 0.8, s, omega=om, delta=16 * om,
                           name="job%d-layered" % i)
    if kind == 3:
        hw = max(4, int(round(np.sqrt(n / (7 * 32)))))
        om = min(1 << 12, pow_om)
        return conv_snn(7, hw, 32, 82.0, s, omega=om, delta=16 * om, name="job%d-conv" % i, threads=1)
    k = 1 << int(np.clip(round(np.log2(n / 8000.0)), 1, 6))
    return netlist(n, int(1.1 * n), 2, min(2000, n // 2), 2.827, min(2048, n // 4), 0.9, 8, s, k=k,
                   name="job%d-netlist" % i)


def job_stream(n_jobs: int = 256, min_nodes: int = 2048, max_nodes: int = 262144, seed: int = 0,
               rate: float = 0.0, arrival_seed: int = 12345):
    """The batched/served workload: n_jobs jobs of job_specs / make_job.  With
    rate > 0, arrival times follow a Poisson process of that many jobs per
    second.  Returns (jobs, arrivals)."""
    import concurrent.futures as cf
    import os

    sizes, kinds = job_specs(n_jobs, min_nodes, max_nodes, seed)
    # every job draws from its own seed, so building them on worker threads
    # (largest first) gives the same jobs as building them in order
    order = sorted(range(n_jobs), key=lambda i: -int(sizes[i]))
    threads = max(1, min(16, os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(threads) as ex:
        built = dict(zip(order, ex.map(lambda i: make_job(i, sizes, kinds, seed), order)))
    jobs = [built[i] for i in range(n_jobs)]
    if rate > 0:
        arng = np.random.default_rng(arrival_seed)
        arrivals = np.cumsum(arng.exponential(1.0 / rate, size=n_jobs))
    else:
        arrivals = np.zeros(n_jobs)
    return jobs, arrivals


WORKLOADS = {
    "rand-4k-e32": rand_4k_e32,
    "rand-64k-e192": rand_64k_e192,
    "layered-256k-e256": layered_256k_e256,
    "conv-6.9m": conv_6_9m,
    "netlist-500k": netlist_500k,
}
