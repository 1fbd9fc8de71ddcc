"""ctypes view of the serial C++ oracle (``oracle/hgp_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``.  The library package never imports
this module and the oracle never imports the library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "hgp_oracle.cpp")
LIB = os.path.join(_HERE, "libhgp_oracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with the host compiler (it is plain serial C++)."""
    if os.environ.get("HGP_ORACLE_LIB"):
        return os.environ["HGP_ORACLE_LIB"]
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        # HGP_ORACLE_LIB names another build of this source (the mutation
        # tests load deliberately broken copies through it)
        path = os.environ.get("HGP_ORACLE_LIB") or LIB
        if path == LIB and not os.path.exists(LIB):
            build()
        L = C.CDLL(path)
        P, i32, i64, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
        sig = {
            "hgpo_graph_new": (C.c_int, [i32, i32, P, P, P, P, P, C.POINTER(C.c_void_p), C.c_char_p, C.c_int]),
            "hgpo_graph_free": (None, [P]),
            "hgpo_graph_dims": (None, [P, P]),
            "hgpo_graph_csr": (None, [P, P, P, P, P, P]),
            "hgpo_graph_incidence": (None, [P, P, P, P]),
            "hgpo_mix64": (u64, [u64]),
            "hgpo_noise": (u64, [u64, i32, i32, u64]),
            "hgpo_noise_cap": (u64, [P]),
            "hgpo_tnorm": (u64, [P, i32]),
            "hgpo_pair": (None, [P, i32, i32, P, P]),
            "hgpo_propose": (C.c_int, [P, i64, i64, u64, i32, P, i32, P, P]),
            "hgpo_match_round": (C.c_int, [i32, P, P, P, P, C.c_char_p, C.c_int]),
            "hgpo_match_round_greedy": (C.c_int, [i32, P, P, P, P, C.c_char_p, C.c_int]),
            "hgpo_match": (C.c_int, [P, i64, i64, i32, P, P, P, P, C.c_char_p, C.c_int]),
            "hgpo_contract": (C.c_int, [P, P, P, C.POINTER(C.c_void_p)]),
            "hgpo_evaluate": (C.c_int, [P, P, i32, i64, i64, P, P, P]),
            "hgpo_phi": (i64, [P, P, P, P, P, P]),
            "hgpo_gain": (i64, [P, P, i32, i32]),
            "hgpo_moves": (C.c_int, [P, P, i32, i32, i32, i64, P, P]),
            "hgpo_refine_rep": (C.c_int, [P, P, i32, i32, i32, i64, i64, P, P, P, P, P, P, P]),
            "hgpo_kway_initial": (C.c_int, [P, i32, i64, i64, P, C.c_char_p, C.c_int]),
            "hgpo_sequence": (C.c_int, [i32, P, P, i64, P, P, P, P, i32, P, P, P]),
            "hgpo_partition": (C.c_int, [P, i64, i64, i32, i32, i32, u64, i32, C.POINTER(C.c_void_p), C.c_char_p, C.c_int]),
            "hgpo_result_free": (None, [P]),
            "hgpo_result_nlevels": (i32, [P]),
            "hgpo_result_nparts": (i32, [P]),
            "hgpo_result_graph": (P, [P, i32]),
            "hgpo_result_level": (None, [P, i32, P]),
            "hgpo_result_gamma": (None, [P, i32, P]),
            "hgpo_result_rho": (None, [P, i32, P]),
            "hgpo_result_ncoarsened": (i32, [P]),
            "hgpo_result_proposal": (None, [P, i32, P, P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class OracleError(RuntimeError):
    pass


def mix64(x: int) -> int:
    return int(lib().hgpo_mix64(C.c_uint64(x)))


def noise(seed: int, a: int, b: int, cap: int) -> int:
    return int(lib().hgpo_noise(seed, a, b, cap))


def sequence(node_w, n_in, moves, rounds=16):
    """Sequence of an explicit move list (Sec. VI-C): `moves` = rows of (node,
    p_s, p_d, gain); node_w / n_in give each node's size and |in(n)|.  Returns
    (node ids in sequence order, chain lengths, links, rounds run)."""
    mv = np.asarray(moves, np.int64).reshape(-1, 4)
    M = mv.shape[0]
    nw = np.ascontiguousarray(node_w, np.int64)
    nin = np.ascontiguousarray(n_in, np.int32)
    cols = [np.ascontiguousarray(mv[:, i], np.int32) for i in range(3)]
    gain = np.ascontiguousarray(mv[:, 3], np.int64)
    seq = np.zeros(max(M, 1), np.int32)
    cl = np.zeros(max(M, 1), np.int32)
    info = np.zeros(3, np.int64)
    rc = lib().hgpo_sequence(int(nw.shape[0]), _p(nw), _p(nin), M, _p(cols[0]), _p(cols[1]), _p(cols[2]),
                             _p(gain), int(rounds), _p(seq), _p(cl), _p(info))
    if rc != 0:
        raise OracleError("bad move list")
    return seq[:M].tolist(), cl[:int(info[2])].tolist(), int(info[0]), int(info[1])


def relabel(he_off, he_nsrc, pins, mode):
    """Constraint variants of the Delta cap (Sec. II-B counts the distinct
    inbound h-edges of a partition; the paper notes that outbound or incident
    counting are reformulations).  Delta only ever counts the h-edges whose
    destination pins touch a part, so relabelling pin roles selects the
    variant: mode 1 (outbound) makes each h-edge's sources its destinations
    and vice versa; mode 2 (incident, also undirected inputs) makes every pin
    a destination.  Blocks stay sorted.  Plain per-h-edge Python."""
    he_off = np.asarray(he_off, np.int64)
    he_nsrc = np.asarray(he_nsrc, np.int32)
    pins = np.asarray(pins, np.int32)
    if mode == 0:
        return he_off, he_nsrc, pins
    out = np.empty_like(pins)
    nsrc = np.empty_like(he_nsrc)
    for e in range(he_nsrc.shape[0]):
        a, b = int(he_off[e]), int(he_off[e + 1])
        src, dst = pins[a:a + int(he_nsrc[e])], pins[a + int(he_nsrc[e]):b]
        if mode == 1:
            out[a:b] = np.concatenate([dst, src])
            nsrc[e] = dst.shape[0]
        else:
            out[a:b] = np.sort(np.concatenate([src, dst]))
            nsrc[e] = 0
    return he_off, nsrc, out


class Graph:
    """Oracle-side hypergraph.  Built from the generator's CSR arrays;
    delta_mode selects the Delta variant (see relabel)."""

    def __init__(self, hg=None, *, n_nodes=None, he_off=None, he_nsrc=None, pins=None,
                 hedge_w=None, node_w=None, delta_mode=0, _handle=None, _owner=None):
        self._owner = _owner
        if _handle is not None:
            self.h = _handle
            self._own = _owner is None
        else:
            if hg is not None:
                n_nodes, he_off, he_nsrc, pins = hg.n_nodes, hg.he_off, hg.he_nsrc, hg.pins
                hedge_w, node_w = hg.hedge_w, hg.node_w
            he_off, he_nsrc, pins = relabel(he_off, he_nsrc, pins, delta_mode)
            he_off = np.ascontiguousarray(he_off, np.int64)
            he_nsrc = np.ascontiguousarray(he_nsrc, np.int32)
            pins = np.ascontiguousarray(pins, np.int32)
            E = he_nsrc.shape[0]
            hw = np.ascontiguousarray(hedge_w if hedge_w is not None else np.ones(E), np.int32)
            nw = np.ascontiguousarray(node_w if node_w is not None else np.ones(n_nodes), np.int32)
            h = C.c_void_p()
            err = C.create_string_buffer(256)
            rc = lib().hgpo_graph_new(int(n_nodes), int(E), _p(he_off), _p(he_nsrc), _p(pins), _p(hw), _p(nw),
                                      C.byref(h), err, 256)
            if rc != 0:
                raise OracleError(err.value.decode())
            self.h = h.value
            self._own = True
        d = np.zeros(3, np.int64)
        lib().hgpo_graph_dims(self.h, _p(d))
        self.N, self.E, self.P = int(d[0]), int(d[1]), int(d[2])

    def __del__(self):
        if getattr(self, "_own", False) and getattr(self, "h", None):
            try:
                lib().hgpo_graph_free(self.h)
            except Exception:  # interpreter teardown: the library may already be gone
                pass
            self.h = None

    # -- structure ---------------------------------------------------------
    def csr(self):
        he_off = np.zeros(self.E + 1, np.int64)
        nsrc = np.zeros(self.E, np.int32)
        pins = np.zeros(self.P, np.int32)
        hw = np.zeros(self.E, np.int32)
        nw = np.zeros(self.N, np.int32)
        lib().hgpo_graph_csr(self.h, _p(he_off), _p(nsrc), _p(pins), _p(hw), _p(nw))
        return he_off, nsrc, pins, hw, nw

    def incidence(self):
        off = np.zeros(self.N + 1, np.int64)
        nin = np.zeros(self.N, np.int32)
        inc = np.zeros(self.P, np.int32)
        lib().hgpo_graph_incidence(self.h, _p(off), _p(nin), _p(inc))
        return off, nin, inc

    # -- evaluation --------------------------------------------------------
    def evaluate(self, rho, nparts, omega=1 << 62, delta=1 << 62):
        rho = np.ascontiguousarray(rho, np.int32)
        out = np.zeros(8, np.int64)
        ps = np.zeros(nparts, np.int64)
        pi = np.zeros(nparts, np.int64)
        rc = lib().hgpo_evaluate(self.h, _p(rho), int(nparts), int(omega), int(delta), _p(out), _p(ps), _p(pi))
        if rc != 0:
            raise OracleError("rho out of range")
        return dict(conn=int(out[0]), cutnet=int(out[1]), max_size=int(out[2]), max_inbound=int(out[3]),
                    violations=int(out[4]), nonempty=int(out[5]), part_size=ps, part_inbound=pi)

    def phi(self, rho):
        rho = np.ascontiguousarray(rho, np.int32)
        L = lib().hgpo_phi(self.h, _p(rho), None, None, None, None)
        off = np.zeros(self.E + 1, np.int64)
        part = np.zeros(L, np.int32)
        cnt = np.zeros(L, np.int32)
        cin = np.zeros(L, np.int32)
        lib().hgpo_phi(self.h, _p(rho), _p(off), _p(part), _p(cnt), _p(cin))
        return off, part, cnt, cin

    # -- coarsening --------------------------------------------------------
    def noise_cap(self) -> int:
        return int(lib().hgpo_noise_cap(self.h))

    def tnorm(self, e: int) -> int:
        return int(lib().hgpo_tnorm(self.h, e))

    def pair(self, n: int, m: int):
        eta = np.zeros(1, np.uint64)
        inter = np.zeros(1, np.int32)
        lib().hgpo_pair(self.h, n, m, _p(eta), _p(inter))
        return int(eta[0]), int(inter[0])

    def propose(self, omega, delta, seed=0, Pi=4, nodes=None):
        if nodes is None:
            cnt = self.N
            nd = None
        else:
            nd = np.ascontiguousarray(nodes, np.int32)
            cnt = nd.shape[0]
        cand = np.zeros((cnt, Pi), np.int32)
        score = np.zeros((cnt, Pi), np.uint64)
        rc = lib().hgpo_propose(self.h, int(omega), int(delta), C.c_uint64(seed), Pi,
                                _p(nd) if nd is not None else None, cnt, _p(cand), _p(score))
        if rc != 0:
            raise OracleError("bad node list")
        return cand, score

    def match(self, omega, delta, cand, score):
        Pi = cand.shape[1]
        cand = np.ascontiguousarray(cand, np.int32)
        score = np.ascontiguousarray(score, np.uint64)
        m = np.zeros(self.N, np.int32)
        rp = np.zeros(Pi + 1, np.int32)
        err = C.create_string_buffer(256)
        rc = lib().hgpo_match(self.h, int(omega), int(delta), Pi, _p(cand), _p(score), _p(m), _p(rp), err, 256)
        if rc != 0:
            raise OracleError(err.value.decode())
        return m, rp

    def contract(self, match):
        match = np.ascontiguousarray(match, np.int32)
        gamma = np.zeros(self.N, np.int32)
        h = C.c_void_p()
        lib().hgpo_contract(self.h, _p(match), _p(gamma), C.byref(h))
        return gamma, Graph(_handle=h.value)

    # -- refinement --------------------------------------------------------
    def gain(self, rho, n, p) -> int:
        rho = np.ascontiguousarray(rho, np.int32)
        return int(lib().hgpo_gain(self.h, _p(rho), int(n), int(p)))

    def moves(self, rho, nparts, rep, theta, omega):
        rho = np.ascontiguousarray(rho, np.int32)
        dst = np.zeros(self.N, np.int32)
        gain = np.zeros(self.N, np.int64)
        lib().hgpo_moves(self.h, _p(rho), int(nparts), rep, theta, int(omega), _p(dst), _p(gain))
        return dst, gain

    def refine_rep(self, rho, nparts, rep, theta, omega, delta):
        """Runs one repetition; returns (new_rho, details)."""
        rho = np.array(rho, np.int32, copy=True)
        N = self.N
        seq = np.zeros(N, np.int32)
        spd = np.zeros(N, np.int32)
        gseq = np.zeros(N, np.int64)
        Ck = np.zeros(N + 1, np.int64)
        Vk = np.zeros(N + 1, np.int64)
        cl = np.zeros(N, np.int32)
        info = np.zeros(6, np.int64)
        lib().hgpo_refine_rep(self.h, _p(rho), int(nparts), rep, theta, int(omega), int(delta), _p(seq), _p(spd),
                              _p(gseq), _p(Ck), _p(Vk), _p(cl), _p(info))
        M = int(info[0])
        return rho, dict(M=M, kstar=int(info[1]), applied_gain=int(info[2]), links=int(info[3]),
                         rounds=int(info[4]), seq=seq[:M], seq_pd=spd[:M], gseq=gseq[:M], C=Ck[:M + 1],
                         V=Vk[:M + 1], chain_len=cl[:int(info[5])])

    def kway_initial(self, k, omega, delta):
        rho = np.zeros(self.N, np.int32)
        err = C.create_string_buffer(256)
        rc = lib().hgpo_kway_initial(self.h, k, int(omega), int(delta), _p(rho), err, 256)
        if rc != 0:
            raise OracleError(err.value.decode())
        return rho

    def partition(self, omega, delta, k=0, Pi=4, theta=16, seed=0, early_exit=True, chains=True,
                  greedy=False) -> "Result":
        # chains=False: the ablation without chain rounds (moves sequenced by gain alone)
        # greedy=True: the ablation with the prototype's greedy matching (Reading R28)
        h = C.c_void_p()
        err = C.create_string_buffer(256)
        rc = lib().hgpo_partition(self.h, int(omega), int(delta), int(k), Pi, theta, C.c_uint64(seed),
                                  int(bool(early_exit)) | (0 if chains else 2) | (4 if greedy else 0),
                                  C.byref(h), err, 256)
        if rc != 0:
            raise OracleError(err.value.decode())
        return Result(h.value, Pi)


class Result:
    def __init__(self, h, Pi):
        self.h = h
        self.Pi = Pi
        L = lib()
        self.nlevels = int(L.hgpo_result_nlevels(h))
        self.nparts = int(L.hgpo_result_nparts(h))
        self.ncoarsened = int(L.hgpo_result_ncoarsened(h))
        self.levels = []
        for lv in range(self.nlevels):
            out = np.zeros(24, np.int64)
            L.hgpo_result_level(h, lv, _p(out))
            self.levels.append(dict(N=int(out[0]), E=int(out[1]), P=int(out[2]), t_coarsen=out[3] * 1e-9,
                                    t_refine=out[4] * 1e-9, conn_after=int(out[5]), moves_applied=int(out[6]),
                                    pairs=[int(x) for x in out[7:7 + Pi + 1]]))

    def __del__(self):
        if getattr(self, "h", None):
            lib().hgpo_result_free(self.h)
            self.h = None

    def graph(self, lv) -> Graph:
        return Graph(_handle=lib().hgpo_result_graph(self.h, lv), _owner=self)

    def gamma(self, lv):
        out = np.zeros(self.levels[lv]["N"], np.int32)
        lib().hgpo_result_gamma(self.h, lv, _p(out))
        return out

    def rho(self, lv=0):
        out = np.zeros(self.levels[lv]["N"], np.int32)
        lib().hgpo_result_rho(self.h, lv, _p(out))
        return out

    def proposal(self, lv):
        N = self.levels[lv]["N"]
        cand = np.zeros((N, self.Pi), np.int32)
        score = np.zeros((N, self.Pi), np.uint64)
        match = np.zeros(N, np.int32)
        lib().hgpo_result_proposal(self.h, lv, _p(cand), _p(score), _p(match))
        return cand, score, match

    @property
    def conn(self):
        return self.levels[0]["conn_after"]
