"""Python binding of ``libhgp.so`` (the C ABI declared in ``include/hgp.h``).

Argument marshalling only: every step of the partitioner runs in the library's
HIP kernels.  PyTorch provides device memory (its caching allocator is handed
to the library as the allocator callback) and the stream (the current torch
stream).  The binding raises if the library is not built; there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhgp.so")

HGP_OK, HGP_E_INVALID, HGP_E_INFEASIBLE, HGP_E_NOMEM, HGP_E_DEVICE, HGP_E_STATE, HGP_E_UNSUPPORTED = range(7)
HGP_MEM_HOST, HGP_MEM_DEVICE = 0, 1
HGP_DELTA_INBOUND, HGP_DELTA_OUTBOUND, HGP_DELTA_INCIDENT = 0, 1, 2
INT64_MAX = (1 << 63) - 1

_STATUS = {0: "OK", 1: "INVALID", 2: "INFEASIBLE", 3: "NOMEM", 4: "DEVICE", 5: "STATE", 6: "UNSUPPORTED"}

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)


class hgp_options(C.Structure):
    _fields_ = [("device", C.c_int32), ("stream", C.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN),
                ("alloc_user", C.c_void_p), ("pi", C.c_int32), ("theta", C.c_int32), ("seed", C.c_uint64),
                ("profile", C.c_int32), ("flags", C.c_int32), ("profile_families", C.c_uint32),
                ("delta_mode", C.c_int32), ("tune", C.c_int32 * 4)]


class hgp_eval(C.Structure):
    _fields_ = [("conn", C.c_int64), ("cutnet", C.c_int64), ("max_size", C.c_int64),
                ("max_inbound", C.c_int64), ("violations", C.c_int64), ("n_parts", C.c_int64)]


class hgp_job(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_hedges", C.c_int32), ("he_off", C.c_void_p), ("he_nsrc", C.c_void_p),
                ("pins", C.c_void_p), ("hedge_w", C.c_void_p), ("node_w", C.c_void_p), ("omega", C.c_int64),
                ("delta", C.c_int64), ("k", C.c_int32), ("arrival_s", C.c_double), ("rho", C.c_void_p),
                ("n_parts", C.c_int32), ("n_levels", C.c_int32), ("conn", C.c_int64), ("violations", C.c_int64),
                ("start_s", C.c_double), ("end_s", C.c_double), ("footprint", C.c_int64), ("status", C.c_int),
                ("reruns", C.c_int32)]


class HgpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_STATUS.get(status, status), msg))
        self.status = status


_lib = None


def lib():
    """Loads libhgp.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libhgp.so is not built; run paper_2605_20497_amd.build.build() "
                              "(or __graft_entry__.build()) first")
        # torch ships its own HIP runtime, requested by an unversioned name;
        # importing torch first makes libhgp.so bind to that same runtime (its
        # soname matches), so the process holds one runtime, not two.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        P, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        sig = {
            "hgp_default_options": (None, [C.POINTER(hgp_options)]),
            "hgp_create": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(hgp_options)]),
            "hgp_destroy": (None, [P]),
            "hgp_release": (C.c_int, [P, i32]),
            "hgp_last_error": (C.c_char_p, [P]),
            "hgp_load_csr": (C.c_int, [P, i32, i32, P, P, P, P, P, C.c_int]),
            "hgp_set_limits": (C.c_int, [P, i64, i64, i32]),
            "hgp_set_kway_limits": (C.c_int, [P, i32, i32, i32, i64, C.POINTER(i64)]),
            "hgp_coarsen": (C.c_int, [P, C.POINTER(i32)]),
            "hgp_refine": (C.c_int, [P]),
            "hgp_get_levels": (C.c_int, [P, P, i64]),
            "hgp_get_cluster_map": (C.c_int, [P, i32, P, i64]),
            "hgp_get_proposal": (C.c_int, [P, i32, P, P, P, i64]),
            "hgp_get_level_graph": (C.c_int, [P, i32, P, P, P, P]),
            "hgp_get_partition": (C.c_int, [P, P, i64, C.POINTER(i32)]),
            "hgp_get_phi": (C.c_int, [P, P, P, P, P, i64, C.POINTER(i64)]),
            "hgp_evaluate": (C.c_int, [P, P, i32, C.POINTER(hgp_eval)]),
            "hgp_evaluate_noalloc": (C.c_int, [P, P, i32, C.POINTER(hgp_eval)]),
            "hgp_refine_rep": (C.c_int, [P, P, i32, i32, P, P, P, P, P, P, P, P]),
            "hgp_kernel_stats": (C.c_int, [P, C.POINTER(C.c_char_p), P, P, C.POINTER(i32)]),
            "hgp_reset_kernel_stats": (C.c_int, [P]),
            "hgp_kernel_work": (C.c_int, [P, P, C.POINTER(i32)]),
            "hgp_level_times": (C.c_int, [P, P, i64]),
            "hgp_kernel_level_stats": (C.c_int, [P, P, i64, C.POINTER(i32)]),
            "hgp_run_jobs": (C.c_int, [C.POINTER(hgp_options), C.POINTER(hgp_job), i64, i32, i64]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


# Kernel families in the library's order (hgp_kernel_stats names).
KERNEL_FAMILIES = ["validate", "transpose", "radix_sort", "scan", "level_stats", "propose", "match", "isolated",
                   "gamma", "contract_edges", "pack", "phi", "part_stats", "gains", "moves", "chains", "rank",
                   "inseq", "events", "select", "apply", "project", "eval", "misc", "propose_dense", "dense_gemm",
                   "gains_gemm"]

EXPORTED = ["hgp_default_options", "hgp_create", "hgp_destroy", "hgp_release", "hgp_last_error", "hgp_load_csr",
            "hgp_set_limits", "hgp_set_kway_limits", "hgp_coarsen", "hgp_refine", "hgp_get_levels", "hgp_get_cluster_map",
            "hgp_get_proposal", "hgp_get_level_graph", "hgp_get_partition", "hgp_get_phi", "hgp_evaluate",
            "hgp_evaluate_noalloc",
            "hgp_refine_rep", "hgp_kernel_stats", "hgp_reset_kernel_stats", "hgp_kernel_work", "hgp_level_times",
            "hgp_kernel_level_stats",
            "hgp_run_jobs"]


def hgp_run_jobs(graphs, workers=1, arrivals=None, hbm_budget=0, pi=4, theta=16, seed=0, device=0, flags=0,
                 delta_mode=0):
    """Runs a list of hypergraphs (workloads.Hypergraph, with their omega,
    delta and k) as jobs on `workers` concurrent contexts; `arrivals` are the
    seconds after the start at which each may be admitted (sorted; default
    all 0).  Returns one dict per job: rho, n_parts, n_levels, conn,
    violations, start_s, end_s, footprint, status, reruns."""
    n = len(graphs)
    arr = [0.0] * n if arrivals is None else [float(a) for a in arrivals]
    jobs = (hgp_job * max(n, 1))()
    keep = []
    rhos = []
    for i, hg in enumerate(graphs):
        cols = [np.ascontiguousarray(hg.he_off, np.int64), np.ascontiguousarray(hg.he_nsrc, np.int32),
                np.ascontiguousarray(hg.pins, np.int32), np.ascontiguousarray(hg.hedge_w, np.int32),
                np.ascontiguousarray(hg.node_w, np.int32)]
        keep.append(cols)
        rho = np.zeros(hg.n_nodes, np.int32)
        rhos.append(rho)
        j = jobs[i]
        j.n_nodes, j.n_hedges = hg.n_nodes, hg.n_hedges
        j.he_off, j.he_nsrc, j.pins, j.hedge_w, j.node_w = (c.ctypes.data for c in cols)
        j.omega, j.delta, j.k = int(hg.omega), int(hg.delta), int(hg.k)
        j.arrival_s = arr[i]
        j.rho = rho.ctypes.data
    opt = hgp_options()
    lib().hgp_default_options(C.byref(opt))
    opt.device, opt.pi, opt.theta, opt.seed, opt.flags = device, pi, theta, seed, flags
    opt.delta_mode = int(delta_mode)
    st = lib().hgp_run_jobs(C.byref(opt), jobs, n, int(workers), int(hbm_budget))
    if st != 0:
        raise HgpError(st, "hgp_run_jobs failed")
    out = []
    for i in range(n):
        j = jobs[i]
        out.append({"rho": rhos[i], "n_parts": j.n_parts, "n_levels": j.n_levels, "conn": j.conn,
                    "violations": j.violations, "start_s": j.start_s, "end_s": j.end_s,
                    "footprint": j.footprint, "status": j.status, "reruns": j.reruns})
    return out


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _torch_allocator(device):
    """Allocator callbacks backed by torch's caching allocator."""
    import torch

    def _alloc(nbytes, stream, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device, stream)
        except Exception:  # noqa: BLE001 - the library turns NULL into HGP_E_NOMEM
            return None

    def _free(ptr, nbytes, stream, user):
        try:
            torch.cuda.caching_allocator_delete(ptr)
        except Exception:  # noqa: BLE001 - interpreter teardown: the process frees everything
            pass

    return ALLOC_FN(_alloc), FREE_FN(_free)


class Partitioner:
    """One library context on one device and torch stream."""

    def __init__(self, device: int = 0, pi: int = 4, theta: int = 16, seed: int = 0, profile: bool = False,
                 use_torch: bool = True, stream=None, sparse_proposal: bool = False, profile_families=(),
                 dense_proposal=None, dense_gains=None, delta_mode=0, no_chains=False, greedy_matching=False,
                 tune=None):
        L = lib()
        opt = hgp_options()
        L.hgp_default_options(C.byref(opt))
        opt.device, opt.pi, opt.theta, opt.seed, opt.profile = device, pi, theta, seed, int(profile)
        # flags: bit 0 hashed proposal everywhere; bit 1 dense (MFMA) proposal wherever it
        # fits; bit 2 never dense; neither of bits 1-2 = chosen per level by cost; bits 3-4
        # the same choice for the in-isolation moves of refinement; bit 5 the ablation
        # without chain rounds; bit 6 the ablation with the prototype's greedy matching
        opt.flags = ((1 if sparse_proposal else 0) | {None: 0, True: 2, False: 4}[dense_proposal]
                     | {None: 0, True: 8, False: 16}[dense_gains] | (32 if no_chains else 0)
                     | (64 if greedy_matching else 0))
        # what Delta counts: 0 inbound h-edges (the paper's), 1 outbound, 2 incident
        opt.delta_mode = int(delta_mode)
        # tile and schedule choices (autotune.py): {"hash_log2": 10..13, "list_gate": 1..64}
        if tune:
            opt.tune[0] = int(tune.get("hash_log2", 0))
            opt.tune[1] = int(tune.get("list_gate", 0))
        # kernel families to time (names as in hgp_kernel_stats); empty = all
        opt.profile_families = sum(1 << KERNEL_FAMILIES.index(f) for f in profile_families)
        self._keep = []
        self._stream = None
        if use_torch:
            import torch
            torch.cuda.set_device(device)
            if stream is None:
                stream = torch.cuda.Stream(device)  # default priority
            opt.stream = C.c_void_p(stream.cuda_stream)
            self._stream = stream
            a, f = _torch_allocator(device)
            opt.alloc, opt.free = a, f
            self._keep += [a, f, stream]
        self.pi, self.theta = pi, theta
        h = C.c_void_p()
        st = L.hgp_create(C.byref(h), C.byref(opt))
        if st != HGP_OK:
            raise HgpError(st, "hgp_create failed")
        self.h = h.value
        self.N = self.E = self.P = 0

    def close(self):
        if getattr(self, "h", None):
            lib().hgp_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def _chk(self, st):
        if st != HGP_OK:
            raise HgpError(st, lib().hgp_last_error(self.h).decode())

    # -- calls with the C ABI's names --------------------------------------
    def hgp_release(self, workspace_too=False):
        self._chk(lib().hgp_release(self.h, 1 if workspace_too else 0))
        self.N = self.E = self.P = 0

    def hgp_load_csr(self, n_nodes, he_off, he_nsrc, pins, hedge_w=None, node_w=None):
        he_off = np.ascontiguousarray(he_off, np.int64)
        he_nsrc = np.ascontiguousarray(he_nsrc, np.int32)
        pins = np.ascontiguousarray(pins, np.int32)
        hw = None if hedge_w is None else np.ascontiguousarray(hedge_w, np.int32)
        nw = None if node_w is None else np.ascontiguousarray(node_w, np.int32)
        E = he_nsrc.shape[0]
        self._chk(lib().hgp_load_csr(self.h, int(n_nodes), int(E), _p(he_off), _p(he_nsrc), _p(pins), _p(hw),
                                     _p(nw), HGP_MEM_HOST))
        self.N, self.E, self.P = int(n_nodes), int(E), int(he_off[-1])

    def hgp_load_csr_device(self, n_nodes, he_off, he_nsrc, pins, hedge_w=None, node_w=None):
        """Same, from torch device tensors (int64 / int32)."""
        import torch
        self._stream.wait_stream(torch.cuda.current_stream())
        ptr = lambda t: None if t is None else C.c_void_p(t.data_ptr())
        self._chk(lib().hgp_load_csr(self.h, int(n_nodes), int(he_nsrc.numel()), ptr(he_off), ptr(he_nsrc),
                                     ptr(pins), ptr(hedge_w), ptr(node_w), HGP_MEM_DEVICE))
        self.N, self.E, self.P = int(n_nodes), int(he_nsrc.numel()), int(pins.numel())

    def hgp_set_limits(self, omega, delta, k=0):
        self._chk(lib().hgp_set_limits(self.h, int(omega), int(delta), int(k)))

    def hgp_set_kway_limits(self, k, eps_num, eps_den, delta=INT64_MAX):
        om = C.c_int64()
        self._chk(lib().hgp_set_kway_limits(self.h, int(k), int(eps_num), int(eps_den), int(delta), C.byref(om)))
        return om.value

    def hgp_coarsen(self):
        n = C.c_int32()
        self._chk(lib().hgp_coarsen(self.h, C.byref(n)))
        self.nlevels = n.value
        return n.value

    def hgp_refine(self):
        self._chk(lib().hgp_refine(self.h))

    def hgp_get_levels(self):
        out = np.zeros(4 * self.nlevels, np.int64)
        self._chk(lib().hgp_get_levels(self.h, _p(out), out.size))
        return out.reshape(-1, 4)

    def hgp_get_cluster_map(self, level):
        n = int(self.hgp_get_levels()[level, 0])
        out = np.zeros(n, np.int32)
        self._chk(lib().hgp_get_cluster_map(self.h, level, _p(out), n))
        return out

    def hgp_get_proposal(self, level):
        n = int(self.hgp_get_levels()[level, 0])
        cand = np.zeros((n, self.pi), np.int32)
        score = np.zeros((n, self.pi), np.uint64)
        match = np.zeros(n, np.int32)
        self._chk(lib().hgp_get_proposal(self.h, level, _p(cand), _p(score), _p(match), n))
        return cand, score, match

    def hgp_get_level_graph(self, level, what=("he_off", "he_nsrc", "pins", "node_w")):
        """Level `level`'s CSR; arrays not named in `what` are not copied (None)."""
        N, E, P, _ = (int(x) for x in self.hgp_get_levels()[level])
        he_off = np.zeros(E + 1, np.int64) if "he_off" in what else None
        nsrc = np.zeros(E, np.int32) if "he_nsrc" in what else None
        pins = np.zeros(P, np.int32) if "pins" in what else None
        nw = np.zeros(N, np.int32) if "node_w" in what else None
        opt = lambda a: _p(a) if a is not None else None
        self._chk(lib().hgp_get_level_graph(self.h, level, opt(he_off), opt(nsrc), opt(pins), opt(nw)))
        return he_off, nsrc, pins, nw

    def hgp_get_partition(self):
        rho = np.zeros(self.N, np.int32)
        k = C.c_int32()
        self._chk(lib().hgp_get_partition(self.h, _p(rho), self.N, C.byref(k)))
        return rho, k.value

    def hgp_get_phi(self):
        need = C.c_int64()
        self._chk(lib().hgp_get_phi(self.h, None, None, None, None, 0, C.byref(need)))
        L = need.value
        off = np.zeros(self.E + 1, np.int64)
        part = np.zeros(L, np.int32)
        cnt = np.zeros(L, np.int32)
        cin = np.zeros(L, np.int32)
        self._chk(lib().hgp_get_phi(self.h, _p(off), _p(part), _p(cnt), _p(cin), L, C.byref(need)))
        return off, part, cnt, cin

    def hgp_evaluate(self, rho=None, n_parts=0):
        ev = hgp_eval()
        r = None if rho is None else np.ascontiguousarray(rho, np.int32)
        self._chk(lib().hgp_evaluate(self.h, _p(r), int(n_parts), C.byref(ev)))
        return dict(conn=ev.conn, cutnet=ev.cutnet, max_size=ev.max_size, max_inbound=ev.max_inbound,
                    violations=ev.violations, n_parts=ev.n_parts)

    def hgp_evaluate_noalloc(self, rho, n_parts):
        """rho: int32 torch tensor on this context's device (N entries)."""
        import torch
        if rho.dtype != torch.int32 or not rho.is_cuda or not rho.is_contiguous():
            raise ValueError("rho must be a contiguous int32 device tensor")
        self._stream.wait_stream(torch.cuda.current_stream())
        ev = hgp_eval()
        self._chk(lib().hgp_evaluate_noalloc(self.h, C.c_void_p(rho.data_ptr()), int(n_parts), C.byref(ev)))
        return dict(conn=ev.conn, cutnet=ev.cutnet, max_size=ev.max_size, max_inbound=ev.max_inbound,
                    violations=ev.violations, n_parts=ev.n_parts)

    def hgp_refine_rep(self, rho, n_parts, rep):
        r = np.array(rho, np.int32, copy=True)
        N = r.shape[0]
        info = np.zeros(4, np.int64)
        seq = np.zeros(N, np.int32)
        sd = np.zeros(N, np.int32)
        gseq = np.zeros(N, np.int64)
        Ck = np.zeros(N + 1, np.int64)
        Vk = np.zeros(N + 1, np.int64)
        mdst = np.zeros(N, np.int32)
        mgain = np.zeros(N, np.int64)
        self._chk(lib().hgp_refine_rep(self.h, _p(r), int(n_parts), int(rep), _p(info), _p(mdst), _p(mgain), _p(seq),
                                       _p(sd), _p(gseq), _p(Ck), _p(Vk)))
        M = int(info[0])
        return r, dict(moves=M, kstar=int(info[1]), gain=int(info[2]), links=int(info[3]), move_dst=mdst,
                       move_gain=mgain, seq=seq[:M],
                       seq_pd=sd[:M], gseq=gseq[:M], C=Ck[:M + 1], V=Vk[:M + 1])

    def hgp_kernel_stats(self):
        cnt = C.c_int32()
        self._chk(lib().hgp_kernel_stats(self.h, None, None, None, C.byref(cnt)))
        n = cnt.value
        names = (C.c_char_p * n)()
        launches = np.zeros(n, np.int64)
        ns = np.zeros(n, np.int64)
        self._chk(lib().hgp_kernel_stats(self.h, names, _p(launches), _p(ns), C.byref(cnt)))
        return {names[i].decode(): (int(launches[i]), int(ns[i])) for i in range(n)}

    def hgp_reset_kernel_stats(self):
        self._chk(lib().hgp_reset_kernel_stats(self.h))

    def hgp_kernel_work(self):
        """Device-counted work units per kernel family while profiled
        (gains: Phi row entries read); {family name: units}."""
        cnt = C.c_int32()
        self._chk(lib().hgp_kernel_work(self.h, None, C.byref(cnt)))
        work = np.zeros(cnt.value, np.int64)
        self._chk(lib().hgp_kernel_work(self.h, _p(work), C.byref(cnt)))
        return {KERNEL_FAMILIES[i]: int(work[i]) for i in range(min(cnt.value, len(KERNEL_FAMILIES)))}

    def hgp_level_times(self):
        out = np.zeros(2 * self.nlevels, np.int64)
        self._chk(lib().hgp_level_times(self.h, _p(out), out.size))
        return out.reshape(-1, 2)

    def hgp_kernel_level_stats(self):
        """{family: array [levels, 3] of (launches, ns, algorithmic bytes)}."""
        nl = C.c_int32()
        self._chk(lib().hgp_kernel_level_stats(self.h, None, 0, C.byref(nl)))
        F = len(KERNEL_FAMILIES)
        out = np.zeros(nl.value * F * 3, np.int64)
        self._chk(lib().hgp_kernel_level_stats(self.h, _p(out), out.size, C.byref(nl)))
        out = out.reshape(nl.value, F, 3)
        return {f: out[:, i, :] for i, f in enumerate(KERNEL_FAMILIES)}

    # -- convenience -------------------------------------------------------
    def load(self, hg):
        self.hgp_load_csr(hg.n_nodes, hg.he_off, hg.he_nsrc, hg.pins, hg.hedge_w, hg.node_w)

    def partition(self, hg, omega=None, delta=None, k=None):
        self.load(hg)
        self.hgp_set_limits(hg.omega if omega is None else omega, hg.delta if delta is None else delta,
                            hg.k if k is None else k)
        self.hgp_coarsen()
        self.hgp_refine()
        return self.hgp_get_partition()
