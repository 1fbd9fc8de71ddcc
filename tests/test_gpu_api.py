"""Entry points of the C ABI beyond the partitioning run itself: the k-way
limits computed from the balance parameter (Sec. VII-A), and allocation
failure (HGP_E_NOMEM) leaving the context usable and destroyable."""
import ctypes as C

import numpy as np
import pytest

from paper_2605_20497_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_kway_limits_from_eps():
    from paper_2605_20497_amd import Partitioner
    hg = W.netlist(6000, 6600, 2, 80, 2.827, 256, 0.9, 8, seed=2, k=8, delta=1 << 15)
    print("case kway eps N", hg.n_nodes, "P", hg.n_pins, flush=True)
    W_tot = int(hg.node_w.sum())
    g = Partitioner()
    g.load(hg)
    om = g.hgp_set_kway_limits(8, 3, 100, 1 << 15)
    # Omega = (1 + 3/100) * ceil(W / 8), rounded down
    assert om == (103 * ((W_tot + 7) // 8)) // 100 == hg.omega
    g.hgp_coarsen()
    g.hgp_refine()
    rho, n = g.hgp_get_partition()
    h = Partitioner()
    rho2, n2 = h.partition(hg, hg.omega, 1 << 15, 8)
    assert n == n2 == 8 and np.array_equal(rho, rho2)
    # eps = 0 with a non-divisible W: ceil(W / k) exactly
    assert g.hgp_set_kway_limits(7, 0, 1, 1 << 15) == (W_tot + 6) // 7
    g.close()
    h.close()


def test_nomem_mid_coarsening_leaves_context_usable():
    import torch
    import paper_2605_20497_amd as pkg
    hg = W.random_snn(3000, 31, seed=5)
    print("case nomem N", hg.n_nodes, "P", hg.n_pins, flush=True)
    L = pkg.lib()
    state = {"n": 0, "fail_after": None}

    def _alloc(nbytes, stream, user):
        state["n"] += 1
        if state["fail_after"] is not None and state["n"] > state["fail_after"]:
            return None
        return torch.cuda.caching_allocator_alloc(int(nbytes), 0, stream)

    def _free(ptr, nbytes, stream, user):
        torch.cuda.caching_allocator_delete(ptr)

    A, F = pkg.ALLOC_FN(_alloc), pkg.FREE_FN(_free)
    opt = pkg.hgp_options()
    L.hgp_default_options(C.byref(opt))
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream(0)
    opt.stream = C.c_void_p(stream.cuda_stream)
    opt.alloc, opt.free = A, F
    h = C.c_void_p()
    assert L.hgp_create(C.byref(h), C.byref(opt)) == pkg.HGP_OK
    p = lambda a: a.ctypes.data_as(C.c_void_p)

    def load():
        return L.hgp_load_csr(h, hg.n_nodes, hg.n_hedges, p(hg.he_off), p(hg.he_nsrc), p(hg.pins), None, None,
                              pkg.HGP_MEM_HOST)

    # the first allocation of the load fails
    state["fail_after"] = 0
    assert load() == pkg.HGP_E_NOMEM
    assert b"allocation" in L.hgp_last_error(h)
    state["fail_after"] = None
    assert load() == pkg.HGP_OK
    assert L.hgp_set_limits(h, 64, 1 << 12, 0) == pkg.HGP_OK
    # an allocation partway through coarsening fails
    state["n"], state["fail_after"] = 0, 6
    nl = C.c_int32()
    assert L.hgp_coarsen(h, C.byref(nl)) == pkg.HGP_E_NOMEM
    assert L.hgp_refine(h) == pkg.HGP_E_STATE
    state["fail_after"] = None
    assert L.hgp_coarsen(h, C.byref(nl)) == pkg.HGP_OK
    assert L.hgp_refine(h) == pkg.HGP_OK
    rho = np.zeros(hg.n_nodes, np.int32)
    k = C.c_int32()
    assert L.hgp_get_partition(h, p(rho), hg.n_nodes, C.byref(k)) == pkg.HGP_OK
    L.hgp_destroy(h)
    ref = pkg.Partitioner()
    rho2, k2 = ref.partition(hg, 64, 1 << 12, 0)
    ref.close()
    assert k.value == k2 and np.array_equal(rho, rho2)


def test_tuning_choices_leave_results_unchanged():
    # the hashed proposal everywhere, with the smallest and largest tables and
    # both extremes of the refinement edge-list gate
    from paper_2605_20497_amd import HgpError, Partitioner
    hg = W.random_snn(20000, 23, seed=9)
    print("case tuning N", hg.n_nodes, "P", hg.n_pins, flush=True)
    ref = Partitioner(sparse_proposal=True)
    rho0, k0 = ref.partition(hg, 256, 2048, 0)
    conn0 = ref.hgp_evaluate()["conn"]
    ref.close()
    for tune in ({"hash_log2": 10, "list_gate": 1}, {"hash_log2": 13, "list_gate": 64}):
        g = Partitioner(sparse_proposal=True, tune=tune)
        rho, k = g.partition(hg, 256, 2048, 0)
        assert k == k0 and np.array_equal(rho, rho0) and g.hgp_evaluate()["conn"] == conn0, tune
        g.close()
    with pytest.raises(HgpError):
        Partitioner(tune={"hash_log2": 9})
