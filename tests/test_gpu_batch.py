"""Batched execution (hgp_run_jobs): jobs of uneven size from the five
workload families run on several concurrent contexts.  Each job's partition
must be the one it gets alone (one worker, one job at a time), the smallest
ones must equal the oracle's, and admission must respect arrival times."""
import numpy as np
import pytest

import oracle
from paper_2605_20497_amd import workloads as W

pytestmark = pytest.mark.gpu


def _digest(a):
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def test_batched_equals_alone_and_oracle():
    from paper_2605_20497_amd import hgp_run_jobs
    jobs, _ = W.job_stream(10, 2048, 6144, seed=3)
    print("jobs", [(j.name, j.n_nodes, j.n_pins) for j in jobs], flush=True)
    alone = hgp_run_jobs(jobs, workers=1)
    arrivals = np.linspace(0.0, 0.05, len(jobs))
    mixed = hgp_run_jobs(jobs, workers=4, arrivals=arrivals)
    for i, (a, b) in enumerate(zip(alone, mixed)):
        assert a["status"] == 0 and b["status"] == 0, (i, a["status"], b["status"])
        assert a["violations"] == 0 and b["violations"] == 0
        assert np.array_equal(a["rho"], b["rho"]), i
        assert (a["conn"], a["n_parts"], a["n_levels"]) == (b["conn"], b["n_parts"], b["n_levels"])
        assert b["start_s"] >= arrivals[i] - 1e-6
        assert b["end_s"] >= b["start_s"]
    order = sorted(range(len(jobs)), key=lambda i: jobs[i].n_pins)[:3]
    for i in order:
        hg = jobs[i]
        res = oracle.Graph(hg).partition(hg.omega, hg.delta, k=hg.k, Pi=4, theta=16, seed=0)
        print("oracle", hg.name, res.nlevels, res.conn, flush=True)
        assert np.array_equal(mixed[i]["rho"], res.rho(0)), hg.name
        assert mixed[i]["conn"] == res.conn


def test_run_jobs_arguments():
    from paper_2605_20497_amd import HgpError, hgp_run_jobs
    jobs, _ = W.job_stream(2, 2048, 2048, seed=1)
    with pytest.raises(HgpError):  # arrivals must be sorted
        hgp_run_jobs(jobs, workers=2, arrivals=[0.1, 0.0])
    with pytest.raises(HgpError):
        hgp_run_jobs(jobs, workers=0)
    assert hgp_run_jobs([], workers=2) == []


def test_release_then_reload():
    """hgp_release frees the job's device memory; the context refuses calls
    that read a job until the next load, and then gives the same result."""
    import paper_2605_20497_amd as pkg
    jobs, _ = W.job_stream(2, 4096, 4096, seed=5)
    p = pkg.Partitioner(device=0)
    try:
        first = [p.partition(hg) for hg in jobs]
        for workspace_too in (False, True):
            p.hgp_release(workspace_too)
            with pytest.raises(pkg.HgpError):
                p.hgp_get_partition()
            with pytest.raises(pkg.HgpError):
                p.hgp_coarsen()
            again = [p.partition(hg) for hg in jobs]
            for (ra, ka), (rb, kb) in zip(first, again):
                assert np.array_equal(ra, rb) and ka == kb
    finally:
        p.close()
