"""Writes tests/golden/job_stream_256.json from the oracle alone: for every job
of the 256-job stream (2,048 to 262,144 nodes, log-uniform, five families;
paper_2605_20497_amd.workloads.job_specs / make_job) the oracle's partition
digest, connectivity and partition count, one oracle run per job in worker
processes.  Jobs of the two families whose serial oracle would take hours at
these sizes (random h-edges of 192 pins, the layered family) are listed
without a digest.  Usage:
    python tests/golden/make_jobstream_golden.py [workers]
"""
import concurrent.futures as cf
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

N_JOBS, MIN_NODES, MAX_NODES, SEED = 256, 2048, 262144, 0
SLOW_FAMILIES = ("rand-e192", "layered")


def digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def run(i):
    import oracle
    from paper_2605_20497_amd import workloads as W
    sizes, kinds = W.job_specs(N_JOBS, MIN_NODES, MAX_NODES, SEED)
    hg = W.make_job(i, sizes, kinds, SEED)
    out = {"job": i, "name": hg.name, "nodes": hg.n_nodes, "pins": hg.n_pins, "omega": hg.omega,
           "delta": hg.delta, "k": hg.k}
    if hg.name.split("-", 1)[1] in SLOW_FAMILIES:
        return out
    g = oracle.Graph(hg)
    t0 = time.time()
    res = g.partition(hg.omega, hg.delta, k=hg.k)
    out.update(nparts=res.nparts, conn=res.conn, rho_sha256=digest(res.rho(0)),
               oracle_seconds=round(time.time() - t0, 1))
    return out


def main(workers: int):
    from paper_2605_20497_amd import workloads as W
    sizes, kinds = W.job_specs(N_JOBS, MIN_NODES, MAX_NODES, SEED)
    order = sorted(range(N_JOBS), key=lambda i: -int(sizes[i]))
    res = {}
    with cf.ProcessPoolExecutor(workers) as ex:
        for r in ex.map(run, order):
            res[r["job"]] = r
            print("job", r["job"], r["name"], r.get("oracle_seconds"), flush=True)
    out = {"n_jobs": N_JOBS, "min_nodes": MIN_NODES, "max_nodes": MAX_NODES, "seed": SEED,
           "jobs": [res[i] for i in range(N_JOBS)]}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "job_stream_256.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 6)
