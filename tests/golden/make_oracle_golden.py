"""Writes tests/golden/<workload>.json from the oracle alone.

Runs the serial oracle on a seeded synthetic workload and stores what the GPU
parity test at full size compares against: the hierarchy sizes, SHA-256
digests of every level's candidates, scores, matching and cluster map, of the
final partition, and the connectivity.  Usage:
    python tests/golden/make_oracle_golden.py rand-64k-e192
(The 65,536-node workload takes about half an hour on one core.)
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2605_20497_amd import workloads as W  # noqa: E402


def digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def main(name: str, Pi: int = 4, theta: int = 16, seed: int = 0):
    hg = W.WORKLOADS[name]()
    g = oracle.Graph(hg)
    t0 = time.time()
    res = g.partition(hg.omega, hg.delta, k=hg.k, Pi=Pi, theta=theta, seed=seed)
    dt = time.time() - t0
    out = {
        "workload": name, "omega": hg.omega, "delta": hg.delta, "k": hg.k, "pi": Pi, "theta": theta,
        "seed": seed, "nlevels": res.nlevels, "nparts": res.nparts, "conn": res.conn,
        "levels": [{"N": L["N"], "E": L["E"], "P": L["P"]} for L in res.levels],
        "proposal": [], "gamma": [],
        "rho_sha256": digest(res.rho(0)),
        "oracle_seconds": round(dt, 1),
    }
    for lv in range(res.ncoarsened):
        cand, score, match = res.proposal(lv)
        out["proposal"].append({"cand": digest(cand), "score": digest(score), "match": digest(match)})
    for lv in range(res.nlevels - 1):
        out["gamma"].append(digest(res.gamma(lv)))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), name + ".json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, "in %.0f s" % dt)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "rand-64k-e192")
