"""Writes tests/golden/refine_rep.json from the oracle alone.

For each full-size case of tests/_refine_cases.py, runs single refinement
repetitions (Sec. VI) of the serial oracle on a seeded partition and stores
SHA-256 digests of every node's in-isolation move and gain, the sequence,
its destinations, the in-sequence gains, C_k, V_k and the partition after
the applied prefix, plus the counts.  Usage:
    python tests/golden/make_refine_golden.py
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
from tests import _refine_cases as RC  # noqa: E402


def digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def main():
    out = {}
    for name in RC.FULL:
        hg, rho, nparts, delta, reps = RC.full_case(name)
        g = oracle.Graph(hg)
        runs = []
        for rep, omega in reps:
            t0 = time.time()
            dst, gain = g.moves(rho, nparts, rep, 16, omega)
            new_rho, d = g.refine_rep(rho, nparts, rep, 16, omega, delta)
            dt = time.time() - t0
            runs.append({"rep": rep, "omega": omega, "moves": d["M"], "kstar": d["kstar"],
                         "gain": d["applied_gain"], "links": d["links"],
                         "move_dst": digest(dst.astype(np.int32)), "move_gain": digest(gain.astype(np.int64)),
                         "seq": digest(d["seq"].astype(np.int32)), "seq_pd": digest(d["seq_pd"].astype(np.int32)),
                         "gseq": digest(d["gseq"].astype(np.int64)), "C": digest(d["C"].astype(np.int64)),
                         "V": digest(d["V"].astype(np.int64)), "rho": digest(new_rho.astype(np.int32)),
                         "oracle_seconds": round(dt, 1)})
            print(name, runs[-1], flush=True)
        out[name] = {"nodes": hg.n_nodes, "pins": hg.n_pins, "nparts": nparts, "delta": delta, "runs": runs}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "refine_rep.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
