"""Autotuner of the library's tile and schedule choices, with a JSON cache.

The choices never change results (the method is deterministic and every
variant computes the same integers); they change time only:
  - hash_log2:  log2 of the hashed proposal's table slots (10..13).  Smaller
                tables let more blocks share a CU; larger ones need fewer
                passes over a node's pins when its neighbourhood is large.
  - list_gate:  repetitions list the h-edges of their movers instead of
                sweeping all h-edges while movers * list_gate < nodes.
  - workers:    concurrent contexts (streams) of the batched job runner.

tune_partition() times one partitioning per candidate on a workload (after an
untimed run of the same candidate) and keeps the fastest; tune_workers() times
the closed-loop job stream for each worker count.  Results go to a JSON cache
keyed by device name and workload; tuned_options() reads it back.
"""
from __future__ import annotations

import json
import os
import time

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")
DEFAULT = {"hash_log2": 12, "list_gate": 4, "workers": 8}
HASH_LOG2 = (11, 12, 13)
LIST_GATE = (2, 4, 8, 16)
WORKERS = (2, 4, 8, 12, 16)


def device_name(device: int = 0) -> str:
    """Marketing name and ISA of the device, e.g. 'AMD Radeon Graphics (gfx950)'."""
    import torch
    arch = getattr(torch.cuda.get_device_properties(device), "gcnArchName", "").split(":")[0]
    name = torch.cuda.get_device_name(device)
    return "%s (%s)" % (name, arch) if arch else name


def load(path: str = CACHE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def save(cache: dict, path: str = CACHE) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _device_entry(cache: dict, name: str) -> dict:
    """The cache's entry for this device name; failing that, one for the same
    ISA (the marketing name the runtime reports can differ between processes
    on one machine, e.g. with and without a profiler's library loaded)."""
    if name in cache:
        return cache[name]
    i = name.rfind(" (")
    if i >= 0 and name.endswith(")"):
        isa = name[i:]
        for key in sorted(cache):
            if key.endswith(isa):
                return cache[key]
    return {}


def tuned_options(workload: str, device: int = 0, path: str = CACHE, name: str | None = None) -> dict:
    """Choices cached for (device, workload), else the defaults."""
    entry = _device_entry(load(path), name or device_name(device)).get(workload, {})
    out = dict(DEFAULT)
    out.update({k: v for k, v in entry.items() if k in DEFAULT})
    return out


def _time_partition(hg, tune, device):
    import torch

    import paper_2605_20497_amd as pkg
    part = pkg.Partitioner(device=device, tune=tune)
    best = None
    for rep in range(2):  # the first run warms the allocator and the code objects
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        part.partition(hg)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if rep > 0:
            best = dt
    part.close()
    return best


def tune_partition(workload: str, device: int = 0, path: str = CACHE, log=print) -> dict:
    """Coordinate search over hash_log2, then list_gate, on one workload."""
    from paper_2605_20497_amd import workloads as W
    hg = W.WORKLOADS[workload]()
    cur = {"hash_log2": DEFAULT["hash_log2"], "list_gate": DEFAULT["list_gate"]}
    timings = {}
    for key, values in (("hash_log2", HASH_LOG2), ("list_gate", LIST_GATE)):
        best_v, best_t = cur[key], None
        for v in values:
            trial = dict(cur, **{key: v})
            t = _time_partition(hg, trial, device)
            timings["%s=%d %s=%d" % ("hash_log2", trial["hash_log2"], "list_gate", trial["list_gate"])] = round(
                t * 1e3, 2)
            log("tune %s %s: %.1f ms" % (workload, trial, t * 1e3))
            if best_t is None or t < best_t:
                best_v, best_t = v, t
        cur[key] = best_v
    cache = load(path)
    entry = cache.setdefault(device_name(device), {}).setdefault(workload, {})
    entry.update(cur)
    entry["ms"] = timings
    save(cache, path)
    return cur


def stream_key(n_jobs: int, max_nodes: int) -> str:
    """Cache key of a job stream of n_jobs jobs of 2,048 to max_nodes nodes."""
    return "job-stream-%d-%d" % (n_jobs, max_nodes)


def tune_workers(n_jobs: int = 256, max_nodes: int = 262144, device: int = 0, path: str = CACHE,
                 log=print) -> int:
    """Closed-loop jobs/s of the job stream for each worker count."""
    import paper_2605_20497_amd as pkg
    from paper_2605_20497_amd import workloads as W
    jobs, _ = W.job_stream(n_jobs, 2048, max_nodes, seed=0)
    pkg.hgp_run_jobs(jobs[:4], workers=1, device=device)
    rates = {}
    for w in WORKERS:
        res = pkg.hgp_run_jobs(jobs, workers=w, device=device)
        rates[w] = len(jobs) / max(r["end_s"] for r in res)
        log("tune workers=%d: %.2f jobs/s" % (w, rates[w]))
    best = max(rates, key=rates.get)
    cache = load(path)
    entry = cache.setdefault(device_name(device), {}).setdefault(stream_key(n_jobs, max_nodes), {})
    entry["workers"] = best
    entry["jobs_per_s"] = {str(k): round(v, 2) for k, v in rates.items()}
    save(cache, path)
    return best


if __name__ == "__main__":
    import sys
    what = sys.argv[1] if len(sys.argv) > 1 else "conv-6.9m"
    if what == "workers":
        tune_workers()
    else:
        tune_partition(what)
