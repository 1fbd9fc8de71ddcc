"""Benchmark of the partitioner's hot path on one MI355X.

One step = one complete partitioning of the synthetic conv-shaped SNN
hypergraph, the largest single-GPU workload: 7 layers of 176 x 176 x 32
neurons (6,938,624 nodes), one h-edge per neuron (source + Poisson(82)
destinations in the 3 x 3 spatial window of the next layer, 575,857,446 pins),
Omega = 2^12, Delta = 2^16.  The step loads from HBM-resident tensors
(on-device validation and incidence build), coarsens every level and refines
every level with Theta = 16 repetitions.  --workload selects another of the
five workloads.

Prints one JSON line: pins/s of the whole step (input pins / step time), the
rooflines of the largest kernels from HIP events over the timed steps
(`roofline` is the one that takes the most time), the per-family breakdown and
per-level figures (pins/s, and GB/s and HBM fraction of the streaming sweeps
from their device-counted algorithmic bytes) from one extra profiled step, the
batched job-stream leg, and the serial oracle's rate on a bounded sample of
the same workload family as the CPU baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# The histogram updates of the proposal and gains sweeps are 32-bit LDS atomic
# adds.  A CU's LDS takes one 64-lane atomic instruction every 4 clocks (16
# lane updates per clock; a conflict-free probe measured 15.2), so 256 CUs at
# 2.4 GHz give 16 * 256 * 2.4 G = 9,830 G updates/s.
LDS_UPDATE_PEAK_GOPS = 16 * 256 * 2.4
# Dense int8 MFMA peak of MI355X (no sparsity), in TOP/s.
INT8_PEAK_TOPS = 5000.0

# Measured HBM traffic per launch on the bench workload, from rocprofv3
# FETCH_SIZE and WRITE_SIZE runs (scaled by what the counters read for a plain
# 256 MiB copy), valid only for the kernel sources they were taken on (sha256
# over each kernel's files below); otherwise traffic is reported as null.
_CSRC = "paper_2605_20497_amd/csrc/"
TRAFFIC_SOURCES = {
    "k_propose": [_CSRC + f for f in ("k_coarsen.hip", "top_select.h", "dev_util.h", "hgp_internal.h")],
    "k_gains16": [_CSRC + f for f in ("k_refine.hip", "scan_lb.h", "dev_util.h", "hgp_internal.h")],
    "k_dense_gemm": [_CSRC + f for f in ("k_dense.hip", "top_select.h", "dev_util.h", "hgp_internal.h")],
    "k_conn_gemm": [_CSRC + f for f in ("k_dense.hip", "top_select.h", "dev_util.h", "hgp_internal.h")],
}
TRAFFIC = {  # {(kernel, sources_sha256): bytes per launch}
    # conv-6.9m, profiles/hbm_counters_conv-6.9m.txt (family averages)
    ("k_propose", "ceba8c1d7c5e9987da1de801fab8d003ec1ebc123fc0ae3e26161dcd2f117bd4"): 16569862888,
    ("k_gains16", "b1669d7b1659b8e798f5e16d669674602c40e91f0ae9c14ed998c7fbd72b872f"): 4293562929,
}


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="conv-6.9m")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU-baseline leg")
    ap.add_argument("--cpu-hw", type=int, default=16,
                    help="grid side of the CPU baseline's conv-shaped sample (7 layers x hw x hw x 32)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (counter calibration)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-plain job stream leg")
    ap.add_argument("--batch-jobs", type=int, default=256)
    ap.add_argument("--batch-workers", type=int, default=0,
                    help="concurrent contexts of the batched leg (0 = the autotuned count, else 8)")
    ap.add_argument("--batch-max-nodes", type=int, default=262144)
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the step: Pi and Theta sweeps and the chain-free ablation on --sweep-workload")
    ap.add_argument("--sweep-workload", default="layered-256k-e256")
    return ap.parse_args()


def sources_sha256(kernel):
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES[kernel]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic(kernel):
    return TRAFFIC.get((kernel, sources_sha256(kernel)))


def algorithmic_bytes(kernel, levels, pi):
    """Compulsory HBM bytes per launch family summed over one step, from the
    level sizes (N, E, P) of the hierarchy.  Ids 4 B, offsets 8 B."""
    tot = 0
    for (N, E, P, _pairs) in levels:
        if kernel == "propose":
            # incidence (inc, inc_off, inc_nin) + h-edge CSR (he_off, he_nsrc, pins, w)
            # + node sizes + candidates/scores written
            tot += 4 * P + 8 * (N + 1) + 4 * N + 8 * (E + 1) + 4 * E + 4 * P + 4 * E + 4 * N + 12 * pi * N
    return tot


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args, hg_full):
    """Serial oracle (one pinned host core), full coarsen + refine on a bounded
    sample of the timed workload's family: the conv-shaped generator on a
    smaller grid (7 layers of cpu_hw x cpu_hw x 32, the same fan-out and
    Delta, Omega scaled by the node ratio with a floor of 64), or for the
    random workload a 4,096-node random hypergraph of the same h-edge size.
    Rate = input pins / wall time.  Beside it: the oracle's own time on the
    full workload, recorded when the stored digests were written."""
    import oracle
    from paper_2605_20497_amd import workloads as W
    core = None
    if hasattr(os, "sched_setaffinity"):
        avail = sorted(os.sched_getaffinity(0))
        core = avail[2] if len(avail) > 2 else avail[0]
        os.sched_setaffinity(0, {core})
    if args.workload.startswith("rand-64k"):
        n = 4096
        omega = max(64, hg_full.omega * n // hg_full.n_nodes)
        hg = W.random_snn(n, 191, seed=0, omega=omega, delta=hg_full.delta)
        sample = "rand-4096-e192 (4,096 nodes, h-edges of 192 pins)"
    else:
        hw = args.cpu_hw
        n = 7 * hw * hw * 32
        omega = max(64, (1 << 12) * n // 6938624)
        hg = W.conv_snn(7, hw, 32, 82.0, seed=0, omega=omega, delta=1 << 16)
        sample = "conv-shaped 7 x %d x %d x 32 (%d nodes)" % (hw, hw, n)
    g = oracle.Graph(hg)
    t0 = time.perf_counter()
    res = g.partition(hg.omega, hg.delta)
    dt = time.perf_counter() - t0
    out = {"value": hg.n_pins / dt, "unit": "pins/s", "cores": 1, "kind": "oracle",
           "sample": "%s, %d pins, Omega=%d, Delta=%d, full coarsen+refine, %d levels, %.1f s"
                     % (sample, hg.n_pins, hg.omega, hg.delta, res.nlevels, dt),
           "cpu_model": _cpu_model(), "nproc": os.cpu_count(), "pinned_core": core,
           "threads_used": 1}
    gold = os.path.join(ROOT, "tests", "golden", args.workload + ".json")
    if os.path.exists(gold):
        with open(gold) as f:
            sec = json.load(f).get("oracle_seconds")
        if sec:
            out["full_workload_oracle"] = {
                "seconds": sec, "pins_per_s": round(hg_full.n_pins / sec, 1),
                "note": "one core of the build container when the stored digests were written"}
    return out


# Families whose kernels count their own algorithmic bytes when profiled.
STREAM_FAMILIES = ("phi", "part_stats", "inseq", "contract_edges", "pack")


def batched_leg(args):
    """Job stream (batch_jobs jobs, 256 by default, of the five workload
    families, log-uniform 2,048 to batch_max_nodes nodes, job i seeded with
    i): the plain one-at-a-time rate
    with every job waiting from the start, the batched rate the same way, then
    Poisson arrivals (seed 12,345) at 1.5x the plain rate served by one worker
    (plain) and by batch_workers concurrent workers (batched).  Latency =
    arrival to partition on the host.  Every job's partition is compared
    between the plain and batched runs, and with the oracle's digest where
    tests/golden holds one for this stream."""
    import hashlib

    import numpy as np
    import paper_2605_20497_amd as pkg
    from paper_2605_20497_amd import workloads as W
    t0 = time.perf_counter()
    jobs, _ = W.job_stream(args.batch_jobs, 2048, args.batch_max_nodes, seed=0)
    gen_s = time.perf_counter() - t0
    print("bench: %d jobs generated in %.1f s" % (len(jobs), gen_s), file=sys.stderr, flush=True)
    pkg.hgp_run_jobs(jobs[:4], workers=1)  # warm-up
    closed = pkg.hgp_run_jobs(jobs, workers=1)
    span = max(r["end_s"] for r in closed)
    rate = 1.5 * len(jobs) / span
    arng = np.random.default_rng(12345)
    arrivals = np.cumsum(arng.exponential(1.0 / rate, size=len(jobs)))

    def summary(res, workers):
        lat = np.array([r["end_s"] - a for r, a in zip(res, arrivals)])
        end = max(r["end_s"] for r in res)
        return {"workers": workers, "jobs_per_s": round(len(res) / (end - arrivals[0]), 2),
                "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
                "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2)}

    if args.batch_workers <= 0:
        from paper_2605_20497_amd import autotune
        args.batch_workers = autotune.tuned_options(autotune.stream_key(len(jobs), args.batch_max_nodes))["workers"]
    closed_b = pkg.hgp_run_jobs(jobs, workers=args.batch_workers)
    span_b = max(r["end_s"] for r in closed_b)
    print("bench: closed-loop runs done", file=sys.stderr, flush=True)
    plain = pkg.hgp_run_jobs(jobs, workers=1, arrivals=arrivals)
    batched = pkg.hgp_run_jobs(jobs, workers=args.batch_workers, arrivals=arrivals)
    runs = {"plain_closed": closed, "batched_closed": closed_b, "plain": plain, "batched": batched}
    status = {k: {str(s): int(c) for s, c in zip(*np.unique([r["status"] for r in v], return_counts=True))}
              for k, v in runs.items()}
    differ = [jobs[i].name for i in range(len(jobs))
              if not all(runs[k][i]["status"] == 0 and np.array_equal(closed[i]["rho"], runs[k][i]["rho"])
                         for k in runs)]
    ok = not differ
    out = {"jobs": len(jobs), "pins": int(sum(j.n_pins for j in jobs)),
           "sizes": "2048-%d nodes, random e32/e192, layered, conv, netlist" % args.batch_max_nodes,
           "generation_s": round(gen_s, 1),
           "plain_closed_jobs_per_s": round(len(jobs) / span, 2),
           "batched_closed_jobs_per_s": round(len(jobs) / span_b, 2), "arrival_rate_per_s": round(rate, 2),
           "plain": summary(plain, 1), "batched": summary(batched, args.batch_workers),
           "status_counts": status,
           "reruns": {k: int(sum(r["reruns"] for r in v)) for k, v in runs.items()},
           "bit_exact_vs_plain": bool(ok), "differing_jobs": differ[:16]}
    gold = os.path.join(ROOT, "tests", "golden", "job_stream_%d.json" % len(jobs))
    if os.path.exists(gold):
        with open(gold) as f:
            g = json.load(f)
        if (g["n_jobs"], g["min_nodes"], g["max_nodes"], g["seed"]) == (len(jobs), 2048, args.batch_max_nodes, 0):
            checked = matched = 0
            for gj, b in zip(g["jobs"], batched):
                if "rho_sha256" not in gj:
                    continue
                checked += 1
                rho = np.ascontiguousarray(b["rho"], np.int32)
                matched += int(hashlib.sha256(rho.tobytes()).hexdigest() == gj["rho_sha256"])
            out["oracle_checked_jobs"] = checked
            out["oracle_matching_jobs"] = matched
    return out


def sweep(args):
    """Parameter sweeps of the method on one workload: Pi (candidates and
    matching rounds) at Theta = 16, Theta (repetitions per level) at Pi = 4,
    the ablation without chain rounds (moves sequenced by gain alone) and the
    one with the prototype's greedy matching.  Per setting: the partition's
    connectivity and violations, the hierarchy depth and the wall time of one
    partitioning (after one untimed run)."""
    import torch

    import paper_2605_20497_amd as pkg
    from paper_2605_20497_amd import workloads as W

    hg = W.WORKLOADS[args.sweep_workload]()
    torch.cuda.set_device(0)

    def run(pi, theta, no_chains=False, greedy=False):
        g = pkg.Partitioner(device=0, pi=pi, theta=theta, no_chains=no_chains, greedy_matching=greedy)
        out = {"pi": pi, "theta": theta, "chains": not no_chains, "matching": "greedy" if greedy else "exact"}
        try:
            for rep in range(2):
                g.load(hg)
                g.hgp_set_limits(hg.omega, hg.delta, hg.k)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                nl = g.hgp_coarsen()
                g.hgp_refine()
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                ev = g.hgp_evaluate()
                out.update(conn=int(ev["conn"]), violations=int(ev["violations"]), parts=int(ev["n_parts"]),
                           levels=int(nl), ms=round(dt * 1e3, 2))
        except pkg.HgpError as e:
            # a setting whose hierarchy outgrows device memory is a result of the sweep, not a crash of it
            import ctypes
            import numpy as np
            lv = np.zeros(4 * 4096, np.int64)
            pkg.lib().hgp_get_levels(g.h, lv.ctypes.data_as(ctypes.c_void_p), lv.size)
            lv = lv.reshape(-1, 4)
            lv = lv[lv[:, 0] > 0]
            out.update(error=str(e), levels_built=len(lv), nodes_last_level=int(lv[-1, 0]) if len(lv) else None,
                       pins_last_level=int(lv[-1, 2]) if len(lv) else None)
        g.close()
        torch.cuda.empty_cache()
        print(json.dumps(out), file=sys.stderr, flush=True)
        return out

    rows = [run(pi, 16) for pi in (1, 2, 3, 4, 6, 8)]
    rows += [run(4, th) for th in (0, 1, 2, 4, 8, 32, 64)]
    rows.append(run(4, 16, no_chains=True))
    rows.append(run(4, 16, greedy=True))
    print(json.dumps({"sweep": args.sweep_workload, "nodes": hg.n_nodes, "pins": hg.n_pins,
                      "omega": hg.omega, "delta": hg.delta, "rows": rows}))


def _roofline_entry(kernel, bound, achieved, peak, unit, traffic_bytes, **extra):
    out = {"kernel": kernel, "bound": bound, "achieved": round(achieved, 2), "peak": peak, "unit": unit,
           "frac": round(achieved / peak, 5), "traffic": traffic_bytes}
    out.update(extra)
    return out


def main():
    args = _args()
    if args.gpus != 1:
        print("bench.py: the partitioner runs on one GPU; --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.sweep:
        sweep(args)
        return
    import numpy as np
    import torch

    import paper_2605_20497_amd as pkg
    from paper_2605_20497_amd import workloads as W

    hg = W.WORKLOADS[args.workload]()
    print("bench: %s generated, %d nodes, %d pins" % (args.workload, hg.n_nodes, hg.n_pins), file=sys.stderr,
          flush=True)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t_he_off = torch.from_numpy(hg.he_off).to(dev)
    t_nsrc = torch.from_numpy(hg.he_nsrc).to(dev)
    t_pins = torch.from_numpy(hg.pins).to(dev)
    t_hw = torch.from_numpy(hg.hedge_w).to(dev)
    t_nw = torch.from_numpy(hg.node_w).to(dev)
    torch.cuda.synchronize()

    if args.calib_copy_mib:
        src = torch.empty(args.calib_copy_mib << 18, dtype=torch.int32, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # Timed steps record HIP events only around the roofline kernels
    # (proposal histogram, gains sweep, the two dense GEMMs) and count the
    # gains' row reads on the device (one atomic per wave); recording events
    # around every launch would add about a sixth to a step.  One extra step
    # after the timed region records every family for the breakdown.
    # tile and schedule choices from the autotuner's cache (defaults without one)
    from paper_2605_20497_amd import autotune
    tune = autotune.tuned_options(args.workload)
    part = pkg.Partitioner(device=0, profile=True, profile_families=("propose", "gains", "dense_gemm", "gains_gemm"),
                           tune=tune)

    def step():
        part.hgp_load_csr_device(hg.n_nodes, t_he_off, t_nsrc, t_pins, t_hw, t_nw)
        part.hgp_set_limits(hg.omega, hg.delta, hg.k)
        part.hgp_coarsen()
        part.hgp_refine()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    part.hgp_reset_kernel_stats()
    level_times = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        level_times.append(part.hgp_level_times())
        print("bench: step %d of %d done" % (i + 1, args.steps), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    stats_timed = part.hgp_kernel_stats()
    work_timed = part.hgp_kernel_work()
    levels = part.hgp_get_levels()
    ev = part.hgp_evaluate()
    card_lv = []
    for lv in range(int(levels.shape[0])):
        he_off = part.hgp_get_level_graph(lv, what=("he_off",))[0]
        card_lv.append(np.diff(he_off).astype(np.int64))
    part.close()

    full = pkg.Partitioner(device=0, profile=True, tune=tune)
    full.hgp_load_csr_device(hg.n_nodes, t_he_off, t_nsrc, t_pins, t_hw, t_nw)
    full.hgp_set_limits(hg.omega, hg.delta, hg.k)
    full.hgp_coarsen()
    full.hgp_refine()
    torch.cuda.synchronize()
    stats = full.hgp_kernel_stats()
    lstats = full.hgp_kernel_level_stats()
    full.close()
    lt = np.median(np.stack(level_times), axis=0)

    # Per level: pins/s of the timed steps, and per streaming family of the
    # profiled step its time, device-counted algorithmic bytes, GB/s and HBM
    # fraction.
    per_level = []
    stream_tot = {f: [0, 0] for f in STREAM_FAMILIES}
    for lv, (N, E, P, pairs) in enumerate(levels.tolist()):
        tc, tr = lt[lv] * 1e-9
        row = {"level": lv, "nodes": N, "pins": P, "coarsen_ms": round(tc * 1e3, 3), "refine_ms": round(tr * 1e3, 3),
               "pins_per_s": (P / (tc + tr)) if tc + tr > 0 else None, "streams": {}}
        for f in STREAM_FAMILIES:
            a = lstats[f][lv] if lv < lstats[f].shape[0] else (0, 0, 0)
            launches, ns, nbytes = int(a[0]), int(a[1]), int(a[2])
            if launches == 0 or ns == 0:
                continue
            gbs = nbytes / ns
            stream_tot[f][0] += ns
            stream_tot[f][1] += nbytes
            row["streams"][f] = {"launches": launches, "ms": round(ns * 1e-6, 3), "bytes": nbytes,
                                 "gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
        per_level.append(row)
    streams = {f: {"ms_per_step": round(ns * 1e-6, 3), "bytes_per_step": nb,
                   "gbs": round(nb / ns, 1) if ns else None,
                   "hbm_frac": round(nb / ns / HBM_PEAK_GBS, 4) if ns else None}
               for f, (ns, nb) in stream_tot.items() if ns}
    # per-family breakdown from the separate fully profiled step
    fam = {k: v for k, v in stats.items() if v[0] > 0}
    total_ns = sum(v[1] for v in fam.values())
    dom = max(fam, key=lambda k: fam[k][1])
    breakdown = {k: {"launches": v[0], "ms_per_step": round(v[1] * 1e-6, 3)}
                 for k, v in sorted(fam.items(), key=lambda kv: -kv[1][1])}

    # Rooflines of the largest kernels, from HIP events over the timed steps;
    # `roofline` is the one that takes the most time per step.
    roofs = {}
    prop = stats_timed.get("propose")
    n_prop = int(round(prop[0] / args.steps)) if prop else 0
    hist_levels = [lv for lv in range(len(card_lv)) if lv < n_prop]
    upd_all = [int((c * (c - 1)).sum()) for c in card_lv]
    if prop and prop[0] > 0:
        # One launch per level on the histogram path (the first n_prop levels):
        # its work is one histogram update per (node, incident h-edge, other
        # pin), sum_e |e| (|e| - 1), a 32-bit LDS atomic add (the hashed
        # table's update adds a probe).
        t_launch = prop[1] / prop[0] * 1e-9
        upd = sum(upd_all[lv] for lv in hist_levels) / max(n_prop, 1)
        nbytes = algorithmic_bytes("propose", levels.tolist()[:n_prop], part.pi) / max(n_prop, 1)
        roofs["k_propose"] = _roofline_entry(
            "k_propose", "alu", upd / t_launch / 1e9, LDS_UPDATE_PEAK_GOPS, "Gop/s", traffic("k_propose"),
            op="histogram update (32-bit LDS atomic add)", ops_per_launch=int(upd),
            avg_launch_ms=round(t_launch * 1e3, 4), ms_per_step=round(prop[1] * 1e-6 / args.steps, 3),
            hbm_compulsory_bytes_per_launch=int(nbytes), hbm_compulsory_gbs=round(nbytes / t_launch / 1e9, 2),
            hbm_frac=round(nbytes / t_launch / 1e9 / HBM_PEAK_GBS, 5))
    gn = stats_timed.get("gains")
    if gn and gn[0] > 0 and work_timed.get("gains", 0) > 0:
        # Phi row entries read (counted on the device): one bin update each,
        # 2 bytes each from the 16-bit row copy.
        t_launch = gn[1] / gn[0] * 1e-9
        visits = work_timed["gains"] / gn[0]
        roofs["k_gains16"] = _roofline_entry(
            "k_gains16", "alu", visits / t_launch / 1e9, LDS_UPDATE_PEAK_GOPS, "Gop/s", traffic("k_gains16"),
            op="row entry read + bin update (32-bit LDS atomic add)", ops_per_launch=int(visits),
            avg_launch_ms=round(t_launch * 1e3, 4), ms_per_step=round(gn[1] * 1e-6 / args.steps, 3),
            row_bytes_gbs=round(2 * visits / t_launch / 1e9, 2))
    dg = stats_timed.get("dense_gemm")
    if dg and dg[0] > 0:
        # The dense proposal computes the same histograms as int8 products on
        # small levels.  Its work is counted as the method's histogram updates
        # of those levels, against the same peak; the MFMA rate of the padded
        # products it issues is reported beside it.
        t_launch = dg[1] / dg[0] * 1e-9
        dense_lv = [lv for lv in range(len(card_lv)) if lv >= n_prop][:int(round(dg[0] / args.steps))]
        upd = sum(upd_all[lv] for lv in dense_lv) / max(len(dense_lv), 1)
        macs = work_timed.get("dense_gemm", 0) / dg[0]
        roofs["k_dense_gemm"] = _roofline_entry(
            "k_dense_gemm", "alu", upd / t_launch / 1e9, LDS_UPDATE_PEAK_GOPS, "Gop/s", traffic("k_dense_gemm"),
            op="histogram update of the method, computed as int8 MFMA products", ops_per_launch=int(upd),
            avg_launch_ms=round(t_launch * 1e3, 4), ms_per_step=round(dg[1] * 1e-6 / args.steps, 3),
            mfma_tops=round(2 * macs / t_launch / 1e12, 2),
            mfma_frac=round(2 * macs / t_launch / 1e12 / INT8_PEAK_TOPS, 4))
    gg = stats_timed.get("gains_gemm")
    if gg and gg[0] > 0:
        t_launch = gg[1] / gg[0] * 1e-9
        macs = work_timed.get("gains_gemm", 0) / gg[0]
        roofs["k_conn_gemm"] = _roofline_entry(
            "k_conn_gemm", "mfma", 2 * macs / t_launch / 1e12, INT8_PEAK_TOPS, "TOP/s", traffic("k_conn_gemm"),
            op="int8 MAC = 2 ops of the padded product (v_mfma_i32_32x32x32_i8)", ops_per_launch=int(2 * macs),
            avg_launch_ms=round(t_launch * 1e3, 4), ms_per_step=round(gg[1] * 1e-6 / args.steps, 3))
    roof = max(roofs.values(), key=lambda r: r["ms_per_step"]) if roofs else None

    out = {
        "metric": "pins/s per coarsen+refine level & % HBM peak; batched vs plain jobs/s, p50/p99",
        "value": hg.n_pins / dt, "unit": "pins/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": args.workload, "nodes": hg.n_nodes, "hedges": hg.n_hedges, "pins": hg.n_pins,
                   "omega": hg.omega, "delta": hg.delta, "pi": part.pi, "theta": part.theta,
                   "levels": int(levels.shape[0]), "partitions": int(ev["n_parts"]), "conn": int(ev["conn"]),
                   "violations": int(ev["violations"])},
        "roofline": roof,
        "rooflines": list(roofs.values()),
        "tuning": {k: tune[k] for k in ("hash_log2", "list_gate")},
        "tuning_device": autotune.device_name(),
        "streams": streams,
        "levels": per_level,
        "kernels": breakdown,
        "dominant_kernel": dom,
        "kernel_time_share": round(total_ns * 1e-9 / dt, 4) if dt > 0 else None,
        "kernels_note": "per-family times, per-level stream figures from one extra fully profiled step; the "
                        "timed steps record events around the roofline kernels only",
    }
    if not args.no_batch:
        print("bench: batched job-stream leg", file=sys.stderr, flush=True)
        out["batched"] = batched_leg(args)
    if not args.no_cpu:
        print("bench: CPU baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args, hg)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
