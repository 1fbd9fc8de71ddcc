"""Benchmark of the partitioner's hot path on one MI355X.

One step = one complete partitioning of the synthetic 65,536-node random
SNN-shaped hypergraph (one h-edge per node: source + 191 distinct uniform
destinations, 12,582,912 pins, Omega = 2^10, Delta = 2^12): load from
HBM-resident tensors (on-device validation and incidence build), every
coarsening level, and refinement of every level with Theta = 16 repetitions.

Prints one JSON line: pins/s of the whole step (input pins / step time), the
per-level pins/s, the rooflines of the largest kernels from HIP events
over the timed steps (`roofline` is the one that takes the most time), the
per-family breakdown, the batched job-stream leg, and the serial oracle's rate
on a bounded sample of the same workload family as the CPU baseline.
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
# The proposal kernel's histogram updates are 32-bit integer adds executed by
# the LDS: at most one per bank per clock, 32 banks per CU, 256 CUs at 2.4 GHz.
LDS_UPDATE_PEAK_GOPS = 256 * 32 * 2.4
# Dense int8 MFMA peak of MI355X (no sparsity), in TOP/s.
INT8_PEAK_TOPS = 5000.0

# Measured HBM traffic per launch on the bench workload, from rocprofv3
# FETCH_SIZE and WRITE_SIZE runs (scaled by what the counters read for a plain
# 256 MiB copy), valid only for the kernel sources they were taken on (sha256
# over each kernel's files below); otherwise traffic is reported as null.
_CSRC = "paper_2605_20497_amd/csrc/"
TRAFFIC_SOURCES = {
    "k_propose": [_CSRC + f for f in ("k_coarsen.hip", "top_select.h", "dev_util.h", "hgp_internal.h")],
    "k_gains16": [_CSRC + f for f in ("k_refine.hip", "dev_util.h", "hgp_internal.h")],
    "k_dense_gemm": [_CSRC + f for f in ("k_dense.hip", "top_select.h", "dev_util.h", "hgp_internal.h")],
    "k_conn_gemm": [_CSRC + f for f in ("k_dense.hip", "top_select.h", "dev_util.h", "hgp_internal.h")],
}
TRAFFIC = {  # {(kernel, sources_sha256): bytes per launch}
    ("k_propose", "d67cc2b673d2efe632ec33285bccf0026b910079dcb412744d199253a4567321"): 6492284725,
    ("k_gains16", "9add569fcb1bf581861266e7849e1af19a3f3d782b5d58384d9954aa51b6b435"): 5173471137,
    ("k_dense_gemm", "7650765301f3707763fbf1a94aa603699eb4970c383675851ebedd006ab0ec68"): 1777133399,
    ("k_conn_gemm", "7650765301f3707763fbf1a94aa603699eb4970c383675851ebedd006ab0ec68"): 556130590,
}


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rand-64k-e192")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU-baseline leg")
    ap.add_argument("--cpu-nodes", type=int, default=4096)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (counter calibration)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-plain job stream leg")
    ap.add_argument("--batch-jobs", type=int, default=64)
    ap.add_argument("--batch-workers", type=int, default=8)
    ap.add_argument("--batch-max-nodes", type=int, default=32768)
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the step: Pi and Theta sweeps and the chain-free ablation on --sweep-workload")
    ap.add_argument("--sweep-workload", default="rand-64k-e192")
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


def cpu_baseline(args):
    """Serial oracle (one host core), full coarsen + refine on a bounded
    sample of the workload family: a random SNN-shaped hypergraph with the
    same h-edge size 192 and the same Delta, on cpu_nodes nodes, Omega scaled
    by the node ratio.  Rate = input pins / wall time."""
    import oracle
    from paper_2605_20497_amd import workloads as W
    n = args.cpu_nodes
    omega = max(16, (1 << 10) * n // 65536)
    hg = W.random_snn(n, 191, seed=0)
    g = oracle.Graph(hg)
    t0 = time.perf_counter()
    res = g.partition(omega, 1 << 12)
    dt = time.perf_counter() - t0
    return {"value": hg.n_pins / dt, "unit": "pins/s", "cores": 1, "kind": "oracle",
            "sample": "rand-%d-e192 (%d nodes, %d pins, Omega=%d, Delta=4096), full coarsen+refine, %d levels, "
                      "%.1f s on one host core" % (n, n, hg.n_pins, omega, res.nlevels, dt)}


def batched_leg(args):
    """Job stream (the five workload families, log-uniform 2,048 to
    batch_max_nodes nodes): the plain one-at-a-time rate with every job
    waiting from the start, then Poisson arrivals at 1.5x that rate served
    by one worker (plain) and by batch_workers concurrent workers (batched).
    Latency = arrival to partition on the host."""
    import numpy as np
    import paper_2605_20497_amd as pkg
    from paper_2605_20497_amd import workloads as W
    jobs, _ = W.job_stream(args.batch_jobs, 2048, args.batch_max_nodes, seed=0)
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

    closed_b = pkg.hgp_run_jobs(jobs, workers=args.batch_workers)
    span_b = max(r["end_s"] for r in closed_b)
    plain = pkg.hgp_run_jobs(jobs, workers=1, arrivals=arrivals)
    batched = pkg.hgp_run_jobs(jobs, workers=args.batch_workers, arrivals=arrivals)
    ok = all(p["status"] == 0 and b["status"] == 0 and np.array_equal(p["rho"], b["rho"])
             for p, b in zip(plain, batched))
    return {"jobs": len(jobs), "pins": int(sum(j.n_pins for j in jobs)),
            "sizes": "2048-%d nodes, random e32/e192, layered, conv, netlist" % args.batch_max_nodes,
            "plain_closed_jobs_per_s": round(len(jobs) / span, 2),
            "batched_closed_jobs_per_s": round(len(jobs) / span_b, 2), "arrival_rate_per_s": round(rate, 2),
            "plain": summary(plain, 1), "batched": summary(batched, args.batch_workers),
            "bit_exact_vs_plain": bool(ok)}


def sweep(args):
    """Parameter sweeps of the method on one workload: Pi (candidates and
    matching rounds) at Theta = 16, Theta (repetitions per level) at Pi = 4,
    and the ablation without chain rounds (moves sequenced by gain alone).
    Per setting: the partition's connectivity and violations, the hierarchy
    depth and the wall time of one partitioning (after one untimed run)."""
    import torch

    import paper_2605_20497_amd as pkg
    from paper_2605_20497_amd import workloads as W

    hg = W.CONFIGS[args.sweep_workload]()
    torch.cuda.set_device(0)

    def run(pi, theta, flags=0):
        g = pkg.Partitioner(device=0, pi=pi, theta=theta)
        if flags:
            g.close()
            g = pkg.Partitioner(device=0, pi=pi, theta=theta, no_chains=True)
        out = None
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
            out = {"pi": pi, "theta": theta, "chains": not flags, "conn": int(ev["conn"]),
                   "violations": int(ev["violations"]), "parts": int(ev["n_parts"]), "levels": int(nl),
                   "ms": round(dt * 1e3, 2)}
        g.close()
        print(json.dumps(out), file=sys.stderr, flush=True)
        return out

    rows = [run(pi, 16) for pi in (1, 2, 3, 4, 6, 8)]
    rows += [run(4, th) for th in (0, 1, 2, 4, 8, 32, 64)]
    rows.append(run(4, 16, flags=1))
    print(json.dumps({"sweep": args.sweep_workload, "nodes": hg.n_nodes, "pins": hg.n_pins,
                      "omega": hg.omega, "delta": hg.delta, "rows": rows}))


def main():
    args = _args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported "
              "(sharding across GPUs is described in DESIGN.md)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.sweep:
        sweep(args)
        return
    import numpy as np
    import torch

    import paper_2605_20497_amd as pkg
    from paper_2605_20497_amd import workloads as W

    hg = W.CONFIGS[args.workload]()
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
    # gains' row reads on the device; recording events around every launch would
    # add about a sixth to the step.  One extra step after the timed region
    # records every family for the breakdown.
    part = pkg.Partitioner(device=0, profile=True, profile_families=("propose", "gains", "dense_gemm", "gains_gemm"))

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
    for _ in range(args.steps):
        step()
        level_times.append(part.hgp_level_times())
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    stats_timed = part.hgp_kernel_stats()
    full = pkg.Partitioner(device=0, profile=True)
    hg_step = (hg.n_nodes, t_he_off, t_nsrc, t_pins, t_hw, t_nw)
    full.hgp_load_csr_device(*hg_step)
    full.hgp_set_limits(hg.omega, hg.delta, hg.k)
    full.hgp_coarsen()
    full.hgp_refine()
    torch.cuda.synchronize()
    stats = full.hgp_kernel_stats()
    full.close()
    levels = part.hgp_get_levels()
    ev = part.hgp_evaluate()
    lt = np.median(np.stack(level_times), axis=0)

    per_level = []
    for lv, (N, E, P, pairs) in enumerate(levels.tolist()):
        tc, tr = lt[lv] * 1e-9
        per_level.append({"level": lv, "nodes": N, "pins": P, "coarsen_ms": round(tc * 1e3, 3),
                          "refine_ms": round(tr * 1e3, 3),
                          "pins_per_s": (P / (tc + tr)) if tc + tr > 0 else None})
    # per-family breakdown from the separate fully profiled step
    fam = {k: v for k, v in stats.items() if v[0] > 0}
    total_ns = sum(v[1] for v in fam.values())
    dom = max(fam, key=lambda k: fam[k][1])
    breakdown = {k: {"launches": v[0], "ms_per_step": round(v[1] * 1e-6, 3)}
                 for k, v in sorted(fam.items(), key=lambda kv: -kv[1][1])}
    # Rooflines of the largest kernels, from HIP events over the timed steps;
    # `roofline` is the one that takes the most time.
    card_lv = []
    for lv in range(int(levels.shape[0])):
        he_off = part.hgp_get_level_graph(lv, what=("he_off",))[0]
        card_lv.append(np.diff(he_off).astype(np.int64))
    work_timed = part.hgp_kernel_work()
    roofs = {}
    prop = stats_timed.get("propose")
    dg = stats_timed.get("dense_gemm")
    n_prop = int(round(prop[0] / args.steps)) if prop else 0
    if prop and prop[0] > 0:
        # One launch per level on the histogram path (the first n_prop levels):
        # histogram updates sum_e |e| (|e| - 1) and the compulsory HBM bytes.
        t_launch = prop[1] / prop[0] * 1e-9
        upd = sum(int((c * (c - 1)).sum()) for c in card_lv[:n_prop]) / max(n_prop, 1)
        ach = upd / t_launch / 1e9
        nbytes = algorithmic_bytes("propose", levels.tolist()[:n_prop], part.pi) / max(n_prop, 1)
        tr = traffic("k_propose")
        roofs["k_propose"] = {
            "kernel": "k_propose", "bound": "alu", "achieved": round(ach, 2), "peak": LDS_UPDATE_PEAK_GOPS,
            "unit": "Gop/s", "frac": round(ach / LDS_UPDATE_PEAK_GOPS, 5), "traffic": tr,
            "op": "histogram update (32-bit LDS atomic add)", "ops_per_launch": int(upd),
            "avg_launch_ms": round(t_launch * 1e3, 4), "ms_per_step": round(prop[1] * 1e-6 / args.steps, 3),
            "hbm_compulsory_bytes_per_launch": int(nbytes),
            "hbm_compulsory_gbs": round(nbytes / t_launch / 1e9, 2),
            "hbm_frac": round(nbytes / t_launch / 1e9 / HBM_PEAK_GBS, 5)}
    gn = stats_timed.get("gains")
    if gn and gn[0] > 0 and work_timed.get("gains", 0) > 0:
        # Phi row entries read (counted on the device): one bin update each,
        # 2 bytes each from the 16-bit row copy.
        t_launch = gn[1] / gn[0] * 1e-9
        visits = work_timed["gains"] / gn[0]
        ach = visits / t_launch / 1e9
        roofs["k_gains16"] = {
            "kernel": "k_gains16", "bound": "alu", "achieved": round(ach, 2), "peak": LDS_UPDATE_PEAK_GOPS,
            "unit": "Gop/s", "frac": round(ach / LDS_UPDATE_PEAK_GOPS, 5), "traffic": traffic("k_gains16"),
            "op": "row entry read + bin update (32-bit LDS atomic add)", "ops_per_launch": int(visits),
            "avg_launch_ms": round(t_launch * 1e3, 4), "ms_per_step": round(gn[1] * 1e-6 / args.steps, 3),
            "row_bytes_gbs": round(2 * visits / t_launch / 1e9, 2)}
    if dg and dg[0] > 0:
        # int8 MACs issued by the dense proposal's products (counted by the
        # library from the padded sizes: planes + 1 products over the upper
        # triangle of 128 x 128 tiles, K = E rounded up to 128)
        macs = work_timed.get("dense_gemm", 0)
        t_launch = dg[1] / dg[0] * 1e-9
        ops = 2.0 * macs / dg[0]
        ach = ops / t_launch / 1e12
        roofs["k_dense_gemm"] = {
            "kernel": "k_dense_gemm", "bound": "mfma", "achieved": round(ach, 2), "peak": INT8_PEAK_TOPS,
            "unit": "TOP/s", "frac": round(ach / INT8_PEAK_TOPS, 5), "traffic": traffic("k_dense_gemm"),
            "op": "int8 MAC = 2 ops (v_mfma_i32_32x32x32_i8)", "ops_per_launch": int(ops),
            "avg_launch_ms": round(t_launch * 1e3, 4), "ms_per_step": round(dg[1] * 1e-6 / args.steps, 3)}
    gg = stats_timed.get("gains_gemm")
    if gg and gg[0] > 0:
        # int8 MACs issued by the dense in-isolation moves (counted by the
        # library: weight planes x padded nodes x padded partitions x E
        # rounded up to 128)
        macs = work_timed.get("gains_gemm", 0)
        t_launch = gg[1] / gg[0] * 1e-9
        ops = 2.0 * macs / gg[0]
        ach = ops / t_launch / 1e12
        roofs["k_conn_gemm"] = {
            "kernel": "k_conn_gemm", "bound": "mfma", "achieved": round(ach, 2), "peak": INT8_PEAK_TOPS,
            "unit": "TOP/s", "frac": round(ach / INT8_PEAK_TOPS, 5), "traffic": traffic("k_conn_gemm"),
            "op": "int8 MAC = 2 ops (v_mfma_i32_32x32x32_i8)", "ops_per_launch": int(ops),
            "avg_launch_ms": round(t_launch * 1e3, 4), "ms_per_step": round(gg[1] * 1e-6 / args.steps, 3)}
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
        "levels": per_level,
        "kernels": breakdown,
        "dominant_kernel": dom,
        "rooflines": list(roofs.values()),
        "kernel_time_share": round(total_ns * 1e-9 / dt, 4) if dt > 0 else None,
        "kernels_note": "per-family times from one extra fully profiled step; the timed steps record "
                        "events around the roofline kernels only",
        "roofline": roof,
    }
    part.close()
    if not args.no_batch:
        out["batched"] = batched_leg(args)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
