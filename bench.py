"""Benchmark of the temporal-betweenness hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload "mid-chunglu-n50k": directed Chung-Lu temporal graph (degree
exponent 2.3, n = 50,000, |E| = 2,000,000, bursty Pareto(1.5) renewal
timestamps over 10^5 ticks), shortest-foremost paths, a fixed sample of
r = 20,000 pairs per step, node and temporal-edge betweenness, c = 25
Rademacher vectors.  One step = one whole pass of the hot path: pair and sign
sampling, forward sweep, reverse dependency sweep, accumulation of the
estimator sums, the MCERA reduction and the bound on the host.  The graph is
resident in HBM before the timed region.

Prints one JSON line (metric: sampled pairs/s) with a "roofline" object for
the dominant kernel (the sweep; algorithmic bytes per launch over its mean
HIP-event duration) and a "cpu_baseline" object (the oracle on the host's
cores over a bounded sample of the same workload).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "mid-chunglu-n50k"
OPT = "sfm"
R_PER_STEP = 20_000
C = 25
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(t, c):
    """Bytes the method must move per launch: the swept window of the edge
    stream (12 B per temporal edge), each recorded appearance-DAG arc written
    and read back (2 x 16 B), the estimator sums of each touched node
    ((2 + c) x 8 B) and each touched temporal edge (8 B)."""
    return (12 * t["window_edges"] + 32 * t["arcs"] + 8 * (2 + c) * t["touched_nodes"]
            + 8 * t["touched_edges"])


def cpu_baseline(G, seed, budget_s=15.0):
    import numpy as np
    import oracle
    og = oracle.Graph.of(G)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
    done = 0
    t_used = 0.0
    batch = 2 * threads
    while t_used < budget_s and done < R_PER_STEP:
        S, Z = oracle.draw_pairs(seed, oracle.STREAM_PAIR, G.n, done, batch)
        lam = oracle.rade_words(seed, done, batch)
        t0 = time.perf_counter()
        oracle.accumulate(og, OPT, S, Z, lam, c=C, mode=1, edges=True, nthreads=threads)
        t_used += time.perf_counter() - t0
        done += batch
    return {"value": done / t_used, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": "first %d pairs of the step's pair stream (sfm, c=%d, node+edge sums), %.1f s" % (
                done, C, t_used)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=2002)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; --gpus %d is not supported (sampled pairs are "
              "independent, so N GPUs would each take 1/N of the pairs)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2304_08356_amd as pk
    from synthgen import workload

    assert torch.cuda.is_available(), "bench needs the GPU"
    G = workload(WORKLOAD)
    gg = pk.Graph.of(G)
    for i in range(args.warmup):
        gg.run(OPT, fixed_r=R_PER_STEP, seed=args.seed + 1000 + i, c=C, edges=True)
    torch.cuda.synchronize()
    tot = {"sweep_ms": 0.0, "launches": 0, "window_edges": 0, "arcs": 0, "touched_nodes": 0,
           "touched_edges": 0}
    t0 = time.perf_counter()
    for k in range(args.steps):
        _, _, res = gg.run(OPT, fixed_r=R_PER_STEP, seed=args.seed + k, c=C, edges=True)
        t = gg.last_timing()
        for key in tot:
            tot[key] += t[key]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pairs = R_PER_STEP * args.steps
    ms_step = wall * 1e3 / args.steps
    kern_ms = tot["sweep_ms"] / max(1, tot["launches"])
    abytes = algorithmic_bytes(tot, C) / max(1, tot["launches"])
    achieved = abytes / (kern_ms / 1e3) / 1e9
    out = {
        "metric": "sampled pairs/s",
        "value": pairs / wall,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64 counts, f64 sums",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "n": G.n, "edges": G.m, "ticks": 100000, "optimality": OPT,
                   "pairs_per_step": R_PER_STEP, "c": C, "edge_betweenness": True},
        "temporal_edges_per_s": tot["window_edges"] / wall,
        "mean_window_edges": tot["window_edges"] / pairs,
        "mean_arcs": tot["arcs"] / pairs,
        "sweep_ms_per_launch": kern_ms,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "mantra::k_sweep", "algorithmic_bytes_per_launch": abytes},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(G, args.seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
