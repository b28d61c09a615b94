"""Benchmark of the temporal-betweenness hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--slabs N]
                    [--no-forms] [--no-serve] [--no-trk] [--no-rtb] [--no-distances]
                    [--no-cpu-baseline]
    python bench.py --calibrate-copy     (plain copy kernel for the traffic counters)
    python bench.py --batching           (n = 10^6 Algorithm 1 and the 256 packed graphs)
    python bench.py --serve-only [--serve-workload NAME] [--serve-requests K]

Workload "mid-chunglu-n50k": directed Chung-Lu temporal graph (degree
exponent 2.3, n = 50,000, |E| = 2,000,000, bursty Pareto(1.5) renewal
timestamps over 10^5 ticks), shortest-foremost paths, a fixed sample of
r = 20,000 pairs per step, node and temporal-edge betweenness, c = 25
Rademacher vectors.  One step = one whole pass of the hot path: pair and sign
sampling, launch ordering, forward sweep, reverse dependency sweep,
accumulation of the estimator sums, the MCERA reduction and the bound on the
host.  The graph is resident in HBM before the timed region.

Prints one JSON line (value: sampled pairs/s of the steps) with
 - "roofline": the sweep kernel's algorithmic bytes per launch over its mean
   HIP-event duration, against the HBM peak; "traffic" is the DRAM bytes per
   launch that rocprofv3's FETCH_SIZE / WRITE_SIZE counters read for this
   kernel source (null once the source differs from the profiled one);
 - "forms": Algorithm 1 at eps = 0.01, delta = 0.1 on the same graph, as
   persistent launches, as one replayed HIP graph per round, and the
   unbatched one-launch-per-pair form (timed on a fixed sample);
 - "serve": requests with Poisson arrivals (random windows, optimalities,
   eps in {0.01, 0.005}) through the serving scheduler: p50/p99 latency;
 - "trk": the same step with the TRK estimator (one sampled optimal walk per
   pair instead of the dependency sweep);
 - "rtb": the RTB estimator (sampled sources, all targets) on the same graph;
 - "distances": Algorithm 2 (sampled temporal distance metrics) from 256
   sources, the paper's seed count, for sh and pfm on the same graph, with
   the oracle's per-source distances timed beside it on 32 sources;
 - "cpu_baseline": the oracle on the host's cores, on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sampled pairs/s + temporal edges/s (HBM GB/s vs peak); p50/p99 request latency"
WORKLOAD = "mid-chunglu-n50k"
OPT = "sfm"
R_PER_STEP = 20_000
C = 25
HBM_PEAK_GBS = 8000.0
SWEEP_SRC = os.path.join(ROOT, "paper_2304_08356_amd", "csrc", "mantra_sweep.hip")

# DRAM traffic of the sweep kernel on the step above (rocprofv3 --pmc
# FETCH_SIZE, then WRITE_SIZE, summed over the k_sweep dispatches of the
# profiled run, divided by their count, and scaled by the ratio of bytes to
# counter bytes that the same counters give for a plain copy of known size),
# valid for the kernel source with this SHA-256 only, profiled at a fixed
# grid of 2,880 slabs (the autotuned grid of a run may differ).
TRAFFIC = {
    "slabs": 2880,
    "sweep_sha256": "a67e4431b25d0edfa880a551c0bc9657cf95bcc31eb000ac9cc62522fbd7ba2c",
    "fetch_bytes_per_launch": 4.9171e+11,   # 2.40101e+08 KiB x 1.99995
    "write_bytes_per_launch": 7.8496e+10,   # 7.66559e+07 KiB x 1.00000
}


def sha256(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def algorithmic_bytes(t, c):
    """Bytes the method must move per launch: the swept window of the edge
    stream (12 B per temporal edge), each recorded appearance-DAG arc written
    and read back (2 x 16 B), the estimator sums of each touched node
    ((2 + c) x 8 B) and each touched temporal edge (8 B)."""
    return (12 * t["window_edges"] + 32 * t["arcs"] + 8 * (2 + c) * t["touched_nodes"]
            + 8 * t["touched_edges"])


def cpu_baseline(G, seed, budget_s=15.0):
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


def tuned_launch(tuned, **over):
    """set_launch arguments that restore an autotuned configuration (arc room
    left automatic), with the given overrides."""
    cfg = {"n_slabs": tuned["n_slabs"], "order": tuned["order"], "hub_nodes": tuned["hub_nodes"],
           "wide_counts": tuned["wide_counts"]}
    cfg.update(over)
    return cfg


def forms(gg, torch, seed, tuned):
    """Algorithm 1 at eps = 0.01, delta = 0.1 (sfm, c = 25) in three launch
    forms; the autotuned configuration is in force again afterwards."""
    out = {}
    for name, cfg in (("batched", {}), ("graph", {"graph_rounds": True})):
        gg.set_launch(**tuned_launch(tuned, **cfg))
        gg.run(OPT, eps=0.01, delta=0.1, seed=seed + 99, c=C)  # warm (pool, capture path)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, res = gg.run(OPT, eps=0.01, delta=0.1, seed=seed, c=C)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out[name] = {"pairs": res["samples"] + res["s_boot"], "rounds": res["rounds"], "wall_s": wall,
                     "pairs_per_s": (res["samples"] + res["s_boot"]) / wall, "xi": res["xi"]}
    # the unbatched form: one single-workgroup launch per pair, on a fixed
    # sample (a whole progressive run this way takes minutes)
    r = 256
    gg.set_launch(**tuned_launch(tuned, per_pair_launch=True))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gg.run(OPT, fixed_r=r, seed=seed, c=C)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out["plain"] = {"pairs": r, "wall_s": wall, "pairs_per_s": r / wall,
                    "note": "fixed sample of %d pairs, one launch per pair" % r}
    gg.set_launch(**tuned_launch(tuned))
    base = out["plain"]["pairs_per_s"]
    for k in ("batched", "graph"):
        out[k]["speedup_vs_plain"] = out[k]["pairs_per_s"] / base
    return out


def trk_step(gg, torch, seed, steps=3):
    """The bench step (sfm, r = 20,000, c = 25, node + edge sums) with the
    TRK estimator."""
    gg.run(OPT, fixed_r=R_PER_STEP, seed=seed + 999, c=C, edges=True, trk=True)
    torch.cuda.synchronize()
    tot = {"sweep_ms": 0.0, "launches": 0, "window_edges": 0, "arcs": 0, "touched_nodes": 0, "touched_edges": 0}
    t0 = time.perf_counter()
    for k in range(steps):
        gg.run(OPT, fixed_r=R_PER_STEP, seed=seed + k, c=C, edges=True, trk=True)
        t = gg.last_timing()
        for key in tot:
            tot[key] += t[key]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = {"steps": steps, "pairs_per_s": R_PER_STEP * steps / wall, "ms_per_step": wall * 1e3 / steps,
           "sweep_ms_per_launch": tot["sweep_ms"] / max(1, tot["launches"]), "hbm_frac": hbm_frac(tot, C),
           "kernel": "mantra::k_sweep<2>"}
    return out


def rtb_step(gg, torch, seed, r=0, steps=2):
    """The bench step's settings (sfm, c = 25, node + edge sums) with the RTB
    estimator: r sampled sources per step (default: two per workgroup of the
    grid, since each source's sweep runs to the end of the span and a launch
    lasts as long as its longest sweeps), each swept to the end of the span
    with the dependencies of every reached target."""
    if r <= 0:
        r = 2 * gg.get_launch()["n_slabs"]
    gg.run(OPT, fixed_r=256, seed=seed + 999, c=C, edges=True, rtb=True)
    torch.cuda.synchronize()
    tot = {"sweep_ms": 0.0, "launches": 0, "window_edges": 0, "arcs": 0, "touched_nodes": 0, "touched_edges": 0}
    t0 = time.perf_counter()
    for k in range(steps):
        gg.run(OPT, fixed_r=r, seed=seed + k, c=C, edges=True, rtb=True)
        t = gg.last_timing()
        for key in tot:
            tot[key] += t[key]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return {"steps": steps, "sources_per_step": r, "sources_per_s": r * steps / wall,
            "ms_per_step": wall * 1e3 / steps, "sweep_ms_per_launch": tot["sweep_ms"] / max(1, tot["launches"]),
            "temporal_edges_per_s": tot["window_edges"] / (tot["sweep_ms"] / 1e3),
            "hbm_frac": hbm_frac(tot, C), "kernel": "mantra::k_sweep<3>"}


def hbm_frac(t, c):
    """Algorithmic bytes of a call's sweep launches over their summed HIP-event
    duration, as a fraction of the HBM peak."""
    if t["sweep_ms"] <= 0:
        return None
    return algorithmic_bytes(t, c) / (t["sweep_ms"] / 1e3) / 1e9 / HBM_PEAK_GBS


def distances(gg, torch, seed, r=256, og=None):
    """Algorithm 2 from r sources (sh and pfm, tau = 0.9), blocking calls;
    beside it the oracle's per-source distances on a bounded sample."""
    out = {}
    for opt in ("sh", "pfm"):
        gg.distances(opt, 16, seed=seed + 1)  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, res = gg.distances(opt, r, seed=seed, tau=0.9)
        wall = time.perf_counter() - t0
        out[opt] = {"sources": r, "wall_ms": wall * 1e3, "gpu_ms": res["gpu_ms"],
                    "temporal_edges_per_s": res["window_edges"] / (res["gpu_ms"] / 1e3),
                    # 12 B per swept edge, and the list of reached nodes written and read back
                    "hbm_frac": (12 * res["window_edges"] + 8 * res["reached_pairs"]) / (res["gpu_ms"] / 1e3) / 1e9 / HBM_PEAK_GBS,
                    "d_lb": res["d_lb"], "d_tau": res["d_tau"], "zeta": res["zeta"], "psi": res["psi"],
                    "rho": res["rho"]}
        if og is not None:
            from oracle import distances as odist
            threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
            S = odist.draw_sources(seed, og.n, 32)
            t0 = time.perf_counter()
            odist.source_hops(og, opt, S, nthreads=threads)
            dt = time.perf_counter() - t0
            out[opt]["cpu_baseline"] = {"value": len(S) / dt, "unit": "sources/s", "cores": threads,
                                        "kind": "oracle",
                                        "sample": "first %d sources of the same source stream, %.1f s" % (len(S), dt)}
    return out


def serve(gg, G, torch, n_req=12, rate=50.0, seed=4002, workload_name=WORKLOAD):
    """Poisson arrivals at `rate` req/s; each request a random window of
    5-100% of the span, a uniform optimality and eps in {0.01, 0.005}."""
    import numpy as np
    from synthgen import request_stream
    reqs = request_stream(n_req, rate, int(G.t.min()), int(G.t.max()), seed)
    opts = ("sh", "fm", "sfm", "pfm")
    lat = [None] * n_req
    pairs = [0] * n_req
    errs = []  # saturated fm counts (E_OVERFLOW): reported, never rounded
    t_start = time.perf_counter()

    def waiter(i, tk):
        ok = True
        try:
            res = tk.poll(timeout_ms=-1)
        except Exception as e:  # noqa: BLE001 - saturated fm counts are reported, not fatal
            res = tk.result
            errs.append(str(e))
            ok = False
        if res is not None:
            pairs[i] = res["samples"] + res["s_boot"]
            if ok:
                lat[i] = res["latency_ms"]
            print("request %d (%s) %s after %.0f ms, %d pairs" % (i, opts[reqs[i]["opt"]], "done" if ok else "failed",
                                                               res["latency_ms"], pairs[i]), file=sys.stderr, flush=True)

    threads = []
    for i, rq in enumerate(reqs):
        delay = t_start + rq["arrival_s"] - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        tk = gg.submit(opts[rq["opt"]], eps=rq["eps"], delta=rq["delta"], seed=rq["seed"] % (2**63), c=C,
                       t0=rq["t0"], t1=rq["t1"])
        th = threading.Thread(target=waiter, args=(i, tk))
        th.start()
        threads.append(th)
    for th in threads:
        th.join()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    L = np.array([x for x in lat if x is not None])
    return {"requests": n_req, "offered_req_per_s": rate, "completed": int(L.size), "wall_s": wall,
            "completed_req_per_s": L.size / wall, "pairs_per_s": sum(pairs) / wall,
            "p50_ms": float(np.percentile(L, 50)) if L.size else None,
            "p99_ms": float(np.percentile(L, 99)) if L.size else None,
            "latency_of": "completed requests", "overflowed": len(errs),
            "workload": workload_name + ", windows/optimalities/eps of the serving recipe"}


def batching(pk, torch, seed):
    """The batching workloads, outside the default run (minutes of graph
    generation): one launch of r = 2,000 sh pairs per graph over the 256
    graphs of packed-256; Algorithm 1 at eps = 0.005, delta = 0.1, c = 16,
    s1 = 4,096 on big-chunglu-n1m for pfm, each round one replayed HIP graph
    at the autotuned grid; fm on the same graph as a fixed sample of one
    first round (4,096 pairs) at that grid, since its walk counts pass 2^64
    (and 2^256) and Algorithm 1 then stops with MANTRA_E_OVERFLOW."""
    from synthgen import workload
    out = {}

    def note(key, d):
        out[key] = d
        print("%s: %s" % (key, json.dumps(d)), file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    gs = workload("packed-256")
    pg = pk.Graph.packed(gs)
    print("packed-256 resident after %.1f s" % (time.perf_counter() - t0), file=sys.stderr, flush=True)
    r = 2000
    pg.run("sh", fixed_r=64, seed=seed + 99, c=C)
    for k in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, res = pg.run("sh", fixed_r=r, seed=seed + k, c=C, raise_on_error=False)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        t = pg.last_timing()
        note("packed_sh", {
            "workload": "packed-256", "graphs": len(gs), "edges": int(sum(g.m for g in gs)), "pairs_per_graph": r,
            "pairs": r * len(gs), "rc": res["rc"], "n_overflow": res["n_overflow"], "wall_s": wall,
            "pairs_per_s": r * len(gs) / wall, "sweep_ms": t["sweep_ms"], "launches": t["launches"],
            "temporal_edges_per_s": t["window_edges"] / max(t["sweep_ms"] / 1e3, 1e-9),
            "hbm_frac": hbm_frac(t, C), "grid_balance": t["balance"], "launch": pg.get_launch()})
    del pg, gs
    t0 = time.perf_counter()
    G = workload("big-chunglu-n1m")
    gg = pk.Graph.of(G)
    print("big-chunglu-n1m resident after %.1f s" % (time.perf_counter() - t0), file=sys.stderr, flush=True)
    gg.set_launch(graph_rounds=True)
    t0 = time.perf_counter()
    tuned = gg.autotune("pfm", seed=seed + 7)
    print("autotuned in %.1f s: %s" % (time.perf_counter() - t0, json.dumps(tuned)), file=sys.stderr, flush=True)

    def timed(opt, **kw):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, res = gg.run(opt, c=16, raise_on_error=False, **kw)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        t = gg.last_timing()
        pairs = res["samples"] + res["s_boot"]
        return {"workload": "big-chunglu-n1m", "optimality": opt, "c": 16, "rc": res["rc"],
                "rounds": res["rounds"], "samples": res["samples"], "s_boot": res["s_boot"], "omega": res["omega"],
                "xi": res["xi"], "n_overflow": res["n_overflow"], "wall_s": wall, "pairs_per_s": pairs / wall,
                "sweep_ms": t["sweep_ms"], "launches": t["launches"],
                "temporal_edges_per_s": t["window_edges"] / max(t["sweep_ms"] / 1e3, 1e-9),
                "hbm_frac": hbm_frac(t, 16), "grid_balance": t["balance"], "launch": tuned}

    note("n1m_pfm", dict(timed("pfm", eps=0.005, delta=0.1, seed=seed, s1=4096), eps=0.005, delta=0.1, s1=4096))
    note("n1m_fm_first_round", dict(timed("fm", fixed_r=4096, seed=seed), fixed_r=4096))
    return out


def calibrate_copy(torch):
    """A plain device-to-device copy of known size, for scaling the traffic
    counters (run under rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE)."""
    n = 1 << 28  # 256 Mi floats = 1 GiB each way
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-distances", action="store_true")
    ap.add_argument("--no-trk", action="store_true")
    ap.add_argument("--serve-only", action="store_true",
                    help="only the serving measurement, on --serve-workload (prints {\"serve\": ...})")
    ap.add_argument("--serve-workload", default=WORKLOAD)
    ap.add_argument("--serve-requests", type=int, default=12)
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--batching", action="store_true",
                    help="only the batching workloads (n = 10^6 Algorithm 1, packed-256; prints {\"batching\": ...})")
    ap.add_argument("--no-rtb", action="store_true")
    ap.add_argument("--slabs", type=int, default=0,
                    help="fixed number of persistent workgroups instead of the autotuner's pick "
                         "(profiling runs: every sweep launch of the run is then alike)")
    ap.add_argument("--seed", type=int, default=2002)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU; --gpus %d is not supported (sampled pairs are "
              "independent, so N GPUs would each take 1/N of the pairs)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench needs the GPU"
    if args.calibrate_copy:
        calibrate_copy(torch)
        return
    import paper_2304_08356_amd as pk
    from synthgen import workload

    if args.batching:
        print(json.dumps({"batching": batching(pk, torch, args.seed)}), flush=True)
        return
    if args.serve_only:
        t0 = time.perf_counter()
        G = workload(args.serve_workload)
        gg = pk.Graph.of(G)
        print("graph %s resident after %.1f s" % (args.serve_workload, time.perf_counter() - t0), file=sys.stderr,
              flush=True)
        print(json.dumps({"serve": serve(gg, G, torch, n_req=args.serve_requests,
                                         workload_name=args.serve_workload)}), flush=True)
        return
    G = workload(WORKLOAD)
    gg = pk.Graph.of(G)
    # launch configuration picked by the autotuner on a calibration sample
    if args.slabs > 0:
        gg.set_launch(n_slabs=args.slabs)
        tuned = gg.get_launch()
    else:
        tuned = gg.autotune(OPT, sample_pairs=R_PER_STEP, seed=args.seed + 7)
    for i in range(args.warmup):
        gg.run(OPT, fixed_r=R_PER_STEP, seed=args.seed + 1000 + i, c=C, edges=True)
    torch.cuda.synchronize()
    tot = {"sweep_ms": 0.0, "launches": 0, "window_edges": 0, "arcs": 0, "touched_nodes": 0,
           "touched_edges": 0}
    bal = 0.0
    t0 = time.perf_counter()
    for k in range(args.steps):
        _, _, res = gg.run(OPT, fixed_r=R_PER_STEP, seed=args.seed + k, c=C, edges=True)
        t = gg.last_timing()
        for key in tot:
            tot[key] += t[key]
        bal += t["balance"] * t["sweep_ms"]
        print("step %d: %.1f ms sweep" % (k, t["sweep_ms"]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pairs = R_PER_STEP * args.steps
    ms_step = wall * 1e3 / args.steps
    kern_ms = tot["sweep_ms"] / max(1, tot["launches"])
    abytes = algorithmic_bytes(tot, C) / max(1, tot["launches"])
    achieved = abytes / (kern_ms / 1e3) / 1e9
    traffic = None
    if TRAFFIC["sweep_sha256"] == sha256(SWEEP_SRC) and TRAFFIC["fetch_bytes_per_launch"]:
        traffic = TRAFFIC["fetch_bytes_per_launch"] + TRAFFIC["write_bytes_per_launch"]
    out = {
        "metric": METRIC,
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
        "grid_balance": bal / max(tot["sweep_ms"], 1e-9),
        "launch": tuned,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "mantra::k_sweep<0>", "algorithmic_bytes_per_launch": abytes,
                     "traffic_slabs": TRAFFIC["slabs"] if traffic is not None else None},
    }
    if not args.no_forms:
        out["forms"] = forms(gg, torch, args.seed, tuned)
    if not args.no_serve:
        out["serve"] = serve(gg, G, torch, n_req=args.serve_requests)
    og = None
    if not args.no_cpu_baseline:
        import oracle
        og = oracle.Graph.of(G)
    if not args.no_trk:
        out["trk"] = trk_step(gg, torch, args.seed)
    if not args.no_rtb:
        out["rtb"] = rtb_step(gg, torch, args.seed)
    if not args.no_distances:
        out["distances"] = distances(gg, torch, args.seed, og=og)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(G, args.seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
