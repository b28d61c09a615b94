"""Benchmark of the temporal-betweenness hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--slabs N]
                    [--no-mid] [--no-forms] [--no-serve] [--no-trk] [--no-rtb] [--no-distances]
                    [--no-optimalities] [--no-cpu-baseline]
    python bench.py --calibrate-copy     (plain copy kernel for the traffic counters)
    python bench.py --batching           (n = 10^6 Algorithm 1 and the 256 packed graphs)
    python bench.py --serve-only [--serve-workload NAME] [--serve-requests K] [--serve-rate R]

Headline workload "serve-chunglu-n2m", the largest graph of the workloads:
directed Chung-Lu temporal graph (degree exponent 2.3, n = 2,000,000,
|E| = 50,000,000, bursty Pareto(1.5) renewal timestamps over 10^6 ticks),
shortest-foremost paths over the whole span, a fixed sample of R pairs per
step, node and temporal-edge betweenness, c = 25 Rademacher vectors.  One
step = one whole pass of the hot path: pair and sign sampling, launch
ordering, forward sweep, reverse dependency sweep, accumulation of the
estimator sums, the MCERA reduction and the bound on the host, and the
estimates copied to host arrays.  The graph is resident in HBM before the
timed region.

Prints one JSON line (value: sampled pairs/s of the steps) with
 - "roofline": the sweep kernel's algorithmic bytes per launch over its mean
   HIP-event duration, against the HBM peak; "traffic" is the DRAM bytes per
   launch that rocprofv3's FETCH_SIZE / WRITE_SIZE counters read for this
   kernel source at this workload and grid (null once either differs);
 - "optimalities": fixed samples of the other optimalities on the same graph;
 - "plain": the unbatched form (one launch per pair) on the step's first
   pairs, against the step's rate;
 - "cpu_baseline": the oracle on the host's cores (all of them, and one), on
   the first pairs of the step's pair stream;
 - "mid": the mid-size workload "mid-chunglu-n50k" (n = 50,000, |E| = 2*10^6,
   sfm, r = 20,000 per step) with its own roofline, and on it: "forms"
   (Algorithm 1 at eps = 0.01, delta = 0.1 batched, as replayed HIP graphs,
   served, and one launch per pair), "serve" (requests with Poisson
   arrivals), "trk", "rtb" and "distances" (the other estimators and
   Algorithm 2).
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
WORKLOAD = "serve-chunglu-n2m"
OPT = "sfm"
# pairs per step: the launch ends when its longest pairs do (a sfm pair on
# this graph sweeps up to 5.5 times the mean window), so a step amortizes
# them over 8,192 pairs; 4,096-pair steps are reported beside it
R_PER_STEP = 8192
R_SMALL = 4096
C = 25
MID = "mid-chunglu-n50k"
MID_R = 20_000
HBM_PEAK_GBS = 8000.0
SWEEP_SRC = os.path.join(ROOT, "paper_2304_08356_amd", "csrc", "mantra_sweep.hip")

# Launch configuration of the headline step: 2,048 hub nodes' state in LDS
# and the grid the device keeps resident with that LDS (1,280 single-wave
# workgroups), the rest automatic.  Taken from a sweep of grids and hub
# counts on this graph (sfm: 1,024-4,096 hubs, 800-1,793 workgroups; with
# 4,096 pairs a step, 1,100 workgroups were 5% faster, with 8,192 the
# resident grid is 12% faster than 1,100); the autotuner itself would take
# minutes here.
HEADLINE_LAUNCH = {"n_slabs": 0, "hub_nodes": 2048}

# DRAM traffic of the sweep kernel (rocprofv3 --pmc FETCH_SIZE, then
# WRITE_SIZE, summed over the k_sweep dispatches of the profiled run, divided
# by their count, and scaled by the ratio of bytes to counter bytes that the
# same counters give for a plain copy of known size), per workload and launch
# configuration, valid for the kernel source with the given SHA-256 at the
# given grid, hub count, own arc buffer and pairs per launch only.
TRAFFIC = {
    "serve-chunglu-n2m": [
        {"slabs": 1280, "hub_nodes": 2048, "arc_cap": 1040577, "pairs_per_launch": 8192,
         "sweep_sha256": "0d36c97e6b258bdd124064d52e060c30ff5d2d5633625e8a1aee9d9f4071ed25",
         "fetch_bytes_per_launch": 2.2094e+13, "write_bytes_per_launch": 1.8402e+12},
    ],
    "mid-chunglu-n50k": [
        {"slabs": 2880, "hub_nodes": 0, "arc_cap": 815414, "pairs_per_launch": 20000,
         "sweep_sha256": "0d36c97e6b258bdd124064d52e060c30ff5d2d5633625e8a1aee9d9f4071ed25",
         "fetch_bytes_per_launch": 4.9429e+11, "write_bytes_per_launch": 7.8774e+10},
        {"slabs": 2688, "hub_nodes": 256, "arc_cap": 1048576, "pairs_per_launch": 20000,
         "sweep_sha256": "0d36c97e6b258bdd124064d52e060c30ff5d2d5633625e8a1aee9d9f4071ed25",
         "fetch_bytes_per_launch": 4.1898e+11, "write_bytes_per_launch": 7.5541e+10},
    ],
}


def sha256(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads():
    return int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1


def algorithmic_bytes(t, c):
    """Bytes the method must move per launch: the swept window of the edge
    stream (12 B per temporal edge), each recorded appearance-DAG arc written
    and read back (2 x 16 B), the estimator sums of each touched node
    ((2 + c) x 8 B) and each touched temporal edge (8 B)."""
    return (12 * t["window_edges"] + 32 * t["arcs"] + 8 * (2 + c) * t["touched_nodes"]
            + 8 * t["touched_edges"])


def hbm_frac(t, c):
    """Algorithmic bytes of a call's sweep launches over their summed HIP-event
    duration, as a fraction of the HBM peak."""
    if t["sweep_ms"] <= 0:
        return None
    return algorithmic_bytes(t, c) / (t["sweep_ms"] / 1e3) / 1e9 / HBM_PEAK_GBS


def traffic_of(workload, launch, pairs):
    """The profiled entry for this workload, kernel source and launch, or None."""
    sha = sha256(SWEEP_SRC)
    for tr in TRAFFIC.get(workload, []):
        if (tr["sweep_sha256"] == sha and tr["slabs"] == launch["n_slabs"] and tr["hub_nodes"] == launch["hub_nodes"]
                and tr["arc_cap"] == launch["arc_cap"] and tr["pairs_per_launch"] == pairs):
            return tr
    return None


def timed_steps(gg, torch, opt, r, steps, warmup, seed, c=C):
    """warmup + steps fixed samples of r pairs (node and edge sums, written to
    the same host arrays every step); totals of the timed steps."""
    import numpy as np
    out = (np.zeros(gg.n), np.zeros(gg.m_input))
    for i in range(warmup):
        gg.run(opt, fixed_r=r, seed=seed + 1000 + i, c=c, edges=True, out=out)
    torch.cuda.synchronize()
    tot = {"sweep_ms": 0.0, "launches": 0, "window_edges": 0, "arcs": 0, "touched_nodes": 0,
           "touched_edges": 0}
    bal = 0.0
    t0 = time.perf_counter()
    for k in range(steps):
        _, _, res = gg.run(opt, fixed_r=r, seed=seed + k, c=c, edges=True, out=out)
        t = gg.last_timing()
        for key in tot:
            tot[key] += t[key]
        bal += t["balance"] * t["sweep_ms"]
        log("step %d: %.1f ms sweep, %d launches" % (k, t["sweep_ms"], t["launches"]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return tot, wall, bal / max(tot["sweep_ms"], 1e-9)


def roofline(tot, workload, launch, kernel, pairs):
    kern_ms = tot["sweep_ms"] / max(1, tot["launches"])
    abytes = algorithmic_bytes(tot, C) / max(1, tot["launches"])
    achieved = abytes / (kern_ms / 1e3) / 1e9
    tr = traffic_of(workload, launch, pairs)
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": tr["fetch_bytes_per_launch"] + tr["write_bytes_per_launch"] if tr else None,
            "kernel": kernel, "algorithmic_bytes_per_launch": abytes, "sweep_ms_per_launch": kern_ms,
            "traffic_slabs": tr["slabs"] if tr else None}


class OracleOneThread(threading.Thread):
    """The oracle on one thread (the first pair of the step's pair stream),
    run beside the GPU sections that follow the timed steps: a host core the
    GPU work does not use."""

    def __init__(self, og, n, seed, opt, c=C):
        super().__init__(daemon=True)
        self.og, self.n, self.seed, self.opt, self.c = og, n, seed, opt, c
        self.dt = None

    def run(self):
        import oracle
        S, Z = oracle.draw_pairs(self.seed, oracle.STREAM_PAIR, self.n, 0, 1)
        lam = oracle.rade_words(self.seed, 0, 1)
        t0 = time.perf_counter()
        oracle.accumulate(self.og, self.opt, S, Z, lam, c=self.c, mode=1, edges=True, nthreads=1)
        self.dt = time.perf_counter() - t0


def cpu_baseline(og, n, seed, opt, one=None, c=C, t_budget=30.0):
    """The oracle (mode 1, OpenMP over pairs) on the first pairs of the step's
    pair stream, on every host thread (one pair per thread, repeated while
    within the budget); and its one-thread figure (one pair)."""
    import oracle
    if one is not None:
        one.join()  # the one-thread run ends before every thread is busy
    threads = host_threads()
    out = {"unit": "pairs/s", "kind": "oracle", "cpu_model": cpu_model(), "cores": threads}
    done, t_used = 0, 0.0
    while done == 0 or (t_used < t_budget and done < 64 * threads):
        S, Z = oracle.draw_pairs(seed, oracle.STREAM_PAIR, n, done, threads)
        lam = oracle.rade_words(seed, done, threads)
        t0 = time.perf_counter()
        oracle.accumulate(og, opt, S, Z, lam, c=c, mode=1, edges=True, nthreads=threads)
        t_used += time.perf_counter() - t0
        done += threads
    out["value"] = done / t_used
    out["sample"] = "first %d pairs of the step's pair stream (%s, c=%d, node+edge sums), %.1f s on %d threads" % (
        done, opt, c, t_used, threads)
    if one is None:
        one = OracleOneThread(og, n, seed, opt, c)
        one.run()
    out["value_1_thread"] = 1.0 / one.dt
    out["sample_1_thread"] = "the first pair of the same stream on one thread, %.1f s" % one.dt
    return out


def plain_fixed(gg, torch, opt, r, seed, tuned):
    """The unbatched form (one single-workgroup launch per pair) on the first
    r pairs of the step's pair stream."""
    gg.set_launch(**tuned_launch(tuned, per_pair_launch=True))
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gg.run(opt, fixed_r=r, seed=seed, c=C, edges=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    finally:
        gg.set_launch(**tuned_launch(tuned))
    return {"pairs": r, "wall_s": wall, "pairs_per_s": r / wall,
            "note": "first %d pairs of the step's pair stream, one launch per pair" % r}


def tuned_launch(tuned, **over):
    """set_launch arguments that restore a launch configuration (arc room
    left automatic), with the given overrides."""
    cfg = {"n_slabs": tuned["n_slabs"], "order": tuned["order"], "hub_nodes": tuned["hub_nodes"],
           "wide_counts": tuned["wide_counts"]}
    cfg.update(over)
    return cfg


def optimalities(gg, torch, seed, plan):
    """Fixed samples of the given optimalities on the headline graph (node and
    edge sums, c = 25): pairs/s, window edges/s and the roofline fraction."""
    out = {}
    for opt, r in plan:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, res = gg.run(opt, fixed_r=r, seed=seed, c=C, edges=True, raise_on_error=False)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        t = gg.last_timing()
        out[opt] = {"pairs": r, "rc": res["rc"], "n_overflow": res["n_overflow"], "wall_s": wall,
                    "pairs_per_s": r / wall, "sweep_ms": t["sweep_ms"], "launches": t["launches"],
                    "temporal_edges_per_s": t["window_edges"] / max(t["sweep_ms"] / 1e3, 1e-9),
                    "mean_window_edges": t["window_edges"] / r, "mean_arcs": t["arcs"] / r,
                    "hbm_frac": hbm_frac(t, C), "grid_balance": t["balance"]}
        log("%s: %s" % (opt, json.dumps(out[opt])))
    return out


# ------------------------------------------------------------------ mid-size workload


def forms(gg, torch, seed, tuned):
    """Algorithm 1 at eps = 0.01, delta = 0.1 (sfm, c = 25) in four launch
    forms on the same request: persistent launches, rounds replayed from one
    captured HIP graph, the serving scheduler (one request submitted alone),
    and one launch per pair.  The last is timed on the run's first 512 pairs
    (a whole run that way takes minutes) and scaled to the run's pair count,
    labelled as such."""
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
    gg.set_launch(**tuned_launch(tuned))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tk = gg.submit(OPT, eps=0.01, delta=0.1, seed=seed, c=C)
    res = tk.poll(timeout_ms=-1)
    wall = time.perf_counter() - t0
    out["served"] = {"pairs": res["samples"] + res["s_boot"], "rounds": res["rounds"], "wall_s": wall,
                     "pairs_per_s": (res["samples"] + res["s_boot"]) / wall, "xi": res["xi"],
                     "latency_ms": res["latency_ms"]}
    r = 512
    gg.set_launch(**tuned_launch(tuned, per_pair_launch=True))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gg.run(OPT, fixed_r=r, seed=seed, c=C)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gg.set_launch(**tuned_launch(tuned))
    n_run = out["batched"]["pairs"]
    out["plain"] = {"pairs_timed": r, "wall_s_timed": wall, "pairs_per_s": r / wall,
                    "pairs": n_run, "wall_s": wall / r * n_run,
                    "note": "one launch per pair, timed on the run's first %d pairs and scaled to its %d pairs"
                            % (r, n_run)}
    base = out["plain"]["pairs_per_s"]
    for k in ("batched", "graph", "served"):
        out[k]["speedup_vs_plain"] = out[k]["pairs_per_s"] / base
    return out


def trk_step(gg, torch, seed, r, steps=3):
    """The mid step (sfm, c = 25, node + edge sums) with the TRK estimator."""
    gg.run(OPT, fixed_r=r, seed=seed + 999, c=C, edges=True, trk=True)
    torch.cuda.synchronize()
    tot = {"sweep_ms": 0.0, "launches": 0, "window_edges": 0, "arcs": 0, "touched_nodes": 0, "touched_edges": 0}
    t0 = time.perf_counter()
    for k in range(steps):
        gg.run(OPT, fixed_r=r, seed=seed + k, c=C, edges=True, trk=True)
        t = gg.last_timing()
        for key in tot:
            tot[key] += t[key]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return {"steps": steps, "pairs_per_s": r * steps / wall, "ms_per_step": wall * 1e3 / steps,
            "sweep_ms_per_launch": tot["sweep_ms"] / max(1, tot["launches"]), "hbm_frac": hbm_frac(tot, C),
            "kernel": "mantra::k_sweep<2, false>"}


def rtb_step(gg, torch, seed, r=0, steps=2):
    """The mid step's settings (sfm, c = 25, node + edge sums) with the RTB
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
            "hbm_frac": hbm_frac(tot, C), "kernel": "mantra::k_sweep<3, false>"}


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
            threads = host_threads()
            S = odist.draw_sources(seed, og.n, 32)
            t0 = time.perf_counter()
            odist.source_hops(og, opt, S, nthreads=threads)
            dt = time.perf_counter() - t0
            out[opt]["cpu_baseline"] = {"value": len(S) / dt, "unit": "sources/s", "cores": threads,
                                        "kind": "oracle",
                                        "sample": "first %d sources of the same source stream, %.1f s" % (len(S), dt)}
    return out


def serve(gg, G, torch, n_req=24, rate=50.0, seed=4002, workload_name=MID, deadline_s=0.0):
    """Poisson arrivals at `rate` req/s; each request a random window of
    5-100% of the span, a uniform optimality and eps in {0.01, 0.005}.
    Latencies are reported over every finished request (a request that fails
    finishes too) and over the completed ones, with their counts.  With a
    deadline, requests still running deadline_s after the first arrival are
    counted as unfinished (they fail when the graph is destroyed)."""
    import numpy as np
    from synthgen import request_stream
    reqs = request_stream(n_req, rate, int(G.t.min()), int(G.t.max()), seed)
    opts = ("sh", "fm", "sfm", "pfm")
    lat = [None] * n_req
    ok_ = [False] * n_req
    pairs = [0] * n_req
    t_start = time.perf_counter()

    def waiter(i, tk):
        ok = True
        res = None
        try:
            while res is None:
                if deadline_s > 0 and time.perf_counter() - t_start > deadline_s:
                    log("request %d unfinished at the deadline" % i)
                    return
                res = tk.poll(timeout_ms=1000 if deadline_s > 0 else -1)
        except Exception:  # noqa: BLE001 - a failed request finishes too (saturated fm counts)
            res = tk.result
            ok = False
        if res is not None:
            pairs[i] = res["samples"] + res["s_boot"]
            lat[i] = res["latency_ms"]
            ok_[i] = ok
            log("request %d (%s, eps %g, window %.0f%%) %s after %.0f ms, %d pairs" % (
                i, opts[reqs[i]["opt"]], reqs[i]["eps"],
                100.0 * (reqs[i]["t1"] - reqs[i]["t0"]) / max(1, int(G.t.max()) - int(G.t.min())),
                "done" if ok else "failed", res["latency_ms"], pairs[i]))

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
    wall = time.perf_counter() - t_start
    if deadline_s <= 0:
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
    La = np.array([x for x in lat if x is not None])
    Lc = np.array([x for x, o in zip(lat, ok_) if x is not None and o])

    def pct(L, q):
        return float(np.percentile(L, q)) if L.size else None

    return {"requests": n_req, "offered_req_per_s": rate, "finished": int(La.size), "completed": int(Lc.size),
            "failed": int(La.size - Lc.size), "unfinished": n_req - int(La.size),
            "deadline_s": deadline_s if deadline_s > 0 else None, "wall_s": wall,
            "completed_req_per_s": Lc.size / wall,
            "pairs_per_s": sum(pairs) / wall,
            "p50_ms": pct(La, 50), "p99_ms": pct(La, 99), "latency_of": "every finished request (failed ones too)",
            "p50_ms_completed": pct(Lc, 50), "p99_ms_completed": pct(Lc, 99),
            "failure": "fm walk counts past 2^64 (MANTRA_E_OVERFLOW at the end of the phase that saturated)",
            "workload": workload_name + ", windows/optimalities/eps of the serving recipe"}


def mid_sections(args, pk, torch):
    from synthgen import workload
    G = workload(MID)
    gg = pk.Graph.of(G)
    log("%s resident" % MID)
    if args.mid_slabs > 0:
        # a fixed grid (profiling runs): no autotuner launches in the profile
        gg.set_launch(n_slabs=args.mid_slabs, hub_nodes=args.mid_hub)
        tuned = gg.get_launch()
    else:
        tuned = gg.autotune(OPT, sample_pairs=MID_R, seed=args.seed + 7)
    tot, wall, bal = timed_steps(gg, torch, OPT, MID_R, max(3, args.steps // 4), 1, args.seed)
    steps = max(3, args.steps // 4)
    out = {"workload": MID, "n": G.n, "edges": G.m, "optimality": OPT, "pairs_per_step": MID_R, "c": C,
           "steps": steps, "pairs_per_s": MID_R * steps / wall, "ms_per_step": wall * 1e3 / steps,
           "temporal_edges_per_s": tot["window_edges"] / wall, "mean_window_edges": tot["window_edges"] / (MID_R * steps),
           "mean_arcs": tot["arcs"] / (MID_R * steps), "grid_balance": bal, "launch": tuned,
           "roofline": roofline(tot, MID, tuned, "mantra::k_sweep<0, false> (LDS bitmap)", MID_R)}
    log("mid: %s" % json.dumps(out))
    if not args.no_forms:
        out["forms"] = forms(gg, torch, args.seed, tuned)
        log("forms: %s" % json.dumps(out["forms"]))
    if not args.no_serve:
        out["serve"] = serve(gg, G, torch, n_req=args.serve_requests, rate=args.serve_rate)
    og = None
    if not args.no_cpu_baseline:
        import oracle
        og = oracle.Graph.of(G)
    if not args.no_trk:
        out["trk"] = trk_step(gg, torch, args.seed, MID_R)
    if not args.no_rtb:
        out["rtb"] = rtb_step(gg, torch, args.seed)
    if not args.no_distances:
        out["distances"] = distances(gg, torch, args.seed, og=og)
    if og is not None:
        out["cpu_baseline"] = cpu_baseline(og, G.n, args.seed, OPT, t_budget=15.0)
        log("mid cpu_baseline: %s" % json.dumps(out["cpu_baseline"]))
    return out


def tiny_section(args, pk, torch):
    """The plain method on tiny-uniform-n100 (n = 100, |E| = 2,000): exact
    all-pairs sh (9,900 pairs) and 500 sampled pairs on the GPU, and the
    oracle on the same all pairs on every host thread and on one."""
    import numpy as np
    from synthgen import workload
    G = workload("tiny-uniform-n100")
    gg = pk.Graph.of(G)
    n = G.n
    S = np.array([s for s in range(n) for z in range(n) if s != z], dtype=np.int32)
    Z = np.array([z for s in range(n) for z in range(n) if s != z], dtype=np.int32)
    gg.count_pairs("sh", S[:64], Z[:64])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gg.count_pairs("sh", S, Z)
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t0
    t0 = time.perf_counter()
    gg.run("sh", fixed_r=500, seed=args.seed, c=C, edges=True)
    torch.cuda.synchronize()
    t_500 = time.perf_counter() - t0
    out = {"workload": "tiny-uniform-n100", "n": n, "edges": G.m, "optimality": "sh",
           "all_pairs": int(S.size), "all_pairs_s": t_all, "all_pairs_per_s": S.size / t_all,
           "sampled_500_s": t_500}
    if not args.no_cpu_baseline:
        import oracle
        og = oracle.Graph.of(G)
        th = host_threads()
        t0 = time.perf_counter()
        oracle.accumulate(og, "sh", S, Z, mode=1, nthreads=th)
        dt = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.accumulate(og, "sh", S, Z, mode=1, nthreads=1)
        dt1 = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": S.size / dt, "unit": "pairs/s", "cores": th, "kind": "oracle",
                               "cpu_model": cpu_model(), "value_1_thread": S.size / dt1,
                               "sample": "all %d ordered pairs (records and node sums), %.2f s on %d threads, "
                                         "%.2f s on one" % (S.size, dt, th, dt1)}
    log("tiny: %s" % json.dumps(out))
    return out


# ------------------------------------------------------------------ other modes


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
        log("%s: %s" % (key, json.dumps(d)))

    t0 = time.perf_counter()
    gs = workload("packed-256")
    pg = pk.Graph.packed(gs)
    log("packed-256 resident after %.1f s" % (time.perf_counter() - t0))
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
    log("big-chunglu-n1m resident after %.1f s" % (time.perf_counter() - t0))
    gg.set_launch(graph_rounds=True)
    t0 = time.perf_counter()
    tuned = gg.autotune("pfm", seed=seed + 7)
    log("autotuned in %.1f s: %s" % (time.perf_counter() - t0, json.dumps(tuned)))

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
    ap.add_argument("--no-mid", action="store_true", help="skip the mid-size workload's sections")
    ap.add_argument("--no-optimalities", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-distances", action="store_true")
    ap.add_argument("--no-trk", action="store_true")
    ap.add_argument("--no-rtb", action="store_true")
    ap.add_argument("--serve-only", action="store_true",
                    help="only the serving measurement, on --serve-workload (prints {\"serve\": ...})")
    ap.add_argument("--serve-workload", default=MID)
    ap.add_argument("--serve-requests", type=int, default=24)
    ap.add_argument("--serve-rate", type=float, default=50.0)
    ap.add_argument("--serve-deadline", type=float, default=0.0,
                    help="seconds after the first arrival at which running requests count as unfinished")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--batching", action="store_true",
                    help="only the batching workloads (n = 10^6 Algorithm 1, packed-256; prints {\"batching\": ...})")
    ap.add_argument("--slabs", type=int, default=0,
                    help="fixed number of persistent workgroups for the headline step (profiling runs)")
    ap.add_argument("--mid-slabs", type=int, default=0,
                    help="fixed grid for the mid-size step instead of the autotuner's (profiling runs)")
    ap.add_argument("--mid-hub", type=int, default=0, help="hub nodes of the fixed mid-size grid (with --mid-slabs)")
    ap.add_argument("--seed", type=int, default=2005)
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
        if args.serve_workload == WORKLOAD:
            gg.set_launch(**HEADLINE_LAUNCH)
        log("graph %s resident after %.1f s" % (args.serve_workload, time.perf_counter() - t0))
        out = serve(gg, G, torch, n_req=args.serve_requests, rate=args.serve_rate, seed=args.seed + 2000,
                    workload_name=args.serve_workload, deadline_s=args.serve_deadline)
        print(json.dumps({"serve": out}), flush=True)
        # requests still running fail here (the graph is destroyed)
        del gg
        return
    t0 = time.perf_counter()
    G = workload(WORKLOAD)
    log("%s generated after %.1f s" % (WORKLOAD, time.perf_counter() - t0))
    gg = pk.Graph.of(G)
    log("%s resident after %.1f s" % (WORKLOAD, time.perf_counter() - t0))
    launch = dict(HEADLINE_LAUNCH)
    if args.slabs > 0:
        launch["n_slabs"] = args.slabs
    gg.set_launch(**launch)
    tuned = gg.get_launch()
    tot, wall, bal = timed_steps(gg, torch, OPT, R_PER_STEP, args.steps, args.warmup, args.seed)
    pairs = R_PER_STEP * args.steps
    out = {
        "metric": METRIC,
        "value": pairs / wall,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64 counts, f64 sums",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "n": G.n, "edges": G.m, "ticks": 1_000_000, "optimality": OPT,
                   "window": "whole span", "pairs_per_step": R_PER_STEP, "c": C, "edge_betweenness": True},
        "temporal_edges_per_s": tot["window_edges"] / wall,
        "mean_window_edges": tot["window_edges"] / pairs,
        "mean_arcs": tot["arcs"] / pairs,
        "sweep_ms_per_launch": tot["sweep_ms"] / max(1, tot["launches"]),
        "launches_per_step": tot["launches"] / args.steps,
        "grid_balance": bal,
        "launch": tuned,
        "roofline": roofline(tot, WORKLOAD, tuned, "mantra::k_sweep<0, true> (reached set in global memory)",
                             R_PER_STEP),
    }
    tot_s, wall_s, bal_s = timed_steps(gg, torch, OPT, R_SMALL, 3, 0, args.seed)
    out["steps_of_%d_pairs" % R_SMALL] = {
        "steps": 3, "pairs_per_s": R_SMALL * 3 / wall_s, "ms_per_step": wall_s * 1e3 / 3,
        "sweep_ms_per_launch": tot_s["sweep_ms"] / max(1, tot_s["launches"]), "grid_balance": bal_s}
    log("headline: %s" % json.dumps(out))
    og = one = None
    if not args.no_cpu_baseline:
        import oracle
        og = oracle.Graph.of(G)
        one = OracleOneThread(og, G.n, args.seed, OPT)
        one.start()
    if not args.no_optimalities:
        out["optimalities"] = optimalities(gg, torch, args.seed, (("pfm", 4096), ("sh", 1024), ("fm", 1024)))
        out["plain"] = plain_fixed(gg, torch, OPT, 16, args.seed, tuned)
        out["plain"]["speedup_of_step"] = out["value"] / out["plain"]["pairs_per_s"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(og, G.n, args.seed, OPT, one=one)
        log("cpu_baseline: %s" % json.dumps(out["cpu_baseline"]))
    del gg, G, og
    if not args.no_mid:
        out["mid"] = mid_sections(args, pk, torch)
        out["tiny"] = tiny_section(args, pk, torch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
