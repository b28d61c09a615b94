"""Serving: requests submitted together share sweep launches (continuous
batching of their progressive-sampling rounds); each result must be the one
the request gets alone (bit-identical sample schedule, sums within 1e-12
relative) and, on the tiny workload, the oracle's Algorithm 1."""
import threading
import time

import numpy as np
import pytest

import oracle
from oracle import mantra as omantra
from parity_util import rel_close
from synthgen import chung_lu_graph, workload

pytestmark = pytest.mark.gpu

EXACT_KEYS = ("samples", "rounds", "omega", "s_boot", "s1", "n_reachable", "n_overflow", "flags")


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need the MI355X"
    import paper_2304_08356_amd as pk
    return pk


@pytest.fixture(scope="module")
def tiny(lib):
    G = workload("tiny-uniform-n100")
    return G, lib.Graph.of(G), oracle.Graph.of(G)


@pytest.fixture(scope="module")
def small_cl(lib):
    G = chung_lu_graph(4000, 80_000, 2.3, 5000, seed=77, times="pareto")
    return G, lib.Graph.of(G)


def same_result(alone, mixed, ctx):
    (nb_a, eb_a, ra), (nb_m, eb_m, rm) = alone, mixed
    assert ra["rc"] == rm["rc"], (ctx, ra["rc"], rm["rc"])
    for k in EXACT_KEYS:
        assert ra[k] == rm[k], (ctx, k, ra[k], rm[k])
    if ra["rc"] != 0:
        return
    assert abs(ra["xi"] - rm["xi"]) <= 1e-12 * abs(ra["xi"]) + 1e-300, ctx
    ok, worst = rel_close(nb_a, nb_m, rel=1e-12, abs_floor=1e-300)
    assert ok, (ctx, worst)
    if eb_a is not None:
        ok, worst = rel_close(eb_a, eb_m, rel=1e-12, abs_floor=1e-300)
        assert ok, (ctx, "edges", worst)


def submit_all(gg, reqs, lib=None):
    import paper_2304_08356_amd as pk
    tickets = [gg.submit(**r) for r in reqs]
    out = []
    for tk in tickets:
        try:
            tk.poll(timeout_ms=-1)
        except pk.MantraError as e:
            assert e.code == -4 and tk.result is not None, e  # saturated counts: reported, not rounded
        out.append((tk.node_bc, tk.edge_bc, tk.result))
    return out


def test_served_mix_matches_oracle_tiny(tiny):
    """The four optimalities served together, each against the oracle's
    Algorithm 1 on the same seed."""
    G, gg, og = tiny
    reqs = [dict(opt=o, eps=0.03, delta=0.1, seed=7 + i, c=16) for i, o in enumerate(("sh", "fm", "sfm", "pfm"))]
    got = submit_all(gg, reqs)
    for r, (nb, _, res) in zip(reqs, got):
        ref = omantra.estimate(og, r["opt"], 0.03, 0.1, r["seed"], c=16, mode=0)
        assert res["status"] == 0
        assert res["s_boot"] == ref["s_boot"] and res["omega"] == ref["omega"] and res["s1"] == ref["s1"]
        assert res["samples"] == ref["samples"] and res["rounds"] == len(ref["rounds"]), r
        ok, worst = rel_close(nb, ref["node_bc"], rel=1e-12, abs_floor=1e-300)
        assert ok, (r, worst)
        assert res["latency_ms"] > 0


def test_alone_vs_mixed(small_cl):
    """Mixed windows, optimalities, accuracies, fixed and progressive
    requests: served together == run alone."""
    G, gg = small_cl
    span = (int(G.t.min()), int(G.t.max()))
    mid = (span[0] + span[1]) // 2
    reqs = [
        dict(opt="sh", eps=0.05, delta=0.1, seed=101, c=16),
        dict(opt="sfm", eps=0.04, delta=0.1, seed=102, c=25, t0=span[0], t1=mid, edges=True),
        dict(opt="pfm", eps=0.05, delta=0.1, seed=103, c=8, t0=mid // 2, t1=span[1]),
        dict(opt="fm", fixed_r=900, seed=104, c=4, edges=True, t0=span[0], t1=span[0] + (span[1] - span[0]) // 5),
        dict(opt="fm", fixed_r=900, seed=107, c=4, t0=span[0], t1=span[0] + (span[1] - span[0]) // 20),
        # fm walk counts over the whole span pass 2^64 (the multiword path is
        # off for fm by default): the request fails with MANTRA_E_OVERFLOW
        dict(opt="fm", fixed_r=900, seed=108, c=4),
        dict(opt="sfm", fixed_r=3000, seed=105, c=25),
        dict(opt="sh", eps=0.08, delta=0.05, seed=106, c=25, t0=mid, t1=span[1], edges=True),
    ]
    alone = [gg.run(**r, raise_on_error=False) for r in reqs]
    for r, a in zip(reqs, alone):
        want = -4 if (r["opt"] == "fm" and "t0" not in r) else 0
        assert a[2]["rc"] == want, (r, a[2])
        if want == 0:
            assert a[2]["n_overflow"] == 0, (r, a[2])
        else:
            assert a[2]["n_overflow"] > 0 and np.all(np.isnan(a[0])), (r, a[2])
    mixed = submit_all(gg, reqs)
    for i, r in enumerate(reqs):
        same_result(alone[i], mixed[i], ctx=r)


def test_admission_by_memory(small_cl, lib):
    """A budget that holds one request at a time still serves a burst
    (admitted one by one), and a request that can never fit is rejected."""
    G, gg = small_cl
    c = 16
    one = 8 * gg.n * (2 + c) + 8 * gg.n * 3 + 64
    reqs = [dict(opt=o, eps=0.06, delta=0.1, seed=300 + i, c=c) for i, o in enumerate(("sh", "sfm", "pfm", "sfm"))]
    alone = [gg.run(**r) for r in reqs]
    gg.serve_config(mem_budget_bytes=one + 1024, max_active=8)
    try:
        with pytest.raises(lib.MantraError) as ei:
            gg.submit(opt="sh", eps=0.06, delta=0.1, seed=1, c=64)
        assert ei.value.code == -5
        mixed = submit_all(gg, reqs)
        for i, r in enumerate(reqs):
            same_result(alone[i], mixed[i], ctx=r)
        # latencies grow along the queue: request k waited for k-1 others
        lat = [m[2]["latency_ms"] for m in mixed]
        assert lat[-1] >= lat[0]
    finally:
        gg.serve_config(0, 0)


def test_poll_semantics(tiny, lib):
    G, gg, og = tiny
    tk = gg.submit("sfm", fixed_r=200, seed=5, c=4)
    res = None
    t_end = time.time() + 60
    while res is None and time.time() < t_end:
        res = tk.poll(timeout_ms=0)
        if res is None:
            time.sleep(0.001)
    assert res is not None and res["status"] == 0 and res["samples"] == 200
    with pytest.raises(lib.MantraError) as ei:
        tk.poll(timeout_ms=0)  # consumed
    assert ei.value.code == -1
    with pytest.raises(lib.MantraError):
        gg.submit("sh", eps=1.5, delta=0.1, seed=1)
    # the served fixed sample equals the blocking one
    nb, _, _ = gg.run("sfm", fixed_r=200, seed=5, c=4)
    ok, worst = rel_close(nb, tk.node_bc, rel=1e-12, abs_floor=1e-300)
    assert ok, worst


def test_concurrent_submitters(small_cl):
    """Requests arriving from several threads while others run."""
    G, gg = small_cl
    reqs = [dict(opt=o, fixed_r=400 + 50 * i, seed=500 + i, c=8) for i, o in
            enumerate(("sh", "pfm", "sfm", "pfm", "sh", "sfm"))]
    alone = [gg.run(**r) for r in reqs]
    out = [None] * len(reqs)

    def worker(i):
        time.sleep(0.01 * i)
        tk = gg.submit(**reqs[i])
        res = tk.poll(timeout_ms=-1)
        out[i] = (tk.node_bc, tk.edge_bc, res)

    th = [threading.Thread(target=worker, args=(i,)) for i in range(len(reqs))]
    for t in th:
        t.start()
    for t in th:
        t.join(timeout=120)
    for i, r in enumerate(reqs):
        assert out[i] is not None, r
        same_result(alone[i], out[i], ctx=r)


def test_destroy_with_pending_requests(lib):
    """Destroying a graph fails what it still holds, and poll reports it."""
    G = chung_lu_graph(2000, 40_000, 2.3, 3000, seed=78, times="pareto")
    gg = lib.Graph.of(G)
    tks = [gg.submit("sh", fixed_r=2000, seed=i, c=4) for i in range(4)]
    gg.close()
    for tk in tks:
        try:
            res = tk.poll(timeout_ms=-1)
            assert res["status"] == 0  # finished before the destroy
        except lib.MantraError as e:
            assert e.code == -6
