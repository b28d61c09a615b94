"""GPU parity of the RTB estimator (appendix on other estimators): the
library's single-source sweep with the all-targets reverse in double
precision, through the C ABI, against the oracle's sum over targets.

Records (reached targets) are exact; f(v|s) and f(e|s) agree to 1e-12
relative (the library sums by a recursion over the appearance DAG, the
oracle target by target); the estimator sums of fixed samples and
Algorithm 1's schedule likewise.
"""
import numpy as np
import pytest

import oracle
from oracle import rtb
from parity_util import OPTS, rel_close
from synthgen import chung_lu_graph, uniform_graph, workload
from test_oracle_brute import tiny_graph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need the MI355X"
    import paper_2304_08356_amd as pk
    return pk


def both(pk, G):
    return pk.Graph.of(G), oracle.Graph.of(G)


def compare_sources(gg, og, opt, S, t0=0, t1=2**31 - 1, ctx="", mode=0):
    S = np.asarray(S, dtype=np.int32)
    rec, nf, ef = gg.source_dependencies(opt, S, t0=t0, t1=t1)
    for q, s in enumerate(S):
        wn, we, reached, sat = rtb.source(og, opt, int(s), t0, t1, mode=mode)
        c = (ctx, opt, q, int(s))
        assert int(rec["flags"][q]) & 2 == 0, ("origin self-check", c)
        assert int(rec["reachable"][q]) == (1 if reached else 0), c
        assert int(rec["sigma"][q]) == reached, c
        assert (int(rec["flags"][q]) & 1) == (1 if sat else 0), c
        ok, worst = rel_close(nf[q], wn, rel=1e-12)
        assert ok, (c, "node f", worst)
        ok, worst = rel_close(ef[q], we, rel=1e-12)
        assert ok, (c, "edge f", worst)
    return rec


def test_tiny_random_graphs(lib):
    from synthgen.graphs import TemporalGraph
    for seed in range(20):
        rng = np.random.default_rng(7000 + seed)
        n, src, dst, t = tiny_graph(rng)
        gg, og = both(lib, TemporalGraph(n, src, dst, t))
        for opt in OPTS:
            compare_sources(gg, og, opt, np.arange(n), ctx="tiny%d" % seed)
            compare_sources(gg, og, opt, np.arange(n), t0=2, t1=5, ctx="tiny-win%d" % seed)


def test_line(lib):
    from synthgen.graphs import TemporalGraph
    n = 30
    src = np.arange(n - 1, dtype=np.int32)
    gg, og = both(lib, TemporalGraph(n, src, src + 1, src + 1))
    for opt in OPTS:
        rec, nf, _ = gg.source_dependencies(opt, np.arange(n))
        for s in range(n):
            want = np.array([(n - 1 - v) / (n - 1) if v > s else 0.0 for v in range(n)])
            assert np.allclose(nf[s], want, rtol=1e-13, atol=0), (opt, s)


@pytest.fixture(scope="module")
def tiny_workload(lib):
    G = workload("tiny-uniform-n100")
    return G, lib.Graph.of(G), oracle.Graph.of(G)


@pytest.mark.parametrize("opt", OPTS)
def test_tiny_workload_sources(tiny_workload, opt):
    G, gg, og = tiny_workload
    compare_sources(gg, og, opt, np.arange(0, G.n, 7), ctx="n100")
    compare_sources(gg, og, opt, np.arange(0, G.n, 13), t0=20, t1=60, ctx="n100-win")


@pytest.mark.parametrize("opt", OPTS)
def test_two_row_ticks(lib, opt):
    """Ticks of 57..168 edges: one row, two rows (in registers), longer."""
    for n, m, T, seed in ((12, 1000, 10, 61), (30, 1300, 10, 64), (20, 1800, 12, 65)):
        gg, og = both(lib, uniform_graph(n, m, T, seed=seed))
        compare_sources(gg, og, opt, np.arange(0, n, 3), ctx="rows%d" % seed)
        gg.set_launch(hub_nodes=8)
        compare_sources(gg, og, opt, np.arange(1, n, 4), ctx="rows-hub%d" % seed)


@pytest.mark.parametrize("opt", OPTS)
def test_long_ticks_and_hubs(lib, opt):
    G = uniform_graph(80, 4000, 6, seed=77)
    gg, og = both(lib, G)
    compare_sources(gg, og, opt, np.arange(0, 80, 9), ctx="bigtick")
    gg.set_launch(hub_nodes=40)
    compare_sources(gg, og, opt, np.arange(0, 80, 9), ctx="bigtick-hub")
    H = chung_lu_graph(600, 9_000, 2.3, 1500, seed=93, times="pareto")
    hg, ho = both(lib, H)
    S = oracle.draw_pairs(95, oracle.STREAM_PAIR, H.n, 0, 4)[0]
    compare_sources(hg, ho, opt, S, ctx="cl", mode=1)
    for K in (128, 1024):
        hg.set_launch(hub_nodes=K)
        compare_sources(hg, ho, opt, S, ctx="cl-hub%d" % K, mode=1)


def test_launch_forms_and_arc_retry(tiny_workload):
    G, gg, og = tiny_workload
    S = np.arange(0, G.n, 11)
    try:
        for cfg in (dict(n_slabs=3), dict(per_pair_launch=True), dict(n_slabs=16, arc_cap=1024)):
            gg.set_launch(**cfg)
            compare_sources(gg, og, "sh", S, ctx=str(cfg))
            compare_sources(gg, og, "pfm", S, ctx=str(cfg))
    finally:
        gg.set_launch()


def test_fixed_sample_sums(tiny_workload):
    G, gg, og = tiny_workload
    r = 60
    for opt in ("sh", "sfm"):
        nb, eb, res = gg.run(opt, fixed_r=r, seed=2001, c=25, edges=True, rtb=True)
        want = rtb.fixed(og, opt, r, 2001, c=25, edges=True)
        ok, worst = rel_close(nb, want["node_bc"], rel=1e-12, abs_floor=1e-300)
        assert ok, (opt, worst)
        ok, worst = rel_close(eb, want["edge_bc"], rel=1e-12, abs_floor=1e-300)
        assert ok, (opt, worst)


def test_progressive_rtb(tiny_workload):
    """Algorithm 1 with the RTB estimator: the same schedule and estimates."""
    G, gg, og = tiny_workload
    nb, _, res = gg.run("sh", eps=0.05, delta=0.1, seed=2001, c=25, rtb=True)
    want = rtb.estimate(og, "sh", 0.05, 0.1, 2001, c=25)
    assert (res["s_boot"], res["omega"], res["s1"], res["samples"], res["rounds"]) == (
        want["s_boot"], want["omega"], want["s1"], want["samples"], want["rounds"])
    ok, worst = rel_close(nb, want["node_bc"], rel=1e-12, abs_floor=1e-300)
    assert ok, worst


def test_served_mix_with_rtb(tiny_workload):
    G, gg, og = tiny_workload
    a = gg.submit("pfm", fixed_r=50, seed=7, c=25, rtb=True)
    b = gg.submit("pfm", fixed_r=300, seed=7, c=25, trk=True)
    c = gg.submit("pfm", fixed_r=300, seed=7, c=25)
    for tk in (a, b, c):
        assert tk.poll(timeout_ms=-1)["rc"] == 0
    na, _, _ = gg.run("pfm", fixed_r=50, seed=7, c=25, rtb=True)
    ok, worst = rel_close(a.node_bc, na, rel=1e-12, abs_floor=1e-300)
    assert ok, worst
