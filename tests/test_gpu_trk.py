"""GPU parity of the TRK estimator (appendix on other estimators): the
library's walks, through the C ABI, against the oracle's path sampler on the
same pairs and draws.

Bit-exact: records, every walk's internal visits per node and uses per edge,
and the estimator sums (sums of small integers are exact in any order);
Algorithm 1 with the TRK estimator: the same schedule and the same
estimates.
"""
import numpy as np
import pytest

import oracle
from oracle import trk
from parity_util import OPTS
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


def compare_walks(gg, og, opt, S, Z, seed, t0=0, t1=2**31 - 1, ctx=""):
    S = np.asarray(S, dtype=np.int32)
    Z = np.asarray(Z, dtype=np.int32)
    rec, nf, ef = gg.sample_paths(opt, S, Z, seed=seed, t0=t0, t1=t1)
    for q in range(len(S)):
        want, nv, ev = trk.path(og, opt, int(S[q]), int(Z[q]), seed, q, oracle.STREAM_PAIR, t0, t1)
        got = {k: int(rec[k][q]) for k in ("reachable", "t_arr", "hops", "sigma")}
        c = (ctx, opt, q, int(S[q]), int(Z[q]), seed)
        assert int(rec["flags"][q]) & 2 == 0, ("walk self-check", c)
        assert got == {k: want[k] for k in got}, (c, got, want)
        assert (int(rec["flags"][q]) & 1) == (want["flags"] & 1), c
        assert np.array_equal(nf[q], nv.astype(np.float64)), (c, np.nonzero(nf[q])[0], np.nonzero(nv)[0])
        assert np.array_equal(ef[q], ev.astype(np.float64)), (c, np.nonzero(ef[q])[0], np.nonzero(ev)[0])
    return rec


def all_pairs(n):
    S, Z = zip(*[(s, z) for s in range(n) for z in range(n) if s != z])
    return np.array(S, dtype=np.int32), np.array(Z, dtype=np.int32)


def test_tiny_random_graphs(lib):
    from synthgen.graphs import TemporalGraph
    for seed in range(20):
        rng = np.random.default_rng(6000 + seed)
        n, src, dst, t = tiny_graph(rng)
        gg, og = both(lib, TemporalGraph(n, src, dst, t))
        S, Z = all_pairs(n)
        for opt in OPTS:
            compare_walks(gg, og, opt, S, Z, seed, ctx="tiny%d" % seed)
            compare_walks(gg, og, opt, S, Z, seed + 7, t0=2, t1=5, ctx="tiny-win%d" % seed)


@pytest.fixture(scope="module")
def tiny_workload(lib):
    G = workload("tiny-uniform-n100")
    return G, lib.Graph.of(G), oracle.Graph.of(G)


@pytest.mark.parametrize("opt", OPTS)
def test_tiny_workload_walks(tiny_workload, opt):
    G, gg, og = tiny_workload
    S, Z = oracle.draw_pairs(2001, oracle.STREAM_PAIR, G.n, 0, 300)
    compare_walks(gg, og, opt, S, Z, 41, ctx="n100")


@pytest.mark.parametrize("opt", OPTS)
def test_two_row_ticks(lib, opt):
    """Ticks of 57..168 edges: one row, two rows (in registers), longer."""
    for n, m, T, seed in ((12, 1000, 10, 61), (30, 1300, 10, 64), (20, 1800, 12, 65)):
        gg, og = both(lib, uniform_graph(n, m, T, seed=seed))
        S, Z = oracle.draw_pairs(seed, 0, n, 0, 80)
        compare_walks(gg, og, opt, S, Z, seed, ctx="rows%d" % seed)


@pytest.mark.parametrize("opt", OPTS)
def test_long_ticks_star_and_hubs(lib, opt):
    G = uniform_graph(80, 4000, 6, seed=77)
    gg, og = both(lib, G)
    S, Z = oracle.draw_pairs(5, 0, G.n, 0, 150)
    compare_walks(gg, og, opt, S, Z, 3, ctx="bigtick")
    gg.set_launch(hub_nodes=40)
    compare_walks(gg, og, opt, S, Z, 3, ctx="bigtick-hub")
    H = chung_lu_graph(3000, 60_000, 2.3, 4000, seed=91, times="pareto")
    hg, ho = both(lib, H)
    S, Z = oracle.draw_pairs(94, oracle.STREAM_PAIR, H.n, 0, 30)
    compare_walks(hg, ho, opt, S, Z, 5, ctx="cl")
    for K in (256, 1024):
        hg.set_launch(hub_nodes=K)
        compare_walks(hg, ho, opt, S, Z, 5, ctx="cl-hub%d" % K)


def test_launch_forms_and_arc_retry(tiny_workload):
    G, gg, og = tiny_workload
    S, Z = oracle.draw_pairs(11, 0, G.n, 0, 200)
    try:
        for cfg in (dict(n_slabs=7), dict(per_pair_launch=True), dict(n_slabs=32, arc_cap=1024)):
            gg.set_launch(**cfg)
            compare_walks(gg, og, "sh", S, Z, 9, ctx=str(cfg))
            compare_walks(gg, og, "fm", S, Z, 9, ctx=str(cfg))
    finally:
        gg.set_launch()


def test_fixed_sample_sums(tiny_workload):
    """r = 400 pairs, c = 25, node and edge sums: exactly the oracle's."""
    G, gg, og = tiny_workload
    r = 400
    for opt in ("sh", "pfm"):
        nb, eb, res = gg.run(opt, fixed_r=r, seed=2001, c=25, edges=True, trk=True)
        want = trk.fixed(og, opt, r, 2001, c=25, edges=True)
        assert np.array_equal(nb, want["node_bc"]), opt
        assert np.array_equal(eb, want["edge_bc"]), opt
        assert res["n_reachable"] == sum(1 for x in want["records"] if x["reachable"])


@pytest.mark.parametrize("opt", ["sh", "sfm", "pfm"])
def test_progressive_trk(tiny_workload, opt):
    """Algorithm 1 with the TRK estimator: schedule and estimates."""
    G, gg, og = tiny_workload
    nb, _, res = gg.run(opt, eps=0.05, delta=0.1, seed=2001, c=25, trk=True)
    want = trk.estimate(og, opt, 0.05, 0.1, 2001, c=25)
    assert (res["s_boot"], res["omega"], res["s1"], res["samples"], res["rounds"]) == (
        want["s_boot"], want["omega"], want["s1"], want["samples"], want["rounds"])
    assert np.array_equal(nb, want["node_bc"])
    assert abs(res["xi"] - want["xi"]) <= 1e-12 * max(1.0, abs(want["xi"]))


def test_mid_workload_walks(lib):
    """Full size (n = 50,000, |E| = 2,000,000): a few pairs per optimality
    (fm: saturated pairs draw no walk, as in the oracle)."""
    G = workload("mid-chunglu-n50k")
    gg, og = both(lib, G)
    S, Z = oracle.draw_pairs(2002, oracle.STREAM_PAIR, G.n, 0, 3)
    for opt in OPTS:
        compare_walks(gg, og, opt, S, Z, 2002, ctx="mid")


def test_served_mix_with_trk(tiny_workload, lib):
    """An ob and a TRK request served together: each equals its blocking run."""
    G, gg, og = tiny_workload
    a = gg.submit("sfm", fixed_r=300, seed=5, c=25, trk=True)
    b = gg.submit("sfm", fixed_r=300, seed=5, c=25)
    ra, rb = a.poll(timeout_ms=-1), b.poll(timeout_ms=-1)
    assert ra["rc"] == 0 and rb["rc"] == 0
    nt, _, _ = gg.run("sfm", fixed_r=300, seed=5, c=25, trk=True)
    no, _, _ = gg.run("sfm", fixed_r=300, seed=5, c=25)
    assert np.array_equal(a.node_bc, nt)
    assert np.allclose(b.node_bc, no, rtol=1e-12, atol=1e-300)
