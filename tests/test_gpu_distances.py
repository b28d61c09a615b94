"""GPU parity of Algorithm 2 (sampled temporal distance metrics): the
library's single-source sweep, through the C ABI, against the oracle.

Bit-exact: the per-hop counts of the sampled (source, node) pairs, D_LB and
D_tau (the same fp64 test on the same integer counts); 1e-12 relative:
zeta, Psi and rho.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import distances as od
from parity_util import OPTS, compare_pairs
from synthgen import chung_lu_graph, uniform_graph, workload
from test_oracle_brute import tiny_graph

pytestmark = pytest.mark.gpu
T_MAX = 2**31 - 1


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need the MI355X"
    import paper_2304_08356_amd as pk
    return pk


def both(pk, G):
    return pk.Graph.of(G), oracle.Graph.of(G)


def close(a, b, rel=1e-12):
    return a == b or abs(a - b) <= rel * max(abs(a), abs(b))


def check(gg, og, opt, r, seed, tau=0.9, t0=0, t1=T_MAX, hist_len=None, ctx=""):
    counts, want = od.distances(og, opt, r, seed, tau, t0, t1)
    L = hist_len or (want["d_lb"] + 2)
    hist, got = gg.distances(opt, r, seed=seed, tau=tau, t0=t0, t1=t1, hist_len=L)
    c = (ctx, opt, r, seed, tau, t0, t1)
    assert hist.tolist() == od.hist_of(counts, L).tolist(), c
    for k in ("sources", "reached_pairs", "d_lb", "d_tau"):
        assert got[k] == want[k], (k, got, want, c)
    for k in ("zeta", "psi", "rho"):
        assert close(got[k], want[k]), (k, got, want, c)
    return got


def test_tiny_random_graphs(lib):
    from synthgen.graphs import TemporalGraph
    for seed in range(25):
        rng = np.random.default_rng(4000 + seed)
        n, src, dst, t = tiny_graph(rng)
        gg, og = both(lib, TemporalGraph(n, src, dst, t))
        for opt in OPTS:
            check(gg, og, opt, 3 * n, seed, tau=0.5, ctx="tiny%d" % seed)
            check(gg, og, opt, 2 * n, seed + 1, tau=1.0, t0=2, t1=4, ctx="tiny-win%d" % seed)


def test_line_closed_form(lib):
    from synthgen.graphs import TemporalGraph
    n = 40
    src = np.arange(n - 1, dtype=np.int32)
    G = TemporalGraph(n, src, src + 1, src + 1)
    gg, og = both(lib, G)
    for opt in OPTS:
        got = check(gg, og, opt, 500, 3, tau=1.0, ctx="line")
        assert got["d_lb"] <= n - 1
    # every source once is not what the sampler does; the estimate is still
    # close to the closed forms zeta = 1/2, Psi = (n + 1) / 3
    _, res = gg.distances("sh", 20000, seed=1)
    assert abs(res["zeta"] - 0.5) < 0.02 and abs(res["psi"] - (n + 1) / 3.0) < 0.5


@pytest.fixture(scope="module")
def tiny_workload(lib):
    G = workload("tiny-uniform-n100")
    return G, lib.Graph.of(G), oracle.Graph.of(G)


@pytest.mark.parametrize("opt", OPTS)
def test_tiny_workload(tiny_workload, opt):
    G, gg, og = tiny_workload
    for tau in (0.0, 0.5, 0.9, 1.0):
        check(gg, og, opt, 256, 2001, tau=tau, ctx="n100")
    check(gg, og, opt, 300, 7, t0=20, t1=60, ctx="n100-win")
    check(gg, og, opt, 100, 8, hist_len=2, ctx="n100-clamp")


@pytest.mark.parametrize("opt", OPTS)
def test_two_row_ticks(lib, opt):
    """Ticks of 57..168 edges: one row, two rows (in registers), longer."""
    for n, m, T, seed in ((12, 1000, 10, 61), (30, 1300, 10, 64), (20, 1800, 12, 65)):
        gg, og = both(lib, uniform_graph(n, m, T, seed=seed))
        check(gg, og, opt, 60, seed, ctx="rows%d" % seed)
        check(gg, og, opt, 60, seed, t0=2, t1=T - 2, ctx="rows-win%d" % seed)


@pytest.mark.parametrize("opt", OPTS)
def test_long_ticks_and_star(lib, opt):
    """Ticks far longer than a batch (the global-scratch tick) and a head
    with 600 in-edges at one time."""
    G = uniform_graph(80, 4000, 6, seed=77)
    gg, og = both(lib, G)
    check(gg, og, opt, 200, 5, ctx="bigtick")
    rng = np.random.default_rng(3)
    n = 700
    src = list(range(1, 601)) + list(rng.integers(0, n, 400))
    dst = [0] * 600 + list(rng.integers(0, n, 400))
    t = [5] * 600 + list(rng.integers(1, 10, 400))
    tr = {}
    for u, v, tt in zip(src, dst, t):
        if u != v:
            tr[(int(u), int(v), int(tt))] = 1
    a = np.array(list(tr.keys()), dtype=np.int32)
    from synthgen.graphs import TemporalGraph
    gs, os_ = both(lib, TemporalGraph(n, a[:, 0].copy(), a[:, 1].copy(), a[:, 2].copy()))
    check(gs, os_, opt, 300, 9, ctx="star")


@pytest.mark.parametrize("opt", OPTS)
def test_hub_state_in_lds(lib, opt):
    H = chung_lu_graph(3000, 60_000, 2.3, 4000, seed=91, times="pareto")
    hg, ho = both(lib, H)
    check(hg, ho, opt, 64, 94, ctx="cl")
    for K in (256, 1024):
        hg.set_launch(hub_nodes=K)
        check(hg, ho, opt, 64, 94, ctx="cl-hub%d" % K)
    G = uniform_graph(80, 4000, 6, seed=77)
    gg, og = both(lib, G)
    gg.set_launch(hub_nodes=40)
    check(gg, og, opt, 100, 6, ctx="bigtick-hub")


def test_launch_configs_same_results(tiny_workload):
    G, gg, og = tiny_workload
    base = gg.distances("sfm", 400, seed=12)
    try:
        for cfg in (dict(n_slabs=3), dict(n_slabs=17, order="drawn"), dict(per_pair_launch=True),
                    dict(hub_nodes=32)):
            gg.set_launch(**cfg)
            h, r = gg.distances("sfm", 400, seed=12)
            assert h.tolist() == base[0].tolist(), cfg
            for k in ("d_lb", "d_tau", "zeta", "psi", "rho", "reached_pairs"):
                assert r[k] == base[1][k], (cfg, k)
    finally:
        gg.set_launch()


def test_pairs_after_distances(tiny_workload):
    """The distance sweep leaves the slabs' per-node scratch as the pair
    sweep expects it: pair records and f(v), f(e) stay bit-exact."""
    G, gg, og = tiny_workload
    S, Z = oracle.draw_pairs(31, oracle.STREAM_PAIR, G.n, 0, 200)
    for opt in OPTS:
        gg.distances(opt, 500, seed=30)
        compare_pairs(gg, og, opt, S, Z, ctx="after-" + opt)


@pytest.fixture(scope="module")
def mid_workload(lib):
    G = workload("mid-chunglu-n50k")
    return G, lib.Graph.of(G), oracle.Graph.of(G)


@pytest.mark.parametrize("opt,r", [("sfm", 48), ("sh", 16), ("fm", 16), ("pfm", 16)])
def test_mid_workload(mid_workload, opt, r):
    """Full size (n = 50,000, |E| = 2,000,000, bursty ticks)."""
    G, gg, og = mid_workload
    check(gg, og, opt, r, 2002, ctx="mid")


def test_hops_limit(lib):
    """A cycle of 65,536 nodes run twice in increasing time: every source
    reaches its predecessor at 65,535 hops, above the limit (E_LIMIT); the
    same graph in a short window afterwards is exact."""
    from synthgen.graphs import TemporalGraph
    n = 65536
    i = np.arange(2 * n, dtype=np.int64)
    G = TemporalGraph(n, (i % n).astype(np.int32), ((i + 1) % n).astype(np.int32), (i + 1).astype(np.int32))
    gg, og = both(lib, G)
    with pytest.raises(lib.MantraError) as e:
        gg.distances("sh", 2, seed=1)
    assert e.value.code == -7
    check(gg, og, "sh", 8, 1, t0=0, t1=3000, ctx="cycle-window")


def test_validation(lib):
    G = workload("tiny-uniform-n100")
    gg = lib.Graph.of(G)
    for kw in (dict(r=0), dict(r=2**31), dict(tau=1.5), dict(tau=-0.1), dict(opt=7)):
        args = dict(opt="sh", r=10, seed=0, tau=0.5)
        args.update(kw)
        with pytest.raises(lib.MantraError):
            gg.distances(**args)
    pk = lib.Graph.packed([uniform_graph(20, 60, 10, seed=1), uniform_graph(30, 90, 10, seed=2)])
    with pytest.raises(lib.MantraError):
        pk.distances("sh", 10)
    # no histogram buffer
    h, res = gg.distances("sh", 10, hist_len=0)
    assert h.size == 0 and res["sources"] == 10 and math.isfinite(res["psi"])
