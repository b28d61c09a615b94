"""GPU parity: the HIP library (through its C ABI) against the oracle.

Bit-exact: sigma, arrival, hops, flags and every per-pair f(v|s,z) and
f(e|s,z) (the same IEEE division of the same exact integers).  Sums: the
spec tolerance, 1e-12 relative (the Rademacher-weighted sums, which
cancel, are compared with an absolute floor of 1e-12 times sum f).
"""
import numpy as np
import pytest

import oracle
from oracle import mantra as omantra
from parity_util import OPTS, compare_pairs, rel_close
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


def all_pairs(n):
    S, Z = zip(*[(s, z) for s in range(n) for z in range(n) if s != z])
    return np.array(S, dtype=np.int32), np.array(Z, dtype=np.int32)


def test_tiny_random_graphs_all_pairs(lib):
    from synthgen.graphs import TemporalGraph
    for seed in range(40):
        rng = np.random.default_rng(seed)
        n, src, dst, t = tiny_graph(rng)
        gg, og = both(lib, TemporalGraph(n, src, dst, t))
        S, Z = all_pairs(n)
        for opt in OPTS:
            compare_pairs(gg, og, opt, S, Z, ctx="tiny%d" % seed)


def test_tiny_windows(lib):
    from synthgen.graphs import TemporalGraph
    for seed in range(15):
        rng = np.random.default_rng(500 + seed)
        n, src, dst, t = tiny_graph(rng, T_hi=7)
        t0 = int(rng.integers(1, 4))
        t1 = int(rng.integers(t0, 8))
        gg, og = both(lib, TemporalGraph(n, src, dst, t))
        S, Z = all_pairs(n)
        for opt in OPTS:
            compare_pairs(gg, og, opt, S, Z, t0, t1, ctx="win%d" % seed)


@pytest.fixture(scope="module")
def tiny_workload(lib):
    G = workload("tiny-uniform-n100")
    return G, lib.Graph.of(G), oracle.Graph.of(G)


def test_tiny_workload_all_pairs_sh(tiny_workload):
    """n = 100, |E| = 2000, t in [1, 100]: all 9,900 ordered pairs, sh."""
    G, gg, og = tiny_workload
    S, Z = all_pairs(G.n)
    compare_pairs(gg, og, "sh", S, Z, edges=False, ctx="C1-all")
    compare_pairs(gg, og, "sh", S[::19], Z[::19], edges=True, ctx="C1-edges")


@pytest.mark.parametrize("opt", ["fm", "sfm", "pfm"])
def test_tiny_workload_sampled(tiny_workload, opt):
    G, gg, og = tiny_workload
    S, Z = oracle.draw_pairs(2001, oracle.STREAM_PAIR, G.n, 0, 500)
    compare_pairs(gg, og, opt, S, Z, ctx="C1-" + opt)


@pytest.mark.parametrize("opt", OPTS)
def test_big_ticks(lib, opt):
    """Ticks far larger than one 256-edge batch: the global-scratch path."""
    G = uniform_graph(80, 4000, 6, seed=77)
    gg, og = both(lib, G)
    S, Z = oracle.draw_pairs(5, 0, G.n, 0, 300)
    compare_pairs(gg, og, opt, S, Z, ctx="bigtick")


# uniform graphs whose ticks hold 57..168 edges: ticks of one row, of two rows
# (held in registers), and longer (the global-scratch path); with 12 or 20
# nodes a head's run of edges crosses the rows' boundary
ROW_GRAPHS = ((12, 1000, 10, 61), (40, 700, 10, 62), (30, 1300, 10, 64), (20, 1800, 12, 65))


@pytest.mark.parametrize("opt", OPTS)
def test_two_row_ticks(lib, opt):
    for n, m, T, seed in ROW_GRAPHS:
        G = uniform_graph(n, m, T, seed=seed)
        gg, og = both(lib, G)
        S, Z = oracle.draw_pairs(seed, 0, G.n, 0, 150)
        compare_pairs(gg, og, opt, S, Z, ctx="rows%d" % seed)
        compare_pairs(gg, og, opt, S, Z, 2, T - 2, ctx="rows-win%d" % seed)
        gg.set_launch(hub_nodes=8)
        compare_pairs(gg, og, opt, S, Z, ctx="rows-hub%d" % seed)


@pytest.mark.parametrize("opt", OPTS)
def test_hub_star_tick(lib, opt):
    """One head with 600 in-edges at one time (a run longer than a batch)."""
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
    G = TemporalGraph(n, a[:, 0].copy(), a[:, 1].copy(), a[:, 2].copy())
    gg, og = both(lib, G)
    S, Z = oracle.draw_pairs(9, 0, n, 0, 400)
    compare_pairs(gg, og, opt, S, Z, ctx="star")


def test_saturation(lib):
    """16 hops x 16 parallel edges: 2^64 shortest paths, one past the 64-bit
    counts (the multiword path takes the pair: MANTRA_REC_WIDE, f exact);
    15 hops give exactly 2^60 in 64 bits."""
    edges = [(i, i + 1, 16 * i + j + 1) for i in range(16) for j in range(16)]
    a = np.array(edges, dtype=np.int32)
    from synthgen.graphs import TemporalGraph
    G = TemporalGraph(17, a[:, 0].copy(), a[:, 1].copy(), a[:, 2].copy())
    gg, og = both(lib, G)
    rec = compare_pairs(gg, og, "sh", [0, 3], [15, 12], ctx="sat")
    assert int(rec["sigma"][0]) == 2**60
    rec, nf, _ = gg.count_pairs("sh", [0], [16], node_f=True)
    assert int(rec["sigma"][0]) == 2**64 - 1 and int(rec["flags"][0]) == 16 and np.all(nf[0, 1:16] == 1.0)
    for opt in ("fm", "sfm", "pfm"):
        compare_pairs(gg, og, opt, [0, 0, 3], [16, 15, 12], ctx="sat-" + opt)


def test_duplicates_and_validation(lib):
    src = np.array([0, 0, 1, 1], dtype=np.int32)
    dst = np.array([1, 1, 2, 2], dtype=np.int32)
    t = np.array([1, 1, 2, 2], dtype=np.int32)
    g = lib.Graph(3, src, dst, t)
    info = g.info()
    assert info["m_unique"] == 2 and info["n_duplicates"] == 2
    rec, nf, ef = g.count_pairs("sh", [0], [2], node_f=True, edge_f=True)
    assert int(rec["sigma"][0]) == 1 and nf[0, 1] == 1.0
    assert list(ef[0]) == [1.0, 1.0, 1.0, 1.0]  # duplicates share their merged edge's value
    with pytest.raises(lib.MantraError):
        lib.Graph(3, np.array([0]), np.array([0]), np.array([1]))  # self-loop
    with pytest.raises(lib.MantraError):
        lib.Graph(3, np.array([0]), np.array([3]), np.array([1]))  # id out of range
    with pytest.raises(lib.MantraError):
        lib.Graph(3, np.array([0]), np.array([1]), np.array([-1]))  # negative time
    with pytest.raises(lib.MantraError):
        g.count_pairs("sh", [1], [1])  # s == z


def test_arc_chunks_and_retry(tiny_workload):
    """Pairs whose DAG arcs exceed the workgroup's own buffer take chunks of
    the launch's shared arc pool (one launch).  With 4 shared chunks for 32
    workgroups, the pairs that find none free run again after the launch on
    the same pool, no more of them at once than there are chunks (two
    launches).  With no shared chunks they are re-run with a full-window
    buffer (two launches).  Results are unchanged in every case."""
    G, gg, og = tiny_workload
    S, Z = oracle.draw_pairs(11, 0, G.n, 0, 300)
    try:
        for no_chunks, nch, launches in ((False, 0, 1), (False, 4, 2), (True, 0, 2)):
            gg.set_launch(n_slabs=32, arc_cap=64, no_arc_chunks=no_chunks, arc_chunks=nch)
            L = gg.get_launch()
            assert L["arc_cap"] == 64 and L["no_arc_chunks"] == int(no_chunks) and L["arc_chunks"] == nch
            compare_pairs(gg, og, "sh", S, Z, ctx="chunks%d-%d" % (no_chunks, nch))
            assert gg.last_timing()["launches"] == launches, (no_chunks, nch)
            compare_pairs(gg, og, "fm", S, Z, ctx="chunks-fm%d-%d" % (no_chunks, nch))
    finally:
        gg.set_launch(0, 0)


def test_stamp_wrap_guard(lib):
    """Slab state words are tagged with 32-bit pair serials that slabs carry
    across launches.  Seeded just below the wrap (after a first launch left
    tagged words in the slabs), and past half the range, the results still
    match the oracle: the library clears the tagged state before a serial
    could wrap."""
    from paper_2304_08356_amd import _lib
    G = uniform_graph(80, 4000, 6, seed=78)  # long ticks too
    gg, og = both(lib, G)
    S, Z = oracle.draw_pairs(6, 0, G.n, 0, 200)
    gg.set_launch(n_slabs=8)
    try:
        for opt in ("sh", "pfm"):
            compare_pairs(gg, og, opt, S, Z, ctx="stamps-before")
            for serial in (2**32 - 12, 2**31 + 6, 2**32 - 2):
                assert _lib._lib.mantra_debug_stamps(gg._h, serial) == 0
                compare_pairs(gg, og, opt, S, Z, ctx="stamps-%d" % serial)
    finally:
        gg.set_launch(0, 0)


@pytest.fixture(scope="module")
def mid_workload(lib):
    G = workload("mid-chunglu-n50k")
    return G, lib.Graph.of(G), oracle.Graph.of(G)


def test_mid_workload_shared_arc_chunks(mid_workload):
    """Full size with a small own arc buffer (4,096 arcs): most pairs write
    their arcs into shared chunks taken and given back across the launch."""
    G, gg, og = mid_workload
    S, Z = oracle.draw_pairs(2002, oracle.STREAM_PAIR, G.n, 0, 12)
    gg.set_launch(arc_cap=4096)
    try:
        compare_pairs(gg, og, "sfm", S, Z, mode=1, ctx="C2-chunks")
        assert gg.last_timing()["launches"] == 1
        compare_pairs(gg, og, "sh", S[:4], Z[:4], mode=1, edges=False, ctx="C2-chunks-sh")
    finally:
        gg.set_launch(0, 0)


def test_mid_workload_sampled_pairs_sfm(mid_workload):
    """Full size (n = 50,000, |E| = 2,000,000, bursty ticks), in the launch
    configuration of the benchmark: pairs 0..15 of the benchmark's pair
    stream, records and per-pair f over nodes and edges."""
    G, gg, og = mid_workload
    S, Z = oracle.draw_pairs(2002, oracle.STREAM_PAIR, G.n, 0, 16)
    compare_pairs(gg, og, "sfm", S, Z, mode=1, ctx="C2-sfm")


@pytest.mark.parametrize("opt", ["sh", "fm", "pfm"])
def test_mid_workload_other_optimalities(mid_workload, opt):
    G, gg, og = mid_workload
    S, Z = oracle.draw_pairs(2002, oracle.STREAM_PAIR, G.n, 100, 4)
    compare_pairs(gg, og, opt, S, Z, mode=1, edges=False, ctx="C2-" + opt)


def check_sums(gpu_node, gpu_edge, osums, r, c_floor=True):
    ok, worst = rel_close(gpu_node, osums.B / r, rel=1e-12, abs_floor=1e-300)
    assert ok, worst
    if gpu_edge is not None:
        ok, worst = rel_close(gpu_edge, osums.E / r, rel=1e-12, abs_floor=1e-300)
        assert ok, worst


def test_fixed_sample_sums_tiny(tiny_workload):
    """r = 500 sampled pairs (sh), node and temporal-edge estimates, and the
    MCERA statistics of the sample (W, R^c)."""
    G, gg, og = tiny_workload
    nb, eb, res = gg.run("sh", fixed_r=500, seed=2001, c=16, edges=True)
    ref = omantra.fixed(og, "sh", 500, seed=2001, c=16, edges=True, mode=0)
    check_sums(nb, eb, ref["sums"], 500)
    assert abs(res["wimpy"] - ref["W"]) <= 1e-12 * abs(ref["W"])
    scale = float(np.max(ref["sums"].B)) / 500
    assert abs(res["mcera"] - ref["Rc"]) <= 1e-12 * max(scale, 1e-300)


@pytest.mark.parametrize("opt", OPTS)
def test_progressive_tiny(tiny_workload, opt):
    """Algorithm 1 end to end against the oracle's loop: same bootstrap
    statistics, sample-size bound, schedule, stop and estimates."""
    G, gg, og = tiny_workload
    nb, _, res = gg.run(opt, eps=0.03, delta=0.1, seed=7, c=16)
    ref = omantra.estimate(og, opt, 0.03, 0.1, 7, c=16, mode=0)
    assert res["s_boot"] == ref["s_boot"]
    assert abs(res["rho_hat"] - ref["rho_hat"]) <= 1e-12 * max(ref["rho_hat"], 1e-300)
    assert abs(res["v_hat"] - ref["v_hat"]) <= 1e-12 * max(ref["v_hat"], 1e-300)
    assert res["omega"] == ref["omega"] and res["s1"] == ref["s1"]
    assert res["samples"] == ref["samples"] and res["rounds"] == len(ref["rounds"])
    assert abs(res["xi"] - ref["xi"]) <= 1e-12 * ref["xi"]
    ok, worst = rel_close(nb, ref["node_bc"], rel=1e-12, abs_floor=1e-300)
    assert ok, worst
    if opt == "fm":
        assert res["flags"] & 1


def test_packed_graphs(lib):
    """Independent graphs in one device graph: per-graph pairs and sums."""
    from synthgen import packed_uniform_graphs
    gs = packed_uniform_graphs(6, seed=41, n_lo=30, n_hi=300, edges_per_node=10, T=50)
    pg = lib.Graph.packed(gs)
    r = 40
    nb, _, res = pg.run("sh", fixed_r=r, seed=9, c=4)
    off = 0
    for gi, G in enumerate(gs):
        og = oracle.Graph.of(G)
        # graph gi's pairs use the stream 4 gi (pair) / 4 gi + 2 (signs)
        S, Z = oracle.draw_pairs(9, 4 * gi, G.n, 0, r)
        sums, _ = oracle.accumulate(og, "sh", S, Z)
        ok, worst = rel_close(nb[off:off + G.n], sums.B / r, rel=1e-12, abs_floor=1e-300)
        assert ok, (gi, worst)
        rec, nf, _ = pg.count_pairs("sh", S[:10], Z[:10], graph=np.full(10, gi))
        for q in range(10):
            want, _, _ = oracle.pair(og, "sh", int(S[q]), int(Z[q]), nodes=False, edges=False)
            assert int(rec["sigma"][q]) == want["sigma"] and int(rec["hops"][q]) == want["hops"]
        off += G.n


def test_repeat_calls_identical(tiny_workload):
    """Slab state (tags, counters, N) is clean between pairs and calls."""
    G, gg, og = tiny_workload
    a, _, _ = gg.run("sfm", fixed_r=300, seed=3, c=8)
    b, _, _ = gg.run("sfm", fixed_r=300, seed=3, c=8)
    ok, worst = rel_close(a, b, rel=1e-12, abs_floor=1e-300)
    assert ok, worst


def test_output_arrays_reused(tiny_workload):
    """Estimates written into caller-given arrays (every value overwritten,
    whatever they held) equal those written into fresh ones (to the sums'
    tolerance: FP64 atomics add the pairs' values in launch order)."""
    G, gg, og = tiny_workload
    a_n, a_e, _ = gg.run("sfm", fixed_r=300, seed=3, c=8, edges=True)
    b_n, b_e, _ = gg.run("pfm", fixed_r=200, seed=5, c=8, edges=True)
    out = (np.full(gg.n, np.nan), np.full(gg.m_input, np.nan))
    for want_n, want_e, opt, r, seed in ((a_n, a_e, "sfm", 300, 3), (b_n, b_e, "pfm", 200, 5),
                                         (a_n, a_e, "sfm", 300, 3)):
        nb, eb, _ = gg.run(opt, fixed_r=r, seed=seed, c=8, edges=True, out=out)
        assert nb is out[0] and eb is out[1]
        assert np.all(np.isfinite(nb)) and np.all(np.isfinite(eb))
        for got, want in ((nb, want_n), (eb, want_e)):
            ok, worst = rel_close(got, want, rel=1e-12, abs_floor=1e-300)
            assert ok, (opt, worst)
    with pytest.raises(ValueError):
        gg.run("sh", fixed_r=10, edges=True, out=(np.zeros(gg.n), np.zeros(gg.m_input - 1)))
    with pytest.raises(ValueError):
        gg.run("sh", fixed_r=10, out=(np.zeros(gg.n, dtype=np.float32), None))


def test_launch_configs_same_results(lib):
    """Pair order, grid size and arc capacity change the schedule only:
    records are bit-identical and sums agree to 1e-12 under every launch
    configuration."""
    G = chung_lu_graph(3000, 60_000, 2.3, 4000, seed=91, times="pareto")
    gg, og = both(lib, G)
    S, Z = oracle.draw_pairs(92, oracle.STREAM_PAIR, G.n, 0, 600)
    ref = None
    configs = [dict(order="longest"), dict(order="drawn"), dict(n_slabs=7, order="longest"),
               dict(n_slabs=64, arc_cap=2048, order="drawn"), dict(hub_nodes=256), dict(n_slabs=9, hub_nodes=1000)]
    try:
        for cfg in configs:
            gg.set_launch(**cfg)
            rec, _, _ = gg.count_pairs("sfm", S, Z)
            nb, eb, res = gg.run("sh", fixed_r=1500, seed=93, c=8, edges=True)
            cur = (rec, nb, eb, res)
            if ref is None:
                ref = cur
                # the oracle on a prefix of the explicit pairs
                compare_pairs(gg, og, "sfm", S[:40], Z[:40], ctx="cfg")
                continue
            assert np.array_equal(rec, ref[0]), cfg
            for x, y in ((nb, ref[1]), (eb, ref[2])):
                ok, worst = rel_close(x, y, rel=1e-12, abs_floor=1e-300)
                assert ok, (cfg, worst)
            assert res["n_reachable"] == ref[3]["n_reachable"] and res["window_edges"] == ref[3]["window_edges"]
        # the autotuner's pick changes nothing either
        best = gg.autotune("sfm", sample_pairs=512, seed=5)
        assert best["n_slabs"] >= 1 and best["order"] in (0, 1)
        assert gg.get_launch()["order"] == best["order"]
        rec, _, _ = gg.count_pairs("sfm", S, Z)
        nb, eb, res = gg.run("sh", fixed_r=1500, seed=93, c=8, edges=True)
        assert np.array_equal(rec, ref[0])
        for x, y in ((nb, ref[1]), (eb, ref[2])):
            ok, worst = rel_close(x, y, rel=1e-12, abs_floor=1e-300)
            assert ok, ("autotuned", best, worst)
    finally:
        gg.set_launch()
    assert gg.get_launch()["order"] == 0


@pytest.mark.parametrize("opt", ["sh", "sfm", "pfm"])
def test_graph_rounds_match_eager(lib, opt):
    """Progressive rounds replayed from one captured HIP graph (several
    replays, with the host's reductions and bound checks between them) give
    the eager launches' schedule, stop and estimates; on the tiny workload
    also the oracle's Algorithm 1."""
    G = workload("tiny-uniform-n100")
    gg, og = both(lib, G)
    eager = gg.run(opt, eps=0.02, delta=0.1, seed=21, c=16)
    gg.set_launch(graph_rounds=True)
    try:
        graph = gg.run(opt, eps=0.02, delta=0.1, seed=21, c=16)
        again = gg.run(opt, eps=0.02, delta=0.1, seed=21, c=16)  # a fresh capture per request
    finally:
        gg.set_launch()
    assert eager[2]["rounds"] >= 3, eager[2]
    ref = omantra.estimate(og, opt, 0.02, 0.1, 21, c=16, mode=0)
    for got in (graph, again):
        for k in ("samples", "rounds", "omega", "s1", "n_reachable", "flags"):
            assert got[2][k] == eager[2][k], (k, got[2][k], eager[2][k])
        ok, worst = rel_close(got[0], eager[0], rel=1e-12, abs_floor=1e-300)
        assert ok, worst
        ok, worst = rel_close(got[0], ref["node_bc"], rel=1e-12, abs_floor=1e-300)
        assert ok, worst
    # a larger graph: rounds of thousands of pairs
    H = chung_lu_graph(4000, 80_000, 2.3, 5000, seed=77, times="pareto")
    hg = lib.Graph.of(H)
    e2 = hg.run(opt, eps=0.04, delta=0.1, seed=22, c=8, edges=True)
    hg.set_launch(graph_rounds=True)
    g2 = hg.run(opt, eps=0.04, delta=0.1, seed=22, c=8, edges=True)
    for k in ("samples", "rounds", "omega", "s1", "n_reachable"):
        assert g2[2][k] == e2[2][k], k
    for x, y in ((g2[0], e2[0]), (g2[1], e2[1])):
        ok, worst = rel_close(x, y, rel=1e-12, abs_floor=1e-300)
        assert ok, worst


def test_per_pair_launches_match(tiny_workload):
    """The unbatched form (one launch per pair) computes the same records
    and sums as the persistent launch."""
    G, gg, og = tiny_workload
    S, Z = oracle.draw_pairs(31, oracle.STREAM_PAIR, G.n, 0, 120)
    rec0, nf0, _ = gg.count_pairs("sfm", S, Z, node_f=True)
    nb0, _, r0 = gg.run("sh", fixed_r=150, seed=32, c=4)
    gg.set_launch(per_pair_launch=True)
    try:
        rec1, nf1, _ = gg.count_pairs("sfm", S, Z, node_f=True)
        nb1, _, r1 = gg.run("sh", fixed_r=150, seed=32, c=4)
        assert gg.last_timing()["launches"] == 150
    finally:
        gg.set_launch()
    assert np.array_equal(rec0, rec1) and np.array_equal(nf0, nf1)
    ok, worst = rel_close(nb0, nb1, rel=1e-12, abs_floor=1e-300)
    assert ok, worst


@pytest.mark.parametrize("opt", OPTS)
def test_hub_state_in_lds(lib, opt):
    """Forward state of the highest-degree nodes kept in LDS: bit-exact on
    random tiny graphs (all pairs), on ticks longer than a batch and on a
    head with 600 in-edges at one time (hub heads and tails on every path)."""
    from synthgen.graphs import TemporalGraph
    for seed in range(6):
        rng = np.random.default_rng(900 + seed)
        n, src, dst, t = tiny_graph(rng)
        gg, og = both(lib, TemporalGraph(n, src, dst, t))
        gg.set_launch(hub_nodes=max(1, n // 3))
        S, Z = all_pairs(n)
        compare_pairs(gg, og, opt, S, Z, ctx="hub-tiny%d" % seed)
    G = uniform_graph(80, 4000, 6, seed=77)
    gg, og = both(lib, G)
    gg.set_launch(hub_nodes=40)
    S, Z = oracle.draw_pairs(5, 0, G.n, 0, 200)
    compare_pairs(gg, og, opt, S, Z, ctx="hub-bigtick")
    H = chung_lu_graph(3000, 60_000, 2.3, 4000, seed=91, times="pareto")
    hg, ho = both(lib, H)
    S, Z = oracle.draw_pairs(94, oracle.STREAM_PAIR, H.n, 0, 60)
    for K in (256, 512, 1024):
        hg.set_launch(hub_nodes=K)
        compare_pairs(hg, ho, opt, S, Z, ctx="hub-cl%d" % K)
        assert hg.get_launch()["hub_nodes"] == K
