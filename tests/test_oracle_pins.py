"""Pins of the oracle's per-pair counts to facts the paper and the
mathematics fix (hand-worked example, textbook reductions, closed forms,
integer invariants).  CPU only."""
import json
import os

import networkx as nx
import numpy as np
import pytest

import oracle
from synthgen import uniform_graph

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
OPTS = ("sh", "fm", "sfm", "pfm")


def _graph(edges, n):
    a = np.array(edges, dtype=np.int32).reshape(-1, 3)
    return n, a[:, 0].copy(), a[:, 1].copy(), a[:, 2].copy()


def all_pairs_f(n, src, dst, t, opt, mode=0, edges=False):
    """Exact b(v) (and b(e)) as the mean of f over all n(n-1) ordered pairs
    (the definition of temporal betweenness, and Appendix A for edges)."""
    g = oracle.Graph(n, src, dst, t)
    S, Z = zip(*[(s, z) for s in range(n) for z in range(n) if s != z])
    sums, recs = oracle.accumulate(g, opt, np.array(S), np.array(Z), mode=mode, edges=edges)
    b = sums.B / (n * (n - 1))
    e = sums.E / (n * (n - 1)) if edges else None
    return b, e, recs


def test_fig3_caption_example():
    fx = json.load(open(os.path.join(GOLDEN, "fig3_example.json")))
    ids = fx["nodes"]
    inv = {v: k for k, v in ids.items()}
    for gname, edges in fx["graphs"].items():
        n, src, dst, t = _graph([[ids[u], ids[v], tt] for u, v, tt in edges], len(ids))
        g = oracle.Graph(n, src, dst, t)
        for opt, want in fx["expect"][gname].items():
            for mode in (0, 1):
                rec, nN, eN = oracle.pair(g, opt, ids["s"], ids["z"], mode=mode)
                assert rec["sigma"] == want["sigma"], (gname, opt)
                assert rec["hops"] == want["hops"], (gname, opt)
                assert rec["t_arr"] == want["t_arr"], (gname, opt)
                got = {inv[v]: int(nN[v]) for v in range(n) if nN[v]}
                assert got == want["N"], (gname, opt, got)


def layered_dag(seed, layers=5, width=4, p=0.55):
    rng = np.random.default_rng(seed)
    nodes = [[layer * width + i for i in range(width)] for layer in range(layers)]
    edges = []
    for layer in range(layers - 1):
        for u in nodes[layer]:
            for v in nodes[layer + 1]:
                if rng.random() < p:
                    edges.append((u, v, layer + 1))
    return layers * width, edges


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("opt", OPTS)
def test_layered_dag_equals_static_brandes(seed, opt):
    """Edges only from layer l to l+1 at time l+1: temporal paths are the
    static paths, all of one length and arrival, so every optimality reduces to
    static shortest-path betweenness (Brandes), computed here by networkx."""
    n, edges = layered_dag(seed)
    n, src, dst, t = _graph(edges, n)
    b, e, _ = all_pairs_f(n, src, dst, t, opt, edges=True)
    G = nx.DiGraph()
    G.add_nodes_from(range(n))
    G.add_edges_from([(u, v) for u, v, _ in edges])
    ref = nx.betweenness_centrality(G, normalized=False)
    for v in range(n):
        assert b[v] == pytest.approx(ref[v] / (n * (n - 1)), rel=1e-12, abs=1e-15)
    eref = nx.edge_betweenness_centrality(G, normalized=False)
    for k, (u, v, _) in enumerate(edges):
        assert e[k] == pytest.approx(eref[(u, v)] / (n * (n - 1)), rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("opt", OPTS)
@pytest.mark.parametrize("n", [2, 5, 9])
def test_time_increasing_line(opt, n):
    """0 -> 1 -> ... -> n-1 with edge i -> i+1 at time i+1: every s < z has
    one path, so b(v) = v (n-1-v) / (n (n-1))."""
    edges = [(i, i + 1, i + 1) for i in range(n - 1)]
    n_, src, dst, t = _graph(edges, n)
    b, _, _ = all_pairs_f(n, src, dst, t, opt)
    for v in range(n):
        assert b[v] == pytest.approx(v * (n - 1 - v) / (n * (n - 1)), rel=1e-15, abs=0)


@pytest.mark.parametrize("opt", OPTS)
def test_single_tick(opt):
    """All edges at one time: no walk has two edges, sigma in {0, 1}, every
    b(v) is 0 and sum_e b(e) = |E| / (n(n-1)) (Lemma 6 with one-hop paths)."""
    g = uniform_graph(12, 40, 1, seed=5)
    b, e, recs = all_pairs_f(g.n, g.src, g.dst, g.t, opt, edges=True)
    assert np.all(b == 0)
    assert set(recs["sigma"].tolist()) <= {0, 1}
    assert e.sum() == pytest.approx(g.m / (g.n * (g.n - 1)), rel=1e-14)


@pytest.fixture(scope="module")
def tiny_workload():
    return uniform_graph(100, 2000, 100, seed=1001)


@pytest.mark.parametrize("opt", OPTS)
def test_integer_invariants_all_pairs(tiny_workload, opt):
    """Per pair, exactly: sum_e N(e) = sum_v N(v) + sigma for sh/sfm/pfm
    (each optimal path of k hops has k edges and k-1 distinct internal nodes);
    sum_v N(v) = sigma (hops-1) for sh/sfm (all optimal paths of one pair have
    the same length); for fm the edge side can only be larger (internal visits
    of s are not counted)."""
    G = tiny_workload
    g = oracle.Graph.of(G)
    rng = np.random.default_rng(7)
    for _ in range(150):
        s, z = rng.choice(G.n, 2, replace=False)
        rec, nN, eN = oracle.pair(g, opt, int(s), int(z))
        assert rec["flags"] == 0
        sv = int(nN.astype(object).sum())
        se = int(eN.astype(object).sum())
        sig = rec["sigma"]
        if not rec["reachable"]:
            assert sv == 0 and se == 0 and sig == 0
            continue
        if opt == "fm":
            assert se >= sv + sig or se == sv + sig
        else:
            assert se == sv + sig
        if opt in ("sh", "sfm"):
            assert sv == sig * (rec["hops"] - 1)
        if opt != "fm":
            assert int(nN.max()) <= sig


def test_cross_optimality_relations(tiny_workload):
    """sigma_pfm <= sigma_fm and sigma_sfm <= sigma_fm (both count subsets of
    the foremost walks); shortest paths never arrive before t* and never take
    more hops than the shortest-foremost ones; pfm and sfm arrive at t*."""
    G = tiny_workload
    g = oracle.Graph.of(G)
    rng = np.random.default_rng(8)
    for _ in range(300):
        s, z = (int(x) for x in rng.choice(G.n, 2, replace=False))
        r = {o: oracle.pair(g, o, s, z, nodes=False, edges=False)[0] for o in OPTS}
        if not r["fm"]["reachable"]:
            assert all(not r[o]["reachable"] for o in OPTS)
            continue
        assert r["pfm"]["sigma"] <= r["fm"]["sigma"]
        assert r["sfm"]["sigma"] <= r["fm"]["sigma"]
        ts = r["fm"]["t_arr"]
        assert r["sfm"]["t_arr"] == ts and r["pfm"]["t_arr"] == ts
        assert r["sh"]["t_arr"] >= ts
        assert r["sh"]["hops"] <= r["sfm"]["hops"]
        assert r["sfm"]["hops"] == r["fm"]["hops"]


@pytest.mark.parametrize("opt", OPTS)
def test_modes_agree_on_tiny_workload(tiny_workload, opt):
    """The explicit-arc and running-aggregate modes give identical counts."""
    G = tiny_workload
    g = oracle.Graph.of(G)
    rng = np.random.default_rng(9)
    for _ in range(60):
        s, z = (int(x) for x in rng.choice(G.n, 2, replace=False))
        r0, n0, e0 = oracle.pair(g, opt, s, z, mode=0)
        r1, n1, e1 = oracle.pair(g, opt, s, z, mode=1)
        assert r0 == r1
        assert np.array_equal(n0, n1) and np.array_equal(e0, e1)


@pytest.mark.parametrize("opt", ["sh", "sfm", "pfm"])
def test_lemma1_and_lemma6_all_pairs(tiny_workload, opt):
    """Lemma 1: sum_v b(v) = rho, the average number of internal nodes of an
    optimal path; Lemma 6: sum_e b(e) = Psi, the average number of edges
    (pairs without a path count 0, as in the definitions)."""
    G = tiny_workload
    g = oracle.Graph.of(G)
    S, Z = zip(*[(s, z) for s in range(G.n) for z in range(G.n) if s != z][::7])
    S, Z = np.array(S), np.array(Z)
    sums, recs = oracle.accumulate(g, opt, S, Z, edges=True)
    rho = 0.0
    psi = 0.0
    for q in range(len(S)):
        rec, nN, eN = oracle.pair(g, opt, int(S[q]), int(Z[q]))
        if rec["reachable"]:
            rho += float(nN.astype(object).sum()) / rec["sigma"]
            psi += float(eN.astype(object).sum()) / rec["sigma"]
    assert sums.B.sum() == pytest.approx(rho, rel=1e-12)
    assert sums.E.sum() == pytest.approx(psi, rel=1e-12)
    if opt in ("sh", "sfm"):
        hops = recs["hops"][recs["reachable"] == 1].astype(np.int64)
        assert sums.B.sum() == pytest.approx(float((hops - 1).sum()), rel=1e-12)
        assert sums.E.sum() == pytest.approx(float(hops.sum()), rel=1e-12)


def test_saturation_chain():
    """16 hops with 16 parallel temporal edges per hop at increasing times:
    16^16 = 2^64 shortest paths, which saturates the uint64 count (flagged,
    never rounded)."""
    edges = []
    for i in range(16):
        for j in range(16):
            edges.append((i, i + 1, 16 * i + j + 1))
    n, src, dst, t = _graph(edges, 17)
    g = oracle.Graph(n, src, dst, t)
    for opt in ("sh", "sfm", "fm"):
        rec, nN, _ = oracle.pair(g, opt, 0, 16)
        if opt == "sh":
            assert rec["sigma"] == 2**64 - 1 and rec["flags"] & oracle.REC_OVERFLOW
    # 15 hops: 16^15 = 2^60 fits exactly
    rec, nN, _ = oracle.pair(g, "sh", 0, 15)
    assert rec["sigma"] == 2**60 and rec["flags"] == 0
    assert int(nN[7]) == 2**60


def test_unreachable_pair_is_zero():
    edges = [(0, 1, 5), (1, 2, 3)]  # 0 -> 1 at 5 cannot continue at 3
    n, src, dst, t = _graph(edges, 3)
    g = oracle.Graph(n, src, dst, t)
    for opt in OPTS:
        rec, nN, eN = oracle.pair(g, opt, 0, 2)
        assert rec == {"reachable": 0, "t_arr": -1, "hops": -1, "flags": 0, "sigma": 0}
        assert not nN.any() and not eN.any()
