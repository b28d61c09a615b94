"""GPU parity of the sweep with the reached set in global node bytes (graphs
of more than 65,536 nodes, where the LDS bitmap does not fit), against the
oracle: tiny random graphs padded with isolated nodes to n = 70,000, so
that the small cases of the other parity tests run through the byte map.

Bit-exact records and per-pair f(v|s,z), f(e|s,z) for all four optimalities,
with windows, long ticks (the global-scratch path), hub state in LDS, and the
TRK walks.
"""
import numpy as np
import pytest

import oracle
from parity_util import OPTS, compare_pairs
from synthgen.graphs import TemporalGraph
from test_oracle_brute import tiny_graph

pytestmark = pytest.mark.gpu
N_PAD = 70_000


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need the MI355X"
    import paper_2304_08356_amd as pk
    return pk


def padded(lib, src, dst, t):
    G = TemporalGraph(N_PAD, np.asarray(src, dtype=np.int32), np.asarray(dst, dtype=np.int32),
                      np.asarray(t, dtype=np.int32))
    gg = lib.Graph.of(G)
    assert gg.n == N_PAD
    return G, gg, oracle.Graph.of(G)


def pairs_of(n_act, rng):
    S, Z = zip(*[(s, z) for s in range(n_act) for z in range(n_act) if s != z])
    S, Z = list(S), list(Z)
    # a few pairs with an isolated endpoint
    for _ in range(6):
        S.append(int(rng.integers(0, n_act)))
        Z.append(int(rng.integers(n_act, N_PAD)))
        S.append(int(rng.integers(n_act, N_PAD)))
        Z.append(int(rng.integers(0, n_act)))
    return np.array(S, dtype=np.int32), np.array(Z, dtype=np.int32)


def test_padded_tiny_random_graphs(lib):
    for seed in range(20):
        rng = np.random.default_rng(90_000 + seed)
        n, src, dst, t = tiny_graph(rng)
        G, gg, og = padded(lib, src, dst, t)
        S, Z = pairs_of(n, rng)
        for opt in OPTS:
            compare_pairs(gg, og, opt, S, Z, ctx="pad%d" % seed)
            compare_pairs(gg, og, opt, S, Z, 2, 5, ctx="pad-win%d" % seed)


@pytest.mark.parametrize("opt", OPTS)
def test_padded_long_ticks_and_hubs(lib, opt):
    """A head with 600 in-edges at one tick and ticks longer than a batch,
    with and without hub state in LDS."""
    rng = np.random.default_rng(91_000)
    n = 700
    src = list(range(1, 601)) + list(rng.integers(0, n, 900))
    dst = [0] * 600 + list(rng.integers(0, n, 900))
    t = [5] * 600 + list(rng.integers(1, 8, 900))
    tr = {}
    for u, v, tt in zip(src, dst, t):
        if u != v:
            tr[(int(u), int(v), int(tt))] = 1
    a = np.array(list(tr.keys()), dtype=np.int32)
    G, gg, og = padded(lib, a[:, 0], a[:, 1], a[:, 2])
    S, Z = oracle.draw_pairs(9, 0, n, 0, 160)
    compare_pairs(gg, og, opt, S, Z, ctx="pad-star")
    gg.set_launch(hub_nodes=64)
    try:
        assert gg.get_launch()["hub_nodes"] == 64
        compare_pairs(gg, og, opt, S, Z, ctx="pad-star-hubs")
    finally:
        gg.set_launch(hub_nodes=0)


@pytest.mark.parametrize("opt", OPTS)
def test_padded_two_row_ticks(lib, opt):
    """Ticks of 57..168 edges (one row, two rows in registers, longer)."""
    from synthgen import uniform_graph
    for n, m, T, seed in ((12, 1000, 10, 61), (40, 700, 10, 62), (20, 1800, 12, 65), (60, 900, 16, 66)):
        U = uniform_graph(n, m, T, seed=seed)
        G, gg, og = padded(lib, U.src, U.dst, U.t)
        S, Z = oracle.draw_pairs(seed, 0, n, 0, 120)
        compare_pairs(gg, og, opt, S, Z, ctx="pad-rows%d" % seed)
        gg.set_launch(hub_nodes=8)
        try:
            compare_pairs(gg, og, opt, S, Z, ctx="pad-rows-hub%d" % seed)
        finally:
            gg.set_launch(hub_nodes=0)


def test_padded_trk_walks(lib):
    from oracle import trk
    for seed in range(6):
        rng = np.random.default_rng(92_000 + seed)
        n, src, dst, t = tiny_graph(rng)
        G, gg, og = padded(lib, src, dst, t)
        S, Z = pairs_of(n, rng)
        for opt in OPTS:
            rec, nf, ef = gg.sample_paths(opt, S, Z, seed=seed)
            for q in range(len(S)):
                want, nv, ev = trk.path(og, opt, int(S[q]), int(Z[q]), seed, q, oracle.STREAM_PAIR)
                c = (seed, opt, q, int(S[q]), int(Z[q]))
                assert int(rec["flags"][q]) & 2 == 0, c
                assert int(rec["sigma"][q]) == want["sigma"] and int(rec["hops"][q]) == want["hops"], c
                assert np.array_equal(nf[q], nv.astype(np.float64)), c
                assert np.array_equal(ef[q], ev.astype(np.float64)), c
