"""The allocation-free entry point (mantra_count_pairs_static) against
mantra_count_pairs, through the C ABI: bit-exact records on two calls in a
row (the second with fewer pairs, the array keeping the first call's
contents), on a second graph after that, and with a node-byte reached set
(a graph above 65,536 nodes); a graph too large for the static array is
refused with MANTRA_E_TOO_LARGE."""
import ctypes

import numpy as np
import pytest

import oracle
from synthgen import uniform_graph, workload
from synthgen.graphs import TemporalGraph
from test_oracle_brute import tiny_graph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need the MI355X"
    import paper_2304_08356_amd as pk
    return pk


def static_records(pk, gg, opt, S, Z, t0=0, t1=2**31 - 1):
    from paper_2304_08356_amd import _lib
    S = np.ascontiguousarray(S, dtype=np.int32)
    Z = np.ascontiguousarray(Z, dtype=np.int32)
    rec = np.zeros(len(S), dtype=pk.REC_DTYPE)
    rc = _lib._lib.mantra_count_pairs_static(gg._h, _lib.OPT[opt], int(t0), int(t1), len(S), None,
                                             S.ctypes.data_as(ctypes.c_void_p), Z.ctypes.data_as(ctypes.c_void_p),
                                             rec.ctypes.data_as(ctypes.c_void_p))
    return rc, rec


def same(pk, gg, opt, S, Z, ctx, t0=0, t1=2**31 - 1):
    rc, got = static_records(pk, gg, opt, S, Z, t0, t1)
    assert rc == 0, (ctx, rc)
    want, _, _ = gg.count_pairs(opt, S, Z, t0, t1)
    for k in ("reachable", "t_arr", "hops", "flags", "sigma"):
        assert np.array_equal(got[k], want[k]), (ctx, opt, k)
    return got


def test_two_calls_then_another_graph(lib):
    G = workload("tiny-uniform-n100")
    gg = lib.Graph.of(G)
    S, Z = oracle.draw_pairs(2001, oracle.STREAM_PAIR, G.n, 0, 500)
    for opt in ("sh", "fm", "sfm", "pfm"):
        same(lib, gg, opt, S, Z, "first")
        same(lib, gg, opt, S[:37], Z[:37], "second, smaller")
    # the records agree with the oracle too
    og = oracle.Graph.of(G)
    _, rec = static_records(lib, gg, "sfm", S[:20], Z[:20])
    for q in range(20):
        want, _, _ = oracle.pair(og, "sfm", int(S[q]), int(Z[q]), nodes=False, edges=False)
        assert (int(rec["sigma"][q]), int(rec["hops"][q]), int(rec["t_arr"][q])) == (
            want["sigma"], want["hops"], want["t_arr"])
    G2 = uniform_graph(80, 4000, 6, seed=77)  # long ticks
    g2 = lib.Graph.of(G2)
    S2, Z2 = oracle.draw_pairs(5, 0, G2.n, 0, 120)
    for opt in ("sh", "pfm"):
        same(lib, g2, opt, S2, Z2, "other graph")
        same(lib, g2, opt, S2[:5], Z2[:5], "other graph, smaller", t0=2, t1=5)
    same(lib, gg, "sh", S[:64], Z[:64], "back to the first graph")


def test_node_bytes_and_too_large(lib):
    rng = np.random.default_rng(90_000)
    n, src, dst, t = tiny_graph(rng)
    G = TemporalGraph(70_000, src, dst, t)
    gg = lib.Graph.of(G)
    S, Z = zip(*[(s, z) for s in range(n) for z in range(n) if s != z])
    for opt in ("sh", "fm", "sfm", "pfm"):
        same(lib, gg, opt, np.array(S), np.array(Z), "node bytes")
    big = workload("mid-chunglu-n50k")
    gb = lib.Graph.of(big)
    rc, _ = static_records(lib, gb, "sh", [0], [1])
    assert rc == 0  # n = 50,000, |E| = 2*10^6: a few workgroups fit
    rc, _ = static_records(lib, gb, "sh", np.zeros(8_000_000, dtype=np.int32), np.ones(8_000_000, dtype=np.int32))
    assert rc == -5  # the pairs and their records alone pass the array
