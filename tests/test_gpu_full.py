"""GPU parity at the full workload sizes, on sampled outputs the oracle can
compute one by one, in the default launch configuration.

* big-chunglu-n1m (n = 10^6, |E| = 2*10^7): pfm, fm and sfm records and
  per-pair f(v|s,z) of sampled pairs, bit-exact; Algorithm 1 at the
  workload's settings against the fixed sample of the same pairs;
* packed-256 (256 graphs, sum |E| ~ 1.1*10^8): the whole r = 2,000 per graph
  sh launch, with the sums of two graphs (the smallest and the first
  quartile) against the oracle's accumulation of the same pairs, and sampled
  records there and on the largest graph.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import mantra as omantra
from parity_util import compare_pairs, rel_close
from synthgen import workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need the MI355X"
    import paper_2304_08356_amd as pk
    return pk


@pytest.fixture(scope="module")
def big(lib):
    G = workload("big-chunglu-n1m")
    return G, lib.Graph.of(G), oracle.Graph.of(G)


@pytest.mark.parametrize("opt", ["pfm", "fm", "sfm"])
def test_big_sampled_pairs(big, opt):
    G, gg, og = big
    S, Z = oracle.draw_pairs(2003, oracle.STREAM_PAIR, G.n, 0, 2)
    compare_pairs(gg, og, opt, S, Z, edges=False, mode=1, ctx="n1m")


def test_big_progressive_runs(big):
    """Algorithm 1 at the workload's settings (eps = 0.005, c = 16,
    s1 = 4,096), capped at one round: the loop runs at full size and its
    round is the sample the fixed-size call computes.  pfm counts past 64
    bits go to the multiword path, so nothing saturates."""
    G, gg, og = big
    nb, _, res = gg.run("pfm", eps=0.005, delta=0.1, seed=2003, c=16, s1=4096, max_samples=4096,
                        raise_on_error=False)
    assert res["rc"] == 0 and res["n_overflow"] == 0, res
    assert res["s1"] == 4096 and res["samples"] == 4096 and res["rounds"] == 1
    assert res["flags"] & 4  # stopped at the (capped) omega
    fx, _, rf = gg.run("pfm", fixed_r=4096, seed=2003, c=16, raise_on_error=False)
    assert rf["rc"] == 0 and rf["n_overflow"] == 0, rf
    assert rf["n_reachable"] == res["n_reachable"]
    ok, worst = rel_close(nb, fx, rel=1e-12, abs_floor=1e-300)
    assert ok, worst


def test_big_pfm_prefix_sums_against_oracle(big):
    """The first 64 pairs of the workload's pair stream (pfm, c = 16): node
    sums, W and R^c against the oracle's accumulation of the same pairs."""
    G, gg, og = big
    r = 64
    nb, _, res = gg.run("pfm", fixed_r=r, seed=2003, c=16, raise_on_error=False)
    ref = omantra.fixed(og, "pfm", r, seed=2003, c=16, mode=1, nthreads=os.cpu_count() or 1)
    assert ref["sums"].n_overflow == 0  # beyond 64 bits the oracle could not compare
    assert res["rc"] == 0 and res["n_overflow"] == 0, res
    assert res["n_reachable"] == int(np.sum(ref["records"]["reachable"] > 0))
    ok, worst = rel_close(nb, ref["sums"].B / r, rel=1e-12, abs_floor=1e-300)
    assert ok, worst
    assert abs(res["wimpy"] - ref["W"]) <= 1e-12 * abs(ref["W"])
    scale = float(np.max(ref["sums"].B)) / r
    assert abs(res["mcera"] - ref["Rc"]) <= 1e-12 * max(scale, 1e-300)


def test_big_autotune(big):
    """The autotuner on the n = 10^6 graph, where device memory bounds the
    grid (candidate grids reallocate the slab pool and its shared arc
    chunks): it keeps a configuration, and a fixed sample run under it gives
    the same sums as under the automatic one."""
    G, gg, og = big
    base, _, r0 = gg.run("pfm", fixed_r=512, seed=2013, c=16)
    tuned = gg.autotune("pfm", sample_pairs=1024, seed=2014)
    try:
        assert tuned["n_slabs"] >= 1 and tuned["arc_cap"] >= 1
        assert gg.get_launch()["n_slabs"] == tuned["n_slabs"]
        nb, _, r1 = gg.run("pfm", fixed_r=512, seed=2013, c=16)
        assert r1["rc"] == 0 and r1["n_reachable"] == r0["n_reachable"]
        ok, worst = rel_close(nb, base, rel=1e-12, abs_floor=1e-300)
        assert ok, worst
    finally:
        gg.set_launch(0, 0)


@pytest.fixture(scope="module")
def packed(lib):
    gs = workload("packed-256")
    return gs, lib.Graph.packed(gs)


def test_packed_256_full_launch(packed):
    gs, pg = packed
    r = 2000
    nb, _, res = pg.run("sh", fixed_r=r, seed=2004, c=4, raise_on_error=False)
    # sh counts past 64 bits go to the multiword path: nothing saturates
    assert res["rc"] == 0 and res["n_overflow"] == 0, res
    ns = np.array([g.n for g in gs])
    off = np.concatenate([[0], np.cumsum(ns)])
    order = np.argsort(ns)
    # sums of whole graphs where the oracle finishes 2,000 sh pairs in
    # seconds; records of sampled pairs on the largest graph
    for gi, n_rec in ((int(order[0]), 4), (int(order[len(order) // 4]), 4), (int(order[-1]), 2)):
        G = gs[gi]
        og = oracle.Graph.of(G)
        S, Z = oracle.draw_pairs(2004, 4 * gi, G.n, 0, r)
        if gi != int(order[-1]):
            sums, _ = oracle.accumulate(og, "sh", S, Z, mode=1)
            assert sums.n_overflow == 0
            ok, worst = rel_close(nb[off[gi]:off[gi + 1]], sums.B / r, rel=1e-12, abs_floor=1e-300)
            assert ok, (gi, G.n, worst)
        compare_pairs(pg_view(pg, gi), og, "sh", S[:n_rec], Z[:n_rec], edges=False, mode=1, ctx="pk%d" % gi)


class pg_view:
    """count_pairs of one graph of a packed device graph (local node ids)."""

    def __init__(self, pg, gi):
        self.pg, self.gi = pg, gi

    def count_pairs(self, opt, S, Z, t0=0, t1=2**31 - 1, node_f=False, edge_f=False):
        rec, nf, _ = self.pg.count_pairs(opt, S, Z, t0, t1, graph=np.full(len(S), self.gi, dtype=np.int32),
                                         node_f=node_f)
        if nf is not None:
            off = int(np.sum(self.pg.node_counts[:self.gi]))
            nf = nf[:, off:off + int(self.pg.node_counts[self.gi])]
        return rec, nf, None
