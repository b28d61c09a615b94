"""The bench's headline step against the oracle, in the launch configuration
the bench times.

serve-chunglu-n2m (n = 2*10^6, |E| = 5*10^7, Chung-Lu exponent 2.3, Pareto
renewal times on 10^6 ticks), sfm, c = 25, node and temporal-edge sums,
the grid resident with 2,048 hub nodes in LDS: the first 16 pairs of the step's
pair stream (the pair stream is counter-based, so they are the first pairs
of every step of that seed), whose sums, W and R^c the oracle accumulates
in about a minute on 16 host threads.  Their records (sigma, arrival, hops)
are compared bit for bit through the explicit-pair entry point too.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import mantra as omantra
from parity_util import rel_close
from synthgen import workload

pytestmark = pytest.mark.gpu

SEED = 2005           # the bench's seed: step k draws its pairs with seed 2005 + k
LAUNCH = {"n_slabs": 0, "hub_nodes": 2048}
R = 16


@pytest.fixture(scope="module")
def headline():
    import torch
    assert torch.cuda.is_available(), "GPU tests need the MI355X"
    import paper_2304_08356_amd as pk
    G = workload("serve-chunglu-n2m")
    gg = pk.Graph.of(G)
    gg.set_launch(**LAUNCH)
    og = oracle.Graph.of(G)
    ref = omantra.fixed(og, "sfm", R, seed=SEED, c=25, edges=True, mode=1, nthreads=os.cpu_count() or 1)
    return G, gg, og, ref


def test_step_sums_against_oracle(headline):
    G, gg, og, ref = headline
    nb, eb, res = gg.run("sfm", fixed_r=R, seed=SEED, c=25, edges=True)
    assert ref["sums"].n_overflow == 0
    assert res["rc"] == 0 and res["n_overflow"] == 0, res
    assert res["n_reachable"] == int(np.sum(ref["records"]["reachable"] > 0))
    ok, worst = rel_close(nb, ref["sums"].B / R, rel=1e-12, abs_floor=1e-300)
    assert ok, worst
    ok, worst = rel_close(eb, ref["sums"].E / R, rel=1e-12, abs_floor=1e-300)
    assert ok, worst
    assert abs(res["wimpy"] - ref["W"]) <= 1e-12 * abs(ref["W"])
    scale = float(np.max(ref["sums"].B)) / R
    assert abs(res["mcera"] - ref["Rc"]) <= 1e-12 * max(scale, 1e-300)


def test_step_records_against_oracle(headline):
    G, gg, og, ref = headline
    S, Z = ref["S"], ref["Z"]
    rec, _, _ = gg.count_pairs("sfm", S, Z)
    want = ref["records"]
    for k in ("reachable", "t_arr", "hops", "sigma"):
        assert np.array_equal(np.asarray(rec[k]).astype(np.int64), np.asarray(want[k]).astype(np.int64)), k
