"""The bench's mid-size step against the oracle, in the launch configuration
the bench times (the autotuner's pick for the workload).

mid-chunglu-n50k (n = 50,000, |E| = 2*10^6, Pareto renewal times on 10^5
ticks), sfm, c = 25, node and temporal-edge sums: the first 512 pairs of the
step's pair stream, whose sums, W and R^c the oracle accumulates in seconds.
Also the blocking call of the paper's problem statement (mantra_estimate)
against mantra_run of the same request.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import mantra as omantra
from parity_util import rel_close
from synthgen import workload

pytestmark = pytest.mark.gpu

SEED = 2002  # the bench's seed: step k draws its pairs with seed 2002 + k


@pytest.fixture(scope="module")
def mid():
    import torch
    assert torch.cuda.is_available(), "GPU tests need the MI355X"
    import paper_2304_08356_amd as pk
    G = workload("mid-chunglu-n50k")
    gg = pk.Graph.of(G)
    gg.autotune("sfm", sample_pairs=4096, seed=SEED + 7)
    return G, gg, oracle.Graph.of(G)


def test_step_prefix_sums_against_oracle(mid):
    G, gg, og = mid
    r, c = 512, 25
    nb, eb, res = gg.run("sfm", fixed_r=r, seed=SEED, c=c, edges=True)
    ref = omantra.fixed(og, "sfm", r, seed=SEED, c=c, edges=True, mode=1, nthreads=os.cpu_count() or 1)
    assert ref["sums"].n_overflow == 0
    assert res["rc"] == 0 and res["n_overflow"] == 0, res
    assert res["n_reachable"] == int(np.sum(ref["records"]["reachable"] > 0))
    ok, worst = rel_close(nb, ref["sums"].B / r, rel=1e-12, abs_floor=1e-300)
    assert ok, worst
    ok, worst = rel_close(eb, ref["sums"].E / r, rel=1e-12, abs_floor=1e-300)
    assert ok, worst
    assert abs(res["wimpy"] - ref["W"]) <= 1e-12 * abs(ref["W"])
    scale = float(np.max(ref["sums"].B)) / r
    assert abs(res["mcera"] - ref["Rc"]) <= 1e-12 * max(scale, 1e-300)


def test_estimate_is_the_default_request(mid):
    """mantra_estimate (whole span, c = 25, node and edge buffers in the
    result) equals mantra_run of the same request."""
    G, gg, og = mid
    nb, eb, res = gg.estimate("pfm", 0.05, 0.1, 31, edges=True)
    nb2, eb2, res2 = gg.run("pfm", eps=0.05, delta=0.1, seed=31, c=25, edges=True)
    assert res["status"] == 0 and res2["rc"] == 0
    for k in ("samples", "rounds", "omega", "s_boot", "s1", "n_reachable"):
        assert res[k] == res2[k], k
    ok, worst = rel_close(nb, nb2, rel=1e-12, abs_floor=1e-300)
    assert ok, worst
    ok, worst = rel_close(eb, eb2, rel=1e-12, abs_floor=1e-300)
    assert ok, worst
    nb3, eb3, _ = gg.estimate("pfm", 0.05, 0.1, 31)
    assert eb3 is None
    ok, worst = rel_close(nb, nb3, rel=1e-12, abs_floor=1e-300)
    assert ok, worst
