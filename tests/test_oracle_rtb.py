"""Pins of the oracle of the RTB estimator (appendix on other estimators).

* f(v|s) against brute-force walk enumeration (every source of random tiny
  graphs, all four optimalities, two windows), f(e|s) likewise;
* the closed form of the time-increasing line: f(v|s) = (n-1-v)/(n-1) for
  v > s, 0 otherwise, and the edge (i, i+1) carries (n-1-i)/(n-1) for i >= s;
* unbiasedness, exactly: the mean of f(v|s) over all sources is the
  betweenness, the mean of the pair dependencies over all ordered pairs.
"""
import numpy as np
import pytest

import oracle
from oracle import rtb
from brute import OPTS, all_walks, pair_brute
from test_oracle_brute import tiny_graph


@pytest.mark.parametrize("seed", range(8))
def test_source_dependencies_brute(seed):
    rng = np.random.default_rng(9000 + seed)
    n, src, dst, t = tiny_graph(rng)
    g = oracle.Graph(n, src, dst, t)
    for t0, t1 in ((0, 2**31 - 1), (2, 5)):
        for s in range(n):
            walks = all_walks(src, dst, t, s, t0, t1)
            for opt in OPTS:
                want_v = np.zeros(n)
                want_e = np.zeros(len(src))
                reach = 0
                for z in range(n):
                    if z == s:
                        continue
                    rec, Nv, Ne = pair_brute(n, src, dst, t, s, z, opt, t0, t1, walks=walks)
                    if not rec["reachable"]:
                        continue
                    reach += 1
                    want_v += np.array(Nv, dtype=np.float64) / rec["sigma"]
                    for e, c in Ne.items():
                        want_e[e] += c / rec["sigma"]
                nf, ef, reached, sat = rtb.source(g, opt, s, t0, t1)
                assert not sat and reached == reach
                assert np.allclose(nf, want_v / (n - 1), rtol=1e-14, atol=0), (opt, s, nf, want_v / (n - 1))
                assert np.allclose(ef, want_e / (n - 1), rtol=1e-14, atol=0), (opt, s)


@pytest.mark.parametrize("n", [2, 5, 12])
def test_line_closed_form(n):
    src = np.arange(n - 1, dtype=np.int32)
    g = oracle.Graph(n, src, src + 1, src + 1)
    for opt in OPTS:
        for s in range(n):
            nf, ef, reached, sat = rtb.source(g, opt, s)
            assert reached == n - 1 - s
            want = np.array([(n - 1 - v) / (n - 1) if v > s else 0.0 for v in range(n)])
            assert np.allclose(nf, want, rtol=1e-15, atol=0)
            # edge (i, i+1) lies on the paths from s to every z > i
            want_e = np.array([(n - 1 - i) / (n - 1) if i >= s else 0.0 for i in range(n - 1)])
            assert np.allclose(ef, want_e, rtol=1e-15, atol=0)


@pytest.mark.parametrize("seed", range(3))
def test_mean_over_sources_is_betweenness(seed):
    rng = np.random.default_rng(9100 + seed)
    n, src, dst, t = tiny_graph(rng, n_lo=5, n_hi=7)
    g = oracle.Graph(n, src, dst, t)
    S, Z = zip(*[(s, z) for s in range(n) for z in range(n) if s != z])
    for opt in OPTS:
        exact, _ = oracle.accumulate(g, opt, np.array(S), np.array(Z), edges=True)
        acc = rtb.accumulate(g, opt, np.arange(n), edges=True)
        assert np.allclose(acc.B / n, exact.B / len(S), rtol=1e-13, atol=1e-300)
        assert np.allclose(acc.E / n, exact.E / len(S), rtol=1e-13, atol=1e-300)
