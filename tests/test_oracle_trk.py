"""Pins of the oracle's TRK path sampler (appendix on other estimators).

* every drawn walk is an optimal walk of its pair (brute-force enumeration,
  all pairs of random tiny graphs, all four optimalities, two windows);
* each optimal walk is drawn with probability 1/sigma_sz (chi-square bound
  over many draws, pairs with several optimal walks);
* the estimator is unbiased: over all ordered pairs and many draws, the
  mean of f is close to the exact betweenness (the ob estimator's mean
  over all pairs), and f(e) likewise for temporal edges;
* the path stream is SplitMix64 keyed as stated.
"""
import math
from collections import Counter

import numpy as np
import pytest

import oracle
from oracle import trk
from brute import OPTS, all_walks
from test_oracle_brute import tiny_graph


def optimal_walks(n, src, dst, t, s, z, opt, t0=0, t1=2**31 - 1, walks=None):
    if walks is None:
        walks = all_walks(src, dst, t, s, t0, t1)
    arr = {}
    for w in walks:
        v, a = int(dst[w[-1]]), int(t[w[-1]])
        if v not in arr or a < arr[v]:
            arr[v] = a
    to_z = [w for w in walks if int(dst[w[-1]]) == z]
    if not to_z:
        return []
    tz = arr[z]
    if opt == "sh":
        k = min(len(w) for w in to_z)
        return [w for w in to_z if len(w) == k]
    if opt == "sfm":
        fore = [w for w in to_z if int(t[w[-1]]) == tz]
        k = min(len(w) for w in fore)
        return [w for w in fore if len(w) == k]
    if opt == "fm":
        return [w for w in to_z if int(t[w[-1]]) == tz]
    return [w for w in to_z if all(int(dst[e]) != s and int(t[e]) == arr[int(dst[e])] for e in w)]


def walk_key(ev):
    return tuple(sorted(int(e) for e in np.nonzero(ev)[0] for _ in range(int(ev[e]))))


@pytest.mark.parametrize("seed", range(10))
def test_drawn_walks_are_optimal(seed):
    rng = np.random.default_rng(8000 + seed)
    n, src, dst, t = tiny_graph(rng)
    g = oracle.Graph(n, src, dst, t)
    for t0, t1 in ((0, 2**31 - 1), (2, 5)):
        for s in range(n):
            walks = all_walks(src, dst, t, s, t0, t1)
            for z in range(n):
                if z == s:
                    continue
                for opt in OPTS:
                    ow = optimal_walks(n, src, dst, t, s, z, opt, t0, t1, walks)
                    rec, nv, ev = trk.path(g, opt, s, z, seed=seed, i=s * n + z, t0=t0, t1=t1)
                    if not ow:
                        assert not rec["reachable"] and nv.sum() == 0 and ev.sum() == 0
                        continue
                    assert rec["sigma"] == len(ow)
                    keys = {tuple(sorted(w)) for w in ow}
                    k = walk_key(ev)
                    assert k in keys, (opt, s, z, k, keys)
                    # internal visits: the walk's nodes other than s and z
                    w = [x for x in ow if tuple(sorted(x)) == k][0]
                    want = Counter(int(dst[e]) for e in w[:-1])
                    for v in (s, z):
                        want.pop(v, None)
                    assert {int(v): int(c) for v, c in enumerate(nv) if c} == dict(want)


def test_walk_distribution_is_uniform_over_optimal_walks():
    """Pairs with 3+ optimal walks: each drawn about 1/sigma of the time."""
    # two layers of three parallel routes, and a fm example with revisits
    src = np.array([0, 0, 0, 1, 2, 3, 4, 4, 4, 5, 6, 7], dtype=np.int32)
    dst = np.array([1, 2, 3, 4, 4, 4, 5, 6, 7, 8, 8, 8], dtype=np.int32)
    t = np.array([1, 1, 1, 2, 2, 2, 3, 3, 3, 4, 4, 4], dtype=np.int32)
    g = oracle.Graph(9, src, dst, t)
    draws = 3000
    for opt in OPTS:
        ow = optimal_walks(9, src, dst, t, 0, 8, opt)
        assert len(ow) == 9
        cnt = Counter(walk_key(trk.path(g, opt, 0, 8, seed=11, i=i)[2]) for i in range(draws))
        assert set(cnt) == {tuple(sorted(w)) for w in ow}
        exp = draws / len(ow)
        chi2 = sum((c - exp) ** 2 / exp for c in cnt.values())
        assert chi2 < 30.0, (opt, chi2, cnt)  # 8 d.o.f.: p ~ 2e-4


@pytest.mark.parametrize("seed", range(3))
def test_unbiased_over_all_pairs(seed):
    rng = np.random.default_rng(8100 + seed)
    n, src, dst, t = tiny_graph(rng, n_lo=5, n_hi=7)
    g = oracle.Graph(n, src, dst, t)
    pairs = [(s, z) for s in range(n) for z in range(n) if s != z]
    S = np.array([p[0] for p in pairs], dtype=np.int32)
    Z = np.array([p[1] for p in pairs], dtype=np.int32)
    for opt in ("sh", "sfm", "pfm"):
        exact, _ = oracle.accumulate(g, opt, S, Z, edges=True)
        b = exact.B / len(pairs)
        e = exact.E / len(pairs)
        reps = 150
        tot = oracle.Sums(n, len(src), 0, True)
        for k in range(reps):
            trk.accumulate(g, opt, S, Z, seed=1000 * seed + k, stream=0, i0=0, sums=tot, edges=True)
        est = tot.B / (reps * len(pairs))
        este = tot.E / (reps * len(pairs))
        # each f is in {0, 1}: standard error <= 0.5 / sqrt(reps * pairs)
        tol = 5 * 0.5 / math.sqrt(reps * len(pairs))
        assert np.max(np.abs(est - b)) < tol, (opt, est, b)
        assert np.max(np.abs(este - e)) < tol, (opt, este, e)


def test_path_stream_is_keyed_splitmix():
    key = oracle.splitmix_nth(77, (1 << 20) + 3 + 1)
    assert trk.trk_word(77, 3, 5, 2) == oracle.splitmix_nth(key, (5 << 16) + 2 + 1)


def test_unreachable_and_overflow_pairs_draw_nothing():
    # s = 0 cannot reach 2 (times decrease)
    src = np.array([0, 1], dtype=np.int32)
    dst = np.array([1, 2], dtype=np.int32)
    t = np.array([5, 1], dtype=np.int32)
    g = oracle.Graph(3, src, dst, t)
    rec, nv, ev = trk.path(g, "sh", 0, 2, seed=1, i=0)
    assert rec["reachable"] == 0 and nv.sum() == 0 and ev.sum() == 0
    # 16 hops x 16 parallel edges: sigma saturates, no walk
    edges = [(i, i + 1, 16 * i + j + 1) for i in range(16) for j in range(16)]
    a = np.array(edges, dtype=np.int32)
    g = oracle.Graph(17, a[:, 0].copy(), a[:, 1].copy(), a[:, 2].copy())
    rec, nv, ev = trk.path(g, "sh", 0, 16, seed=1, i=0)
    assert rec["flags"] & oracle.REC_OVERFLOW and nv.sum() == 0 and ev.sum() == 0
    rec, nv, ev = trk.path(g, "sh", 0, 15, seed=1, i=0)  # sigma = 2^60: a walk of 15 hops
    assert rec["sigma"] == 2**60 and int(ev.sum()) == 15 and int(nv.sum()) == 14
