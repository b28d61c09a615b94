"""The oracle against brute-force walk enumeration on random tiny graphs.

Pins oracle.pair (both modes) for all four optimalities: sigma, arrival,
hops, N(v) for every node and N(e) for every temporal edge.
"""
import numpy as np
import pytest

import oracle
from brute import OPTS, all_walks, is_simple, pair_brute


def tiny_graph(rng, n_lo=3, n_hi=7, m_hi=22, T_hi=6):
    n = int(rng.integers(n_lo, n_hi + 1))
    T = int(rng.integers(1, T_hi + 1))
    m_want = int(rng.integers(2, m_hi + 1))
    trip = set()
    for _ in range(4 * m_want):
        u, v = rng.integers(0, n, 2)
        if u == v:
            continue
        trip.add((int(u), int(v), int(rng.integers(1, T + 1))))
        if len(trip) >= m_want:
            break
    trip = sorted(trip)
    rng.shuffle(trip)
    a = np.array(trip, dtype=np.int32).reshape(-1, 3)
    return n, a[:, 0].copy(), a[:, 1].copy(), a[:, 2].copy()


def check_graph(n, src, dst, t, t0=0, t1=2**31 - 1):
    g = oracle.Graph(n, src, dst, t)
    for s in range(n):
        walks = all_walks(src, dst, t, s, t0, t1)
        for z in range(n):
            if z == s:
                continue
            for opt in OPTS:
                want, wNv, wNe = pair_brute(n, src, dst, t, s, z, opt, t0, t1, walks=walks)
                for mode in (0, 1):
                    got, nN, eN = oracle.pair(g, opt, s, z, t0, t1, mode=mode)
                    ctx = (opt, s, z, mode, n, src.tolist(), dst.tolist(), t.tolist())
                    assert got["flags"] & oracle.REC_SELFCHECK == 0, ctx
                    for k in ("reachable", "t_arr", "hops", "sigma"):
                        assert got[k] == want[k], (k, got, want, ctx)
                    assert [int(x) for x in nN] == wNv, (nN.tolist(), wNv, ctx)
                    we = [wNe.get(e, 0) for e in range(len(src))]
                    assert [int(x) for x in eN] == we, (eN.tolist(), we, ctx)


@pytest.mark.parametrize("seed", range(60))
def test_random_tiny(seed):
    rng = np.random.default_rng(seed)
    n, src, dst, t = tiny_graph(rng)
    check_graph(n, src, dst, t)


@pytest.mark.parametrize("seed", range(15))
def test_random_tiny_windowed(seed):
    rng = np.random.default_rng(10_000 + seed)
    n, src, dst, t = tiny_graph(rng, T_hi=7)
    t0 = int(rng.integers(1, 4))
    t1 = int(rng.integers(t0, 8))
    check_graph(n, src, dst, t, t0, t1)


@pytest.mark.parametrize("seed", range(10))
def test_dense_ties(seed):
    """Few ticks, many edges per tick: equal times must never chain."""
    rng = np.random.default_rng(20_000 + seed)
    n, src, dst, t = tiny_graph(rng, n_lo=4, n_hi=6, m_hi=26, T_hi=3)
    check_graph(n, src, dst, t)


@pytest.mark.parametrize("seed", range(20))
def test_optimal_walks_are_simple_except_fm(seed):
    """Reading: for sh, sfm and pfm the optimal walks are simple paths, so
    counting walks equals counting the paths of Definition 1."""
    rng = np.random.default_rng(30_000 + seed)
    n, src, dst, t = tiny_graph(rng)
    for s in range(n):
        walks = all_walks(src, dst, t, s)
        arr = {}
        for w in walks:
            v = int(dst[w[-1]])
            arr[v] = min(arr.get(v, 1 << 40), int(t[w[-1]]))
        for z in range(n):
            if z == s:
                continue
            to_z = [w for w in walks if int(dst[w[-1]]) == z]
            if not to_z:
                continue
            k = min(len(w) for w in to_z)
            assert all(is_simple(w, src, dst) for w in to_z if len(w) == k)
            fore = [w for w in to_z if int(t[w[-1]]) == arr[z]]
            k2 = min(len(w) for w in fore)
            assert all(is_simple(w, src, dst) for w in fore if len(w) == k2)
