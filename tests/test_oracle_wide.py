"""Pins of the oracle's exact (unbounded-integer) pair counts.

* equal integers to brute-force walk enumeration on random tiny graphs, all
  optimalities, with windows;
* equal to the 64-bit oracle wherever that one did not saturate;
* closed forms beyond 64 bits: a line of k hops with p parallel edges at
  increasing times has sigma_sh = p^k, sigma_sfm = p^(k-1) (the last hop
  must take its earliest edge) and every internal node on every walk;
  complete layered graphs of widths w_i (all edges of a layer at one time)
  have sigma = prod w_i and N(v) = sigma / w_i for a node of layer i.
"""
import numpy as np
import pytest

import oracle
from oracle import wide
from brute import OPTS, all_walks, pair_brute
from test_oracle_brute import tiny_graph


@pytest.mark.parametrize("seed", range(10))
def test_brute_force(seed):
    rng = np.random.default_rng(9500 + seed)
    n, src, dst, t = tiny_graph(rng)
    for t0, t1 in ((0, 2**31 - 1), (2, 5)):
        for s in range(n):
            walks = all_walks(src, dst, t, s, t0, t1)
            for z in range(n):
                if z == s:
                    continue
                for opt in OPTS:
                    r1, Nv1, Ne1 = pair_brute(n, src, dst, t, s, z, opt, t0, t1, walks=walks)
                    r2, Nv2, Ne2 = wide.pair_exact(n, src, dst, t, opt, s, z, t0, t1)
                    assert {k: r2[k] for k in r1} == r1, (opt, s, z)
                    assert Nv2 == Nv1
                    assert Ne2 == {k: v for k, v in Ne1.items() if v}


def test_agrees_with_64_bit_oracle():
    from synthgen import uniform_graph
    G = uniform_graph(60, 900, 40, seed=4)
    g = oracle.Graph.of(G)
    S, Z = oracle.draw_pairs(3, 0, G.n, 0, 40)
    for opt in OPTS:
        for s, z in zip(S, Z):
            rec, nN, eN = oracle.pair(g, opt, int(s), int(z))
            r2, Nv, Ne = wide.pair_exact(G.n, G.src, G.dst, G.t, opt, int(s), int(z))
            if rec["flags"] & oracle.REC_OVERFLOW:
                continue
            assert {k: r2[k] for k in ("reachable", "t_arr", "hops", "sigma")} == \
                {k: rec[k] for k in ("reachable", "t_arr", "hops", "sigma")}
            assert [int(x) for x in nN] == Nv
            assert {k: int(x) for k, x in enumerate(eN) if x} == Ne


def parallel_line(k, p):
    e = [(i, i + 1, p * i + j + 1) for i in range(k) for j in range(p)]
    a = np.array(e, dtype=np.int64)
    return k + 1, a[:, 0], a[:, 1], a[:, 2]


@pytest.mark.parametrize("k,p", [(16, 16), (20, 16), (33, 7)])
def test_parallel_line(k, p):
    n, src, dst, t = parallel_line(k, p)
    rec, Nv, Ne = wide.pair_exact(n, src, dst, t, "sh", 0, k)
    assert rec["sigma"] == p**k and rec["hops"] == k
    assert Nv == [0] + [p**k] * (k - 1) + [0]
    assert set(Ne.values()) == {p ** (k - 1)}  # each edge on the walks through it
    rec, Nv, _ = wide.pair_exact(n, src, dst, t, "sfm", 0, k)
    assert rec["sigma"] == p ** (k - 1) and rec["t_arr"] == p * (k - 1) + 1
    rec, _, _ = wide.pair_exact(n, src, dst, t, "pfm", 0, k)
    assert rec["sigma"] == 1


def test_layered_widths():
    widths = [1, 9, 17, 5, 13, 11, 23, 29, 31, 37, 41, 43, 47, 53, 59, 61, 1]  # product > 2^64
    nodes, edges, off = [], [], 0
    for w in widths:
        nodes.append(list(range(off, off + w)))
        off += w
    for i in range(len(widths) - 1):
        for u in nodes[i]:
            for v in nodes[i + 1]:
                edges.append((u, v, i + 1))
    a = np.array(edges, dtype=np.int64)
    sigma = int(np.prod([w for w in widths], dtype=object))
    assert sigma > 2**64
    for opt in OPTS:
        rec, Nv, _ = wide.pair_exact(off, a[:, 0], a[:, 1], a[:, 2], opt, 0, off - 1)
        assert rec["sigma"] == sigma, opt
        for i, layer in enumerate(nodes[1:-1], start=1):
            for v in layer:
                assert Nv[v] == sigma // widths[i]
