"""Pins of the oracle of Algorithm 2 (sampled temporal distance metrics).

* per-source distances against brute-force walk enumeration (every source,
  every target, all four optimalities, whole span and windows);
* hand-worked graphs where the optimalities give different distances;
* closed forms of the time-increasing and time-decreasing lines;
* with every node taken once as a source, the formulas give the exact
  diameter, connectivity rate, average distance and average number of
  internal nodes, computed here straight from their definitions over all
  pairs' brute-force distances;
* with a sample of sources, the per-source forms of the theorem's proof
  (zeta as the mean of |N(u, D)| / (n - 1), Psi as a ratio of sums) and the
  invariance under repeating the whole sample;
* the sample-size statement: r = ln n / eps^2 sources give zeta within eps.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import distances as od
from brute import OPTS, all_walks, pair_brute
from test_oracle_brute import tiny_graph


def brute_hops(n, src, dst, t, opt, t0=0, t1=2**31 - 1):
    H = np.full((n, n), -1, dtype=np.int64)
    for s in range(n):
        walks = all_walks(src, dst, t, s, t0, t1)
        for z in range(n):
            if z != s:
                rec, _, _ = pair_brute(n, src, dst, t, s, z, opt, t0, t1, walks=walks)
                if rec["reachable"]:
                    H[s, z] = rec["hops"]
    return H


@pytest.mark.parametrize("seed", range(12))
def test_source_hops_brute(seed):
    rng = np.random.default_rng(7000 + seed)
    n, src, dst, t = tiny_graph(rng)
    g = oracle.Graph(n, src, dst, t)
    windows = [(0, 2**31 - 1), (2, 4)]
    for t0, t1 in windows:
        for opt in OPTS:
            want = brute_hops(n, src, dst, t, opt, t0, t1)
            for mode in (0, 1):
                got = od.source_hops(g, opt, np.arange(n), t0, t1, mode=mode)
                assert (got == want).all(), (opt, mode, t0, t1, got.tolist(), want.tolist())


def test_hand_worked_optimalities():
    # s=0 -> z=3 directly at t=10; 0 -> 1 at t=1, 1 -> 2 at t=2, 2 -> 3 at t=3;
    # 0 -> 2 at t=5.  sh: d(0,3)=1, d(0,2)=1.  sfm / fm: 3 first reached at
    # t=3 by 0-1-2-3 (3 hops); 2 first reached at t=2 (2 hops).  pfm: the
    # same walks (every prefix is foremost).
    src = np.array([0, 0, 1, 2, 0], dtype=np.int32)
    dst = np.array([3, 1, 2, 3, 2], dtype=np.int32)
    t = np.array([10, 1, 2, 3, 5], dtype=np.int32)
    g = oracle.Graph(4, src, dst, t)
    want = {"sh": [-1, 1, 1, 1], "sfm": [-1, 1, 2, 3], "fm": [-1, 1, 2, 3], "pfm": [-1, 1, 2, 3]}
    for opt, w in want.items():
        assert od.source_hops(g, opt, [0])[0].tolist() == w, opt
    # a foremost arrival whose fewest hops is not the pfm walk's: 0->1 (t=1),
    # 1->2 (t=2), 0->2 (t=2) and 2->3 (t=3): 2 is first reached at t=2 in one
    # hop (sfm) and by 0-1-2 too; pfm counts both, its distance is their
    # fewest hops (1); 3 is at 2 hops for every optimality
    src = np.array([0, 1, 0, 2], dtype=np.int32)
    dst = np.array([1, 2, 2, 3], dtype=np.int32)
    t = np.array([1, 2, 2, 3], dtype=np.int32)
    g = oracle.Graph(4, src, dst, t)
    for opt in OPTS:
        assert od.source_hops(g, opt, [0])[0].tolist() == [-1, 1, 1, 2], opt


def line(n, increasing=True):
    src = np.arange(n - 1, dtype=np.int32)
    dst = src + 1
    t = (src + 1) if increasing else (n - src)
    return src, dst, t.astype(np.int32)


@pytest.mark.parametrize("n", [2, 3, 7, 20])
def test_line_closed_forms(n):
    src, dst, t = line(n)
    g = oracle.Graph(n, src, dst, t)
    for opt in OPTS:
        H = od.source_hops(g, opt, np.arange(n))
        for u in range(n):
            for v in range(n):
                assert H[u, v] == (v - u if v > u else -1)
        res = od.algorithm2(n, n, od.hop_counts(H), 1.0)
        assert res["d_lb"] == n - 1 and res["d_tau"] == n - 1
        assert res["zeta"] == 0.5
        assert math.isclose(res["psi"], (n + 1) / 3.0, rel_tol=1e-15)
        rho = sum((n - d) * (d - 1) for d in range(1, n)) / (n * (n - 1))
        assert math.isclose(res["rho"], rho, rel_tol=1e-15, abs_tol=0.0)
        # effective diameter: least h with sum_{d<=h} (n - d) >= tau n(n-1)/2
        for tau in (0.0, 0.3, 0.5, 0.9):
            cum, want = 0, None
            for h in range(1, n):
                cum += n - h
                if cum >= tau * n * (n - 1) / 2:
                    want = h
                    break
            if tau == 0.0:
                want = 0
            assert od.algorithm2(n, n, od.hop_counts(H), tau)["d_tau"] == want, (n, tau)


@pytest.mark.parametrize("n", [3, 9])
def test_decreasing_line(n):
    src, dst, t = line(n, increasing=False)
    g = oracle.Graph(n, src, dst, t)
    for opt in OPTS:
        res = od.algorithm2(n, n, od.hop_counts(od.source_hops(g, opt, np.arange(n))), 0.9)
        assert res["d_lb"] == 1 and res["d_tau"] == 1 and res["psi"] == 1.0 and res["rho"] == 0.0
        assert math.isclose(res["zeta"], 1.0 / n, rel_tol=1e-15)


@pytest.mark.parametrize("seed", range(8))
def test_all_sources_give_exact_quantities(seed):
    rng = np.random.default_rng(7100 + seed)
    n, src, dst, t = tiny_graph(rng, n_lo=4, n_hi=7)
    for opt in OPTS:
        H = brute_hops(n, src, dst, t, opt)
        d = H[H >= 0]
        res = od.algorithm2(n, n, od.hop_counts(H), 1.0)
        # definitions over all ordered pairs of distinct nodes
        assert res["d_lb"] == (int(d.max()) if d.size else 0)
        assert res["reached_pairs"] == d.size
        assert math.isclose(res["zeta"], d.size / (n * (n - 1)), rel_tol=1e-15)
        if d.size:
            assert math.isclose(res["psi"], float(d.mean()), rel_tol=1e-13)
            assert res["d_tau"] == res["d_lb"]  # tau = 1: the diameter itself
        else:
            assert res["psi"] == 0.0 and res["d_tau"] == -1
        assert math.isclose(res["rho"], float(np.sum(d - 1)) / (n * (n - 1)), rel_tol=1e-13, abs_tol=1e-300)


@pytest.mark.parametrize("seed", range(4))
def test_sampled_sources_forms(seed):
    rng = np.random.default_rng(7200 + seed)
    n, src, dst, t = tiny_graph(rng, n_lo=5, n_hi=7)
    g = oracle.Graph(n, src, dst, t)
    S = rng.integers(0, n, size=11).astype(np.int32)
    for opt in OPTS:
        H = od.source_hops(g, opt, S)
        res = od.algorithm2(n, len(S), od.hop_counts(H), 0.5)
        reach = (H >= 0).sum(axis=1)
        # zeta = mean over the sampled sources of |N(u, D)| / (n - 1)
        assert math.isclose(res["zeta"], float(np.mean(reach / (n - 1))), rel_tol=1e-14)
        if reach.sum():
            dsum = np.where(H >= 0, H, 0).sum()
            assert math.isclose(res["psi"], dsum / reach.sum(), rel_tol=1e-14)
        # the sample repeated twice: the same estimates
        H2 = np.concatenate([H, H])
        assert od.algorithm2(n, 2 * len(S), od.hop_counts(H2), 0.5) == dict(res, sources=2 * len(S),
                                                                           reached_pairs=2 * res["reached_pairs"])


def test_sources_are_the_pair_draws_first_coordinate():
    S = od.draw_sources(99, 1000, 64)
    S2, _ = oracle.draw_pairs(99, od.STREAM_SRC, 1000, 0, 64)
    assert (S == S2).all() and S.min() >= 0 and S.max() < 1000
    counts = np.bincount(od.draw_sources(5, 10, 20000), minlength=10)
    assert counts.min() > 1800 and counts.max() < 2200


def test_zeta_within_eps_at_theorem_sample_size():
    from synthgen import uniform_graph
    G = uniform_graph(40, 120, 50, seed=3)
    g = oracle.Graph.of(G)
    exact = od.algorithm2(G.n, G.n, od.hop_counts(od.source_hops(g, "sh", np.arange(G.n))), 0.9)
    eps = 0.15
    r = int(math.ceil(math.log(G.n) / eps ** 2))
    for seed in range(10):
        _, res = od.distances(g, "sh", r, seed)
        assert abs(res["zeta"] - exact["zeta"]) <= eps, (seed, res, exact)


def test_hist_of_clamps():
    h = od.hist_of({1: 3, 2: 5, 7: 1}, 4)
    assert h.tolist() == [0, 3, 5, 1]
