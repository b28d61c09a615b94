"""Pins of the oracle's random numbers, bound arithmetic and progressive loop.
CPU only."""
import math

import numpy as np
import pytest

import oracle
from oracle import bounds, mantra
from synthgen import uniform_graph


def test_splitmix64_published_outputs():
    """SplitMix64 (Steele, Lea, Flood 2014): the first outputs of the
    reference generator seeded with 1234567, and with 0."""
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    assert [oracle.splitmix_nth(1234567, k) for k in range(1, 6)] == want
    assert oracle.splitmix_nth(0, 1) == 0xE220A8397B1DCDAF


def test_word_is_keyed_splitmix():
    key = oracle.splitmix_nth(42, 1 + 3)
    assert oracle.word(42, 3, 5, 2) == oracle.splitmix_nth(key, 4 * 5 + 2 + 1)


def test_pairs_uniform_over_ordered_pairs():
    """Pairs are uniform over s != z (Section 4.1): chi-square on n = 6."""
    n = 6
    k = 60_000
    S, Z = oracle.draw_pairs(7, oracle.STREAM_PAIR, n, 0, k)
    assert np.all(S != Z) and S.min() >= 0 and Z.max() < n
    cnt = np.zeros((n, n))
    np.add.at(cnt, (S, Z), 1)
    exp = k / (n * (n - 1))
    chi2 = sum((cnt[s, z] - exp) ** 2 / exp for s in range(n) for z in range(n) if s != z)
    # 29 degrees of freedom: P(chi2 > 58.3) ~ 1e-3
    assert chi2 < 58.3


def test_pairs_index_based():
    """Pair i is a function of (seed, stream, i) only."""
    S1, Z1 = oracle.draw_pairs(3, 0, 1000, 0, 50)
    S2, Z2 = oracle.draw_pairs(3, 0, 1000, 20, 30)
    assert np.array_equal(S1[20:], S2) and np.array_equal(Z1[20:], Z2)


def test_xi_zero_sample_closed_form():
    """With R^c = W = v = 0, Eq. (1) gives R~ = 0, Eq. (2) gives R = 2L/r and
    Eq. (3) gives xi = 4L/r + 4L/r + L/(3r) = (25/3) L / r."""
    for r in (10, 1000, 123457):
        for d in (0.1, 0.01):
            L = math.log(4 / d)
            assert bounds.xi(0.0, 0.0, 0.0, 25, r, d) == pytest.approx(25.0 / 3.0 * L / r, rel=1e-14)


def test_xi_limits_and_monotonicity():
    """xi falls with r at fixed per-sample statistics, grows with W, v and
    R^c, and shrinks towards 2 R^c as r grows (every other term vanishes)."""
    prev = float("inf")
    for r in (100, 1000, 10_000, 100_000, 10**7):
        x = bounds.xi(0.01, 0.02, 0.02, 16, r, 0.05)
        assert x < prev
        prev = x
    assert bounds.xi(0.01, 0.02, 0.02, 16, 10**12, 0.05) == pytest.approx(0.02, rel=1e-3)
    base = bounds.xi(0.01, 0.02, 0.02, 16, 5000, 0.05)
    assert bounds.xi(0.02, 0.02, 0.02, 16, 5000, 0.05) > base
    assert bounds.xi(0.01, 0.04, 0.02, 16, 5000, 0.05) > base
    assert bounds.xi(0.01, 0.02, 0.04, 16, 5000, 0.05) > base
    assert bounds.xi(0.01, 0.02, 0.02, 16, 5000, 0.01) > base


def test_hoeffding_union_bound():
    """r = ln(2n/delta)/(2 eps^2) makes the union of n two-sided Hoeffding
    tails 2 n exp(-2 r eps^2) at most delta."""
    for n, e, d in [(100, 0.05, 0.1), (10**6, 0.005, 0.1), (50_000, 0.01, 0.01)]:
        r = bounds.hoeffding(n, e, d)
        assert 2 * n * math.exp(-2 * r * e * e) <= d
        assert 2 * n * math.exp(-2 * (r - 1) * e * e) > d


def test_omega_monotone():
    """Theorem 3's size grows with rho, shrinks with eps and delta."""
    base = bounds.omega(0.01, 3.0, 0.01, 0.05, 1000)
    assert bounds.omega(0.01, 6.0, 0.01, 0.05, 1000) > base
    assert bounds.omega(0.01, 3.0, 0.02, 0.05, 1000) < base
    assert bounds.omega(0.01, 3.0, 0.01, 0.10, 1000) < base
    assert bounds.omega(0.0, 3.0, 0.01, 0.05, 1000) == bounds.hoeffding(1000, 0.01, 0.05)


def test_first_size_is_least():
    for v in (0.0, 0.001, 0.01, 0.2):
        s = bounds.first_size(50, 10**6, v, 0.01, 0.025)
        assert bounds.xi_zero(v, s, 0.025) <= 0.01
        if s > 50:
            assert bounds.xi_zero(v, s - 1, 0.025) > 0.01


def test_next_size_is_ceil_six_fifths():
    for p in range(1, 2000):
        assert bounds.next_size(p) == max(p + 1, -(-6 * p // 5))


@pytest.fixture(scope="module")
def tiny():
    G = uniform_graph(60, 900, 60, seed=1101)
    g = oracle.Graph.of(G)
    S, Z = zip(*[(s, z) for s in range(G.n) for z in range(G.n) if s != z])
    sums, _ = oracle.accumulate(g, "sh", np.array(S), np.array(Z))
    return G, g, sums.B / (G.n * (G.n - 1))


def test_progressive_guarantee(tiny):
    """Theorem 5: with probability >= 1 - delta the output's supremum
    deviation from the exact betweenness is at most eps.  Over 40 seeds at
    delta = 0.1 the failure count must stay well below the 4 the bound
    allows (the paper reports SD <= eps on every run)."""
    G, g, exact = tiny
    eps, delta = 0.02, 0.1
    fails = 0
    for seed in range(40):
        out = mantra.estimate(g, "sh", eps, delta, seed, c=16)
        sd = float(np.max(np.abs(out["node_bc"] - exact)))
        fails += sd > eps
        assert out["samples"] <= out["omega"]
        assert out["xi"] <= eps or out["samples"] >= out["omega"]
    assert fails <= 4


def test_fixed_r_is_unbiased_mean(tiny):
    """The ob estimator is unbiased (Section 4.1): its mean over a large
    sample approaches the exact betweenness."""
    G, g, exact = tiny
    out = mantra.fixed(g, "sh", 20_000, seed=5, c=4)
    assert float(np.max(np.abs(out["node_bc"] - exact))) < 0.01
