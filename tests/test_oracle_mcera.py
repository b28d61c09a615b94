"""Pins of the oracle's round statistics (Section 4.2, Theorem 1's inputs;
Algorithm 1's per-round update of the estimates) and of Theorem 3's sample
size, to values computed here independently of the oracle.  CPU only.

* W = max_v (1/r) sum_i f_i(v)^2 (the empirical wimpy variance) and
  R^c = (1/c) sum_j max_v (1/r) sum_i lambda_{j,i} f_i(v) (the c-MCERA: a
  signed supremum over every node, untouched ones included) are computed
  from f values that brute-force walk enumeration gives as exact fractions,
  on the oracle's own pair list and sign words.  A slip such as f written for
  f^2, or |.| taken for the signed supremum, changes the value here: the last
  test plants both in the oracle's outputs and checks that the comparison
  fails.
* Special sign words: every lambda = +1 gives R^c = max_v sum f / r; every
  lambda = -1 gives R^c = -min_v sum f / r.
* Theorem 3 with rho = v is the sample size of Bernstein's inequality for one
  function with values in [0, 1] (two-sided): the least r with
  2 exp(-r eps^2 / (2 v + 2 eps / 3)) <= delta.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from brute import all_walks, pair_brute
from oracle import bounds, mantra
from test_oracle_brute import tiny_graph

OPTS = ("sh", "fm", "sfm", "pfm")


def brute_sums(n, src, dst, t, opt, S, Z, lam, c):
    """Exact per-node sums of f, f^2 and lambda_j f over the pairs (fractions)."""
    walks = {}
    B = [Fraction(0)] * n
    W = [Fraction(0)] * n
    R = [[Fraction(0)] * c for _ in range(n)]
    for q, (s, z) in enumerate(zip(S.tolist(), Z.tolist())):
        if s not in walks:
            walks[s] = all_walks(src, dst, t, s)
        rec, Nv, _ = pair_brute(n, src, dst, t, s, z, opt, walks=walks[s])
        if rec["sigma"] == 0:
            continue
        for v in range(n):
            if Nv[v]:
                f = Fraction(Nv[v], rec["sigma"])
                B[v] += f
                W[v] += f * f
                for j in range(c):
                    R[v][j] += -f if (int(lam[q]) >> j) & 1 else f
    return B, W, R


def brute_stats(B, W, R, r, c):
    w = max(W) / r
    rc = sum(max(R[v][j] for v in range(len(R))) for j in range(c)) / (c * r)
    return float(w), float(rc)


def oracle_stats(n, src, dst, t, opt, S, Z, lam, c):
    g = oracle.Graph(n, src, dst, t)
    sums, _ = oracle.accumulate(g, opt, S, Z, lam, c=c, mode=0)
    W, Rc, _ = mantra.round_stats(sums, len(S))
    return sums, W, Rc


def case(seed, r=40, c=6):
    rng = np.random.default_rng(50_000 + seed)
    n, src, dst, t = tiny_graph(rng, n_lo=5, n_hi=6, m_hi=34, T_hi=3)
    S, Z = oracle.draw_pairs(777 + seed, oracle.STREAM_PAIR, n, 0, r)
    lam = np.array([oracle.word(777 + seed, oracle.STREAM_RADE, q, 0) for q in range(r)], dtype=np.uint64)
    return n, src, dst, t, S, Z, lam, c


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("opt", OPTS)
def test_round_stats_against_brute_force(seed, opt):
    n, src, dst, t, S, Z, lam, c = case(seed)
    B, W, R = brute_sums(n, src, dst, t, opt, S, Z, lam, c)
    w_want, rc_want = brute_stats(B, W, R, len(S), c)
    sums, w_got, rc_got = oracle_stats(n, src, dst, t, opt, S, Z, lam, c)
    assert w_got == pytest.approx(w_want, rel=1e-12, abs=1e-15)
    assert rc_got == pytest.approx(rc_want, rel=1e-12, abs=1e-15)
    for v in range(n):
        assert sums.B[v] == pytest.approx(float(B[v]), rel=1e-12, abs=1e-15)
        assert sums.W[v] == pytest.approx(float(W[v]), rel=1e-12, abs=1e-15)


def test_cases_exercise_fractional_f():
    """The cases above must hold dependencies strictly between 0 and 1 (else
    f^2 = f and the comparison could not tell them apart)."""
    for opt in OPTS:
        frac = 0
        for seed in range(12):
            n, src, dst, t, S, Z, lam, c = case(seed)
            B, W, R = brute_sums(n, src, dst, t, opt, S, Z, lam, c)
            frac += sum(1 for v in range(n) if W[v] != B[v])
        assert frac >= 10, opt


@pytest.mark.parametrize("opt", OPTS)
def test_all_plus_signs(opt):
    """lambda_{j,i} = +1 for every i, j: R^c = max_v sum_i f_i(v) / r."""
    n, src, dst, t, S, Z, _, c = case(3)
    lam = np.zeros(len(S), dtype=np.uint64)
    B, _, _ = brute_sums(n, src, dst, t, opt, S, Z, lam, 0)
    _, _, rc = oracle_stats(n, src, dst, t, opt, S, Z, lam, c)
    assert rc == pytest.approx(float(max(B)) / len(S), rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("opt", OPTS)
def test_all_minus_signs(opt):
    """lambda_{j,i} = -1 for every i, j: R^c = max_v (-sum_i f_i(v)) / r =
    -min_v sum_i f_i(v) / r, over every node (the source of every pair and
    nodes no optimal walk visits have sum 0, so here R^c = 0 while the
    supremum of |.| would be max_v sum f / r > 0)."""
    n, src, dst, t, S, Z, _, c = case(3)
    lam = np.full(len(S), (1 << 64) - 1, dtype=np.uint64)
    B, _, _ = brute_sums(n, src, dst, t, opt, S, Z, lam, 0)
    _, _, rc = oracle_stats(n, src, dst, t, opt, S, Z, lam, c)
    assert rc == pytest.approx(-float(min(B)) / len(S), rel=1e-12, abs=1e-15)
    # a graph where every node is internal to some sampled pair's walks:
    # the directed cycle 0 -> 1 -> ... -> n-1 -> 0 at increasing times, pairs
    # (i, i+2 mod n) whose one walk visits i+1
    n2 = 6
    src2 = np.arange(n2, dtype=np.int32)
    dst2 = ((np.arange(n2) + 1) % n2).astype(np.int32)
    t2 = np.arange(1, n2 + 1, dtype=np.int32)
    S2 = np.arange(n2 - 1, dtype=np.int32)
    Z2 = ((S2 + 2) % n2).astype(np.int32)
    lam2 = np.full(len(S2), (1 << 64) - 1, dtype=np.uint64)
    B2, _, _ = brute_sums(n2, src2, dst2, t2, opt, S2, Z2, lam2, 0)
    _, _, rc2 = oracle_stats(n2, src2, dst2, t2, opt, S2, Z2, lam2, 3)
    assert rc2 == pytest.approx(-float(min(B2)) / len(S2), rel=1e-12, abs=1e-15)


def test_line_wimpy_variance():
    """sh on the time-increasing line 0 -> 1 -> ... -> n-1 (edge i at time
    i+1): every f is 0 or 1, so W = max_v sum_i f_i(v) / r; over all ordered
    pairs that sum is v (n-1-v), largest at the middle node."""
    n = 9
    src = np.arange(n - 1, dtype=np.int32)
    dst = src + 1
    t = src + 1
    S, Z = zip(*[(s, z) for s in range(n) for z in range(n) if s != z])
    S, Z = np.array(S, dtype=np.int32), np.array(Z, dtype=np.int32)
    r = len(S)
    lam = np.zeros(r, dtype=np.uint64)
    _, W, Rc = oracle_stats(n, src, dst, t, "sh", S, Z, lam, 4)
    best = max(v * (n - 1 - v) for v in range(n))
    assert W == pytest.approx(best / r, rel=1e-14)
    assert Rc == pytest.approx(best / r, rel=1e-14)


def test_planted_slips_are_caught():
    """The comparison above fails when f is summed in place of f^2, or when
    the supremum is taken over |.|: both slips planted in the oracle's
    outputs."""
    caught_w = caught_abs = 0
    for opt in OPTS:
        for seed in range(13):
            n, src, dst, t, S, Z, lam, c = case(seed % 12)
            if seed == 12:  # every sign -1 (random words often agree with |.|)
                lam = np.full(len(S), (1 << 64) - 1, dtype=np.uint64)
            B, W, R = brute_sums(n, src, dst, t, opt, S, Z, lam, c)
            w_want, rc_want = brute_stats(B, W, R, len(S), c)
            sums, _, _ = oracle_stats(n, src, dst, t, opt, S, Z, lam, c)
            r = len(S)
            w_slip = max(float(np.max(sums.B)), 0.0) / r           # f for f^2
            rc_slip = math.fsum(np.abs(sums.R).max(axis=0).tolist()) / (c * r)  # |.| for the signed sup
            caught_w += not (w_slip == pytest.approx(w_want, rel=1e-12, abs=1e-15))
            caught_abs += not (rc_slip == pytest.approx(rc_want, rel=1e-12, abs=1e-15))
    assert caught_w >= 8
    assert caught_abs >= 8


@pytest.mark.parametrize("v", [0.01, 0.05, 0.1, 0.25])
@pytest.mark.parametrize("eps", [0.005, 0.01, 0.05])
@pytest.mark.parametrize("delta", [0.01, 0.1])
def test_omega_reduces_to_bernstein(v, eps, delta):
    """Theorem 3 with rho = v: ln(2 rho / v) + ln(1/delta) = ln(2/delta), the
    size Bernstein's inequality gives for one function in [0, 1] with
    variance v: the least r with 2 exp(-r eps^2 / (2 v + 2 eps / 3)) <= delta.
    The failure share is passed as it is (Algorithm 1 passes delta/2)."""
    om = bounds.omega(v, v, eps, delta, 1000)

    def tail(r):
        return 2.0 * math.exp(-r * eps * eps / (2.0 * v + 2.0 * eps / 3.0))

    assert tail(om) <= delta * (1 + 1e-12)
    assert tail(om - 1) > delta * (1 - 1e-12)
