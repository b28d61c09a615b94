"""The oracle's bound arithmetic -- TEST INFRASTRUCTURE ONLY.

Plain float64 transcriptions of the paper's sample-size and supremum
deviation bounds, one function per statement:

* ``xi``        -- Theorem 1, Eqs. (1)-(3): the SD bound from the c-MCERA.
* ``omega``     -- Theorem 3, the numeric approximation at the end of its
                   proof: (2 v + 2 eps/3) / eps^2 * (ln(2 rho / v) + ln(1/d)).
* ``hoeffding`` -- Section 4.2: r = ln(2n/d) / (2 eps^2).
* ``first_size``-- the first schedule element of Algorithm 1: the least s in
                   [s', omega] whose Eq. (3) with R = 0 is at most eps.

Readings (the paper is silent or garbled on these):
* a round's failure share is delta_i = delta / 2^(i+1) and the bootstrap's is
  delta/2, so the shares sum to at most delta;
* the first element's search uses delta_1 = delta / 4;
* a negative Rademacher bound R~ is clamped at 0 before the square roots
  (the c-MCERA is a signed supremum and can fall below minus the
  concentration term, which would put a negative number under Eq. (2)'s
  root; the quantity it bounds is non-negative, so the clamp does not
  loosen the bound);
* omega falls back to Hoeffding's size when the bootstrap saw no internal
  node (v = 0 or rho = 0), and is never below s'.

Parity: omega with rho = v is pinned to Bernstein's sample size for one
function; the constants of xi's Eqs. (1)-(3) and omega's ln(2 rho / v)
factor beyond rho = v have no independent source ("parity unpinned" beyond
the special cases, monotonicity and statistical checks in the tests).
"""
from __future__ import annotations

import math


def xi(Rc: float, W: float, vhat: float, c: int, r: int, delta: float) -> float:
    """Theorem 1 at failure probability ``delta`` (Eqs. (1), (2), (3))."""
    L = math.log(4.0 / delta)
    Rt = Rc + math.sqrt(4.0 * W * L / (c * r))
    Rt = max(Rt, 0.0)
    R = Rt + L / r + math.sqrt((L / r) ** 2 + 2.0 * L * Rt / r)
    return 2.0 * R + math.sqrt(2.0 * L * (vhat + 4.0 * R) / r) + L / (3.0 * r)


def xi_zero(vhat: float, r: int, delta: float) -> float:
    """Eq. (3) with R set to 0 (used to pick the first sample size)."""
    L = math.log(4.0 / delta)
    return math.sqrt(2.0 * L * vhat / r) + L / (3.0 * r)


def hoeffding(n: int, eps: float, delta: float) -> int:
    return int(math.ceil(math.log(2.0 * n / delta) / (2.0 * eps * eps)))


def omega(vhat: float, rho: float, eps: float, delta: float, n: int) -> int:
    """Theorem 3 sample size at failure probability ``delta``."""
    if vhat <= 0.0 or rho <= 0.0:
        return hoeffding(n, eps, delta)
    x = (2.0 * vhat + 2.0 * eps / 3.0) / (eps * eps) * (math.log(2.0 * rho / vhat) + math.log(1.0 / delta))
    return int(math.ceil(x))


def bootstrap_size(eps: float, delta: float) -> int:
    """s' = ln(1/delta)/eps (footnote to Algorithm 1's description)."""
    return int(math.ceil(math.log(1.0 / delta) / eps))


def first_size(s_boot: int, om: int, vhat: float, eps: float, delta1: float) -> int:
    lo, hi = s_boot, om
    if xi_zero(vhat, hi, delta1) > eps:
        return hi
    while lo < hi:
        mid = (lo + hi) // 2
        if xi_zero(vhat, mid, delta1) <= eps:
            hi = mid
        else:
            lo = mid + 1
    return lo


def next_size(prev: int) -> int:
    """s_i = ceil(1.2 s_{i-1}) in integer arithmetic."""
    return max(prev + 1, (6 * prev + 4) // 5)
