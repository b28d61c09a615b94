"""The oracle of Algorithm 2 -- TEST INFRASTRUCTURE ONLY.

Sampled temporal distance metrics (appendix on temporal distance metrics,
Algorithm 2): r sources drawn uniformly at random, a temporal BFS from each,
per-hop counts of the reached pairs, then the rescaled cumulative counts R[h]
give the diameter lower bound D_LB, the effective diameter D_tau, the
connectivity rate zeta, the average distance Psi and the average number of
internal nodes rho.

* ``source_hops`` (oracle.c ``orc_source_hops``): the distance of every node
  from one source is the hop count of the pair record of ``pair``, read for
  all targets after one forward pass.  Pinned by brute-force walk enumeration
  (tests/brute.py) on tiny graphs and by closed forms on lines and stars.
* ``algorithm2``: the closing formulas, in exact rational arithmetic (Python
  ``Fraction``), converted to float at the end.  Pinned by its definitions:
  with every node taken once as a source, D_LB, zeta, Psi and rho equal the
  exact diameter, connectivity rate and average distances computed straight
  from all pairs' distances; closed forms on the time-increasing line.

Readings (the paper's listing is garbled; each is listed in the design
notes):
* R[h] is cumulative (pairs at distance <= h): the listing's Psi sums
  (R[h] - R[h-1]) h and its zeta is R[D_LB] / (n (n - 1)), which only make
  sense for cumulative counts, and the appendix's |N(h)| is cumulative;
* the rescaling and the Psi sum run over every h in [0, D_LB] (the listing's
  loop bound D_LB - 1 would leave R[D_LB], the divisor, unscaled and drop the
  pairs at distance D_LB from Psi);
* pairs (u, u) are not counted (zeta's n (n - 1) counts ordered pairs of
  distinct nodes, and d(u, u) = 0 adds nothing to Psi);
* D_tau's test R[h] / R[D_LB] >= tau is taken as float(c_h) / float(c_D)
  >= tau on the integer counts c (the same fp64 decision on both sides; the
  n / r factor cancels exactly in the rationals);
* with no reachable sampled pair, D_LB = 0, D_tau = -1 (the listing's
  initial value) and Psi = 0;
* rho (Section 2's average number of internal nodes over all n (n - 1)
  pairs, unreachable pairs adding 0) is estimated as
  sum_h (h - 1)(R[h] - R[h-1]) / (n (n - 1)).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from . import Graph, T_MAX, _opt, _p, draw_pairs, lib

STREAM_SRC = 3
HOPS_LIMIT = 65534


def source_hops(g: Graph, opt, S, t0: int = 0, t1: int = T_MAX, mode: int = 1, nthreads: int = 0) -> np.ndarray:
    """int32 [len(S), n]: distance of every node from each source (-1: not
    reachable, or the source itself)."""
    import ctypes
    S = np.ascontiguousarray(S, dtype=np.int32)
    k = int(S.shape[0])
    out = np.empty((k, g.n), dtype=np.int32)
    L = lib()
    if not getattr(L, "_src_hops_typed", False):
        L.orc_source_hops.restype = ctypes.c_int
        L.orc_source_hops.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_int32]
        L._src_hops_typed = True
    if k:
        rc = L.orc_source_hops(g._h, _opt(opt), int(t0), int(t1), int(mode), k, _p(S), _p(out), int(nthreads))
        if rc != 0:
            raise ValueError("oracle: bad source arguments")
    return out


def draw_sources(seed: int, n: int, r: int) -> np.ndarray:
    """Sources 0..r-1 of the source stream: node = floor(word * n / 2^64),
    the first coordinate of the pair draw (uniform with replacement)."""
    S, _ = draw_pairs(seed, STREAM_SRC, n, 0, r)
    return S


def hop_counts(hops: np.ndarray) -> dict:
    """{h: number of (source, node) pairs at distance exactly h}."""
    d = hops[hops >= 0]
    vals, cnt = np.unique(d, return_counts=True)
    return {int(h): int(c) for h, c in zip(vals, cnt)}


def algorithm2(n: int, r: int, counts: dict, tau: float) -> dict:
    """Algorithm 2's closing formulas from the per-hop counts of r sources."""
    if any(h > HOPS_LIMIT for h in counts):
        raise OverflowError("distance above %d" % HOPS_LIMIT)
    d_lb = max([h for h, c in counts.items() if c > 0], default=0)
    scale = Fraction(n, r)
    # R[h]: rescaled number of sampled pairs at distance <= h
    R = []
    run = 0
    for h in range(d_lb + 1):
        run += counts.get(h, 0)
        R.append(scale * run)
    total = run
    RD = R[d_lb]
    psi = Fraction(0)
    rho_num = Fraction(0)
    for h in range(1, d_lb + 1):
        step = R[h] - R[h - 1]
        psi += step * h
        rho_num += step * (h - 1)
    d_tau = -1
    if total:
        psi = psi / RD
        run = 0
        for h in range(d_lb + 1):
            run += counts.get(h, 0)
            if float(run) / float(total) >= tau:
                d_tau = h
                break
    pairs = Fraction(n * (n - 1))
    return dict(sources=r, reached_pairs=total, d_lb=d_lb, d_tau=d_tau, zeta=float(RD / pairs),
                psi=float(psi), rho=float(rho_num / pairs))


def distances(g: Graph, opt, r: int, seed: int, tau: float = 0.9, t0: int = 0, t1: int = T_MAX,
              nthreads: int = 0):
    """Algorithm 2 with the sources of ``seed``: (counts dict, result dict)."""
    S = draw_sources(seed, g.n, r)
    counts = hop_counts(source_hops(g, opt, S, t0, t1, nthreads=nthreads))
    return counts, algorithm2(g.n, r, counts, tau)


def hist_of(counts: dict, hist_len: int) -> np.ndarray:
    """The counts as a histogram of hist_len bins, the last bin taking every
    larger distance."""
    out = np.zeros(hist_len, dtype=np.uint64)
    for h, c in counts.items():
        out[min(h, hist_len - 1)] += c
    return out
