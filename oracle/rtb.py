"""The oracle of the RTB estimator -- TEST INFRASTRUCTURE ONLY.

The random temporal betweenness estimator of the appendix on other
estimators: a sample is a source s drawn uniformly from the nodes, and
f(v|s) = (1/(n-1)) * sum over targets z != s of sigma_sz(v) / sigma_sz,
f(e|s) likewise for temporal edges.

* ``source`` (oracle.c ``orc_rtb``): that definition written out, target
  by target, from the pair counts of ``pair`` (double-double sums over the
  targets).  Pinned against brute-force walk enumeration on tiny graphs and
  the closed form of the time-increasing line, f(v|s) = (n-1-v)/(n-1) for
  v > s.
* ``fixed`` / ``estimate``: the estimator sums and Algorithm 1 with samples
  being sources (the first coordinate of the pair draw).
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import STREAM_BOOT, STREAM_PAIR, T_MAX, Graph, Sums, _opt, _p, draw_pairs, lib, rade_words
from . import bounds

_typed = False


def _lib():
    global _typed
    L = lib()
    if not _typed:
        P = ctypes.c_void_p
        L.orc_rtb.restype = ctypes.c_int
        L.orc_rtb.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                              P, P, P, ctypes.c_int32]
        _typed = True
    return L


def source(g: Graph, opt, s: int, t0: int = 0, t1: int = T_MAX, mode: int = 0, nthreads: int = 0):
    """(f over nodes [n], f over edges [m], reached targets, saturated?)."""
    nf = np.zeros(g.n)
    ef = np.zeros(g.m)
    reached = ctypes.c_int64()
    rc = _lib().orc_rtb(g._h, _opt(opt), int(t0), int(t1), int(s), int(mode), _p(nf), _p(ef),
                        ctypes.byref(reached), int(nthreads))
    if rc < 0:
        raise ValueError("oracle: bad source")
    return nf, ef, int(reached.value), rc == 1


def accumulate(g: Graph, opt, S, lam=None, c: int = 0, sums: Sums = None, t0: int = 0, t1: int = T_MAX,
               edges: bool = False, mode: int = 0):
    if sums is None:
        sums = Sums(g.n, g.m, c, edges)
    if lam is None:
        lam = np.zeros(len(S), dtype=np.uint64)
    for q, s in enumerate(S):
        nf, ef, reached, sat = source(g, opt, int(s), t0, t1, mode)
        if sat:
            sums.n_overflow += 1
            continue
        sums.bhi += nf
        sums.whi += nf * nf
        if c:
            sign = np.array([-1.0 if (int(lam[q]) >> j) & 1 else 1.0 for j in range(c)])
            sums.rhi.reshape(g.n, c)[:, :] += np.outer(nf, sign)
        if edges:
            sums.ehi += ef
    sums.r += len(S)
    return sums


def fixed(g: Graph, opt, r: int, seed: int, c: int = 25, t0: int = 0, t1: int = T_MAX, edges: bool = False):
    S, _ = draw_pairs(seed, STREAM_PAIR, g.n, 0, r)
    sums = accumulate(g, opt, S, rade_words(seed, 0, r), c, None, t0, t1, edges)
    return dict(node_bc=sums.B / r, edge_bc=(sums.E / r) if edges else None, sums=sums, S=S)


def estimate(g: Graph, opt, eps, delta, seed, c=25, t0=0, t1=T_MAX, max_samples=None):
    """Algorithm 1 with the RTB estimator's f (same schedule and bounds)."""
    sb = bounds.bootstrap_size(eps, delta)
    S, _ = draw_pairs(seed, STREAM_BOOT, g.n, 0, sb)
    boot = accumulate(g, opt, S, None, 0, None, t0, t1)
    rho = math.fsum(boot.B.tolist()) / sb
    vhat = min(0.25, float(np.max(boot.W)) / sb)
    om = max(sb, bounds.omega(vhat, rho, eps, delta / 2.0, g.n))
    if max_samples:
        om = min(om, int(max_samples))
    s1 = min(bounds.first_size(sb, om, vhat, eps, delta / 4.0), om)
    sums = Sums(g.n, g.m, c, False)
    prev, i = 0, 0
    while True:
        i += 1
        si = s1 if i == 1 else min(bounds.next_size(prev), om)
        k = si - prev
        S, _ = draw_pairs(seed, STREAM_PAIR, g.n, prev, k)
        accumulate(g, opt, S, rade_words(seed, prev, k), c, sums, t0, t1)
        r = si
        W = max(float(np.max(sums.W)), 0.0) / r
        M = sums.R.max(axis=0) / r
        Rc = math.fsum(M.tolist()) / c
        xi = bounds.xi(Rc, W, min(0.25, W), c, r, delta / 2.0 ** (i + 1))
        if r >= om or xi <= eps:
            break
        prev = si
    return dict(node_bc=sums.B / r, samples=r, rounds=i, xi=xi, s_boot=sb, rho_hat=rho, v_hat=vhat, omega=om,
                s1=s1)
