"""The oracle of the TRK estimator -- TEST INFRASTRUCTURE ONLY.

The temporal Riondato-Kornaropoulos estimator of the appendix on other
estimators: per sampled pair (s, z) one optimal walk drawn backwards with
probability 1/sigma_sz (the appendix's path sampler and its theorem), and
f(v) = 1 if v is an internal node of the walk (for fm walks, which may
revisit a node: the number of internal visits), f(e) = the walk's uses of e.

* ``path`` (oracle.c ``orc_trk_path``): the walk, on the explicit appearance
  DAG of ``pair``; its draws are arranged by edge (one draw picks the
  predecessor appearance and the edge into it at once, with the same
  probabilities as the paper's two-level choice) in the order (time, head
  id, tail id), r = floor(word * W / 2^64), the first candidate whose
  running weight exceeds r.  Pinned by brute-force walk enumeration (every
  drawn walk is optimal), by its distribution (each optimal walk about
  1/sigma_sz of the draws) and by unbiasedness (mean f over all pairs and
  many draws close to the exact betweenness).
* ``accumulate`` / ``fixed`` / ``estimate``: the estimator sums and
  Algorithm 1 with f replaced by the walk indicator; the sums are of small
  integers, so they are exact in any order.

Draw j of the pair with index i in its pair stream (stream number q, the
pair stream's) uses the SplitMix64 output (i * 2^16 + j + 1) of the
generator started at the (2^20 + q + 1)-th output of the one started at seed.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import (STREAM_BOOT, STREAM_PAIR, T_MAX, Graph, Record, Sums, _opt, _p, draw_pairs, lib,
               rade_words)
from . import bounds

_typed = False


def _lib():
    global _typed
    L = lib()
    if not _typed:
        P = ctypes.c_void_p
        L.orc_trk_path.restype = ctypes.c_int
        L.orc_trk_path.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, P, P, P]
        L.orc_trk_word.restype = ctypes.c_uint64
        L.orc_trk_word.argtypes = [ctypes.c_uint64] * 4
        _typed = True
    return L


def trk_word(seed: int, stream: int, i: int, j: int) -> int:
    return int(_lib().orc_trk_word(seed, stream, i, j))


def path(g: Graph, opt, s: int, z: int, seed: int, i: int, stream: int = STREAM_PAIR, t0: int = 0,
         t1: int = T_MAX):
    """(record dict, visits per node uint64[n], uses per edge uint64[m])."""
    rec = Record()
    nv = np.zeros(g.n, dtype=np.uint64)
    ev = np.zeros(g.m, dtype=np.uint64)
    rc = _lib().orc_trk_path(g._h, _opt(opt), int(t0), int(t1), int(s), int(z), int(seed), int(stream), int(i),
                             ctypes.byref(rec), _p(nv), _p(ev))
    if rc == -1:
        raise ValueError("oracle: bad pair arguments")
    if rc == -2:
        raise AssertionError("oracle: a walk step's total disagrees with its count")
    r = {"reachable": rec.reachable, "t_arr": rec.t_arr, "hops": rec.hops, "flags": rec.flags,
         "sigma": int(rec.sigma)}
    return r, nv, ev


def accumulate(g: Graph, opt, S, Z, seed: int, stream: int, i0: int, lam=None, c: int = 0, sums: Sums = None,
               t0: int = 0, t1: int = T_MAX, edges: bool = False):
    """Add the walks of pairs i0.. (S[q], Z[q]) into ``sums``."""
    S = np.asarray(S)
    Z = np.asarray(Z)
    if sums is None:
        sums = Sums(g.n, g.m, c, edges)
    if lam is None:
        lam = np.zeros(len(S), dtype=np.uint64)
    recs = []
    for q in range(len(S)):
        rec, nv, ev = path(g, opt, int(S[q]), int(Z[q]), seed, i0 + q, stream, t0, t1)
        recs.append(rec)
        if rec["flags"] & 1:
            sums.n_overflow += 1
            continue
        f = nv.astype(np.float64)
        sums.bhi += f
        sums.whi += f * f
        if c:
            sign = np.array([-1.0 if (int(lam[q]) >> j) & 1 else 1.0 for j in range(c)])
            sums.rhi.reshape(g.n, c)[:, :] += np.outer(f, sign)
        if edges:
            sums.ehi += ev.astype(np.float64)
    sums.r += len(S)
    return sums, recs


def fixed(g: Graph, opt, r: int, seed: int, c: int = 25, t0: int = 0, t1: int = T_MAX, edges: bool = False):
    S, Z = draw_pairs(seed, STREAM_PAIR, g.n, 0, r)
    lam = rade_words(seed, 0, r)
    sums, recs = accumulate(g, opt, S, Z, seed, STREAM_PAIR, 0, lam, c, None, t0, t1, edges)
    return dict(node_bc=sums.B / r, edge_bc=(sums.E / r) if edges else None, sums=sums, records=recs)


def estimate(g: Graph, opt, eps, delta, seed, c=25, t0=0, t1=T_MAX, s1_override=None, max_samples=None):
    """Algorithm 1 with the TRK estimator's f (same schedule and bounds)."""
    import math
    sb = bounds.bootstrap_size(eps, delta)
    S, Z = draw_pairs(seed, STREAM_BOOT, g.n, 0, sb)
    boot, _ = accumulate(g, opt, S, Z, seed, STREAM_BOOT, 0, None, 0, None, t0, t1)
    rho = math.fsum(boot.B.tolist()) / sb
    vhat = min(0.25, float(np.max(boot.W)) / sb)
    om = max(sb, bounds.omega(vhat, rho, eps, delta / 2.0, g.n))
    if max_samples:
        om = min(om, int(max_samples))
    s1 = s1_override or bounds.first_size(sb, om, vhat, eps, delta / 4.0)
    s1 = min(s1, om)
    sums = Sums(g.n, g.m, c, False)
    prev, i = 0, 0
    while True:
        i += 1
        si = s1 if i == 1 else min(bounds.next_size(prev), om)
        k = si - prev
        S, Z = draw_pairs(seed, STREAM_PAIR, g.n, prev, k)
        accumulate(g, opt, S, Z, seed, STREAM_PAIR, prev, rade_words(seed, prev, k), c, sums, t0, t1)
        r = si
        W = max(float(np.max(sums.W)), 0.0) / r
        M = sums.R.max(axis=0) / r
        Rc = math.fsum(M.tolist()) / c
        xi = bounds.xi(Rc, W, min(0.25, W), c, r, delta / 2.0 ** (i + 1))
        if r >= om or xi <= eps:
            break
        prev = si
    return dict(node_bc=sums.B / r, samples=r, rounds=i, xi=xi, s_boot=sb, rho_hat=rho, v_hat=vhat, omega=om,
                s1=s1, n_overflow=sums.n_overflow + boot.n_overflow)
