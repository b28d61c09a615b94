"""Algorithm 1 (MANTRA) on the oracle -- TEST INFRASTRUCTURE ONLY.

The progressive-sampling loop in the paper's order: bootstrap (s' pairs from
the BOOT stream -> rho^, v^ -> omega), first sample size, then rounds that
grow the sample geometrically, add Rademacher columns, update the sums, take
the maxima over all nodes and stop when |S_i| >= omega or xi <= eps.
"""
from __future__ import annotations

import math

import numpy as np

from . import (STREAM_BOOT, STREAM_PAIR, T_MAX, Graph, Sums, accumulate, draw_pairs,
               rade_words)
from . import bounds


def bootstrap(g: Graph, opt, eps, delta, seed, t0=0, t1=T_MAX, mode=1):
    sb = bounds.bootstrap_size(eps, delta)
    S, Z = draw_pairs(seed, STREAM_BOOT, g.n, 0, sb)
    sums, recs = accumulate(g, opt, S, Z, c=0, t0=t0, t1=t1, mode=mode)
    rho = math.fsum(sums.B.tolist()) / sb
    wb = float(np.max(sums.W)) / sb if g.n else 0.0
    vhat = min(0.25, wb)
    om = max(sb, bounds.omega(vhat, rho, eps, delta / 2.0, g.n))
    return dict(s_boot=sb, rho_hat=rho, w_boot=wb, v_hat=vhat, omega=om,
                n_overflow=sums.n_overflow)


def round_stats(sums: Sums, r: int):
    W = max(float(np.max(sums.W)), 0.0) / r
    R = sums.R
    M = R.max(axis=0) / r if sums.c else np.zeros(0)
    Rc = math.fsum(M.tolist()) / sums.c if sums.c else 0.0
    return W, Rc, M


def estimate(g: Graph, opt, eps, delta, seed, c=25, t0=0, t1=T_MAX, s1_override=None,
             max_samples=None, edges=False, mode=1, nthreads=0):
    boot = bootstrap(g, opt, eps, delta, seed, t0, t1, mode)
    om = boot["omega"]
    if max_samples:
        om = min(om, int(max_samples))
    s1 = s1_override or bounds.first_size(boot["s_boot"], om, boot["v_hat"], eps, delta / 4.0)
    s1 = min(s1, om)
    sums = Sums(g.n, g.m, c, edges)
    prev, i = 0, 0
    rounds = []
    while True:
        i += 1
        si = s1 if i == 1 else min(bounds.next_size(prev), om)
        k = si - prev
        S, Z = draw_pairs(seed, STREAM_PAIR, g.n, prev, k)
        lam = rade_words(seed, prev, k)
        accumulate(g, opt, S, Z, lam, c, sums, t0, t1, mode, edges, nthreads)
        r = si
        W, Rc, M = round_stats(sums, r)
        di = delta / 2.0 ** (i + 1)
        xi = bounds.xi(Rc, W, min(0.25, W), c, r, di)
        rounds.append(dict(r=r, W=W, Rc=Rc, xi=xi, delta_i=di))
        if r >= om or xi <= eps:
            break
        prev = si
    out = dict(boot, node_bc=sums.B / r, edge_bc=(sums.E / r) if edges else None, samples=r,
               rounds=rounds, xi=rounds[-1]["xi"], n_overflow=sums.n_overflow, s1=s1,
               omega=om, sums=sums)
    return out


def fixed(g: Graph, opt, r, seed, c=25, t0=0, t1=T_MAX, edges=False, mode=1, nthreads=0):
    """Fixed sample size: r pairs from the PAIR stream, estimates sum f / r."""
    S, Z = draw_pairs(seed, STREAM_PAIR, g.n, 0, r)
    lam = rade_words(seed, 0, r)
    sums, recs = accumulate(g, opt, S, Z, lam, c, None, t0, t1, mode, edges, nthreads)
    W, Rc, M = round_stats(sums, r) if r else (0.0, 0.0, None)
    return dict(node_bc=sums.B / r, edge_bc=(sums.E / r) if edges else None, sums=sums,
                records=recs, W=W, Rc=Rc, S=S, Z=Z)
