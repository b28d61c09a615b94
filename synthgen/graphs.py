"""Seeded generators for directed temporal graphs and request streams.

A temporal graph is a set of triples (u, v, t) with u != v and integer t >= 1
(Preliminaries, "Temporal Graphs, and Paths": the edge set is a *set*, so
exact duplicate triples never occur).  The paper measures on public temporal
networks (Table 1); these generators stand in for them with seeded synthetic
graphs of the same kind (sparse, directed, power-law or uniform endpoints,
uniform or bursty timestamps).

Every generator returns int32 numpy arrays; nothing here computes paths,
counts or betweenness.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np


@dataclasses.dataclass
class TemporalGraph:
    n: int
    src: np.ndarray  # int32 [m]
    dst: np.ndarray  # int32 [m]
    t: np.ndarray  # int32 [m]
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.src.shape[0])

    @property
    def t_min(self) -> int:
        return int(self.t.min()) if self.m else 0

    @property
    def t_max(self) -> int:
        return int(self.t.max()) if self.m else 0


def _dup_mask(src: np.ndarray, dst: np.ndarray, t: np.ndarray, n: int) -> np.ndarray:
    """True at every position whose triple already occurred at a lower index
    (a hash table over the packed triples: every occurrence but the first)."""
    import pandas as pd
    tmax = int(t.max()) + 1 if t.size else 1
    key = (src.astype(np.int64) * n + dst.astype(np.int64)) * tmax + t.astype(np.int64)
    return pd.Series(key).duplicated(keep="first").to_numpy()


def _inv_cdf(cum: np.ndarray, x: np.ndarray) -> np.ndarray:
    """searchsorted(cum, x, side="right") for unsorted x, done on sorted x
    (a merge instead of one cache-missing binary search per draw)."""
    order = np.argsort(x)
    out = np.empty(x.shape[0], dtype=np.int64)
    out[order] = np.searchsorted(cum, x[order], side="right")
    return out


def _draw(rng: np.random.Generator, k: int, n: int, cum: Optional[np.ndarray]):
    if cum is None:
        u = rng.integers(0, n, size=k, dtype=np.int64)
        v = rng.integers(0, n - 1, size=k, dtype=np.int64)
        v = v + (v >= u)
        return u, v
    u = _inv_cdf(cum, rng.random(k))
    v = _inv_cdf(cum, rng.random(k))
    np.minimum(u, n - 1, out=u)
    np.minimum(v, n - 1, out=v)
    return u.astype(np.int64), v.astype(np.int64)


def _endpoints_for_times(rng, n, t, cum):
    """Draw endpoints for every timestamp in ``t``; redraw self-loops and
    duplicate triples until the triples form a set of exactly len(t)."""
    m = t.shape[0]
    u, v = _draw(rng, m, n, cum)
    bad = (u == v) | _dup_mask(u, v, t, n)
    while bad.any():
        idx = np.nonzero(bad)[0]
        nu, nv = _draw(rng, idx.shape[0], n, cum)
        u[idx] = nu
        v[idx] = nv
        bad = (u == v) | _dup_mask(u, v, t, n)
    return u.astype(np.int32), v.astype(np.int32)


def uniform_times(rng: np.random.Generator, m: int, T: int) -> np.ndarray:
    return rng.integers(1, T + 1, size=m, dtype=np.int64).astype(np.int32)


def pareto_renewal_times(rng: np.random.Generator, m: int, T: int, alpha: float = 1.5) -> np.ndarray:
    """Bursty event times: a renewal process with Pareto(alpha, x_m=1) gaps,
    min-max scaled and floored onto the integer ticks [1, T]."""
    gaps = (1.0 - rng.random(m)) ** (-1.0 / alpha)
    c = np.cumsum(gaps)
    lo, hi = c[0], c[-1]
    if hi <= lo:
        return np.ones(m, dtype=np.int32)
    x = np.floor((c - lo) / (hi - lo) * (T - 1)).astype(np.int64) + 1
    np.clip(x, 1, T, out=x)
    return x.astype(np.int32)


def uniform_graph(n: int, m: int, T: int, seed: int, name: str = "") -> TemporalGraph:
    """Endpoints uniform over ordered pairs u != v, times uniform on [1, T]."""
    rng = np.random.default_rng(seed)
    t = uniform_times(rng, m, T)
    u, v = _endpoints_for_times(rng, n, t, None)
    return TemporalGraph(n, u, v, t, name)


def chung_lu_weights(n: int, gamma: float) -> np.ndarray:
    return (np.arange(1, n + 1, dtype=np.float64)) ** (-1.0 / (gamma - 1.0))


def chung_lu_graph(n: int, m: int, gamma: float, T: int, seed: int, times: str = "uniform",
                   alpha: float = 1.5, permute: bool = True, name: str = "") -> TemporalGraph:
    """Directed Chung-Lu graph: tails and heads are drawn independently with
    probability proportional to w_i = i^(-1/(gamma-1)) over the same node
    order (so in- and out-degree correlate).  Node ids are then shuffled by one
    random permutation so that an id says nothing about the degree."""
    rng = np.random.default_rng(seed)
    w = chung_lu_weights(n, gamma)
    cum = np.cumsum(w)
    cum /= cum[-1]
    if times == "uniform":
        t = uniform_times(rng, m, T)
    elif times == "pareto":
        t = pareto_renewal_times(rng, m, T, alpha)
    else:
        raise ValueError(times)
    u, v = _endpoints_for_times(rng, n, t, cum)
    if permute:
        perm = rng.permutation(n).astype(np.int32)
        u = perm[u]
        v = perm[v]
    # one more shuffle of the edge order: generators never hand out sorted input
    order = rng.permutation(m)
    return TemporalGraph(n, u[order], v[order], t[order], name)


def packed_uniform_graphs(G: int, seed: int, n_lo: int = 1000, n_hi: int = 100000,
                          edges_per_node: int = 20, T: int = 10000):
    """G independent uniform temporal graphs with n log-uniform in [n_lo, n_hi]
    and |E| = edges_per_node * n."""
    rng = np.random.default_rng(seed)
    ns = np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), size=G)).astype(np.int64)
    seeds = rng.integers(0, 2**62, size=G)
    return [uniform_graph(int(ns[g]), int(edges_per_node * ns[g]), T, int(seeds[g]), name=f"pk{g}")
            for g in range(G)]


def request_stream(n_req: int, rate: float, t_min: int, t_max: int, seed: int):
    """Poisson arrivals; each request covers a window of U[0.05,1] of the span
    at a uniform offset, an optimality uniform over the four, eps in
    {0.01, 0.005} and delta = 0.1."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_req)
    arrive = np.cumsum(gaps) - gaps[0]
    span = t_max - t_min
    out = []
    for i in range(n_req):
        frac = rng.uniform(0.05, 1.0)
        width = max(1, int(round(frac * span)))
        off = int(rng.integers(0, span - width + 1)) if span - width >= 0 else 0
        t0 = t_min + off
        t1 = min(t_max, t0 + width)
        out.append({
            "arrival_s": float(arrive[i]),
            "t0": int(t0),
            "t1": int(t1),
            "opt": int(rng.integers(0, 4)),
            "eps": float(rng.choice([0.01, 0.005])),
            "delta": 0.1,
            "seed": int(rng.integers(0, 2**62)),
        })
    return out


# Workload recipes.  Seeds per workload k: graph 1000+k, pair stream 2000+k,
# request stream 4000+k.
WORKLOADS = {
    "tiny-uniform-n100": dict(kind="uniform", n=100, m=2000, T=100, gseed=1001, pseed=2001,
                              opt="sh", r=500),
    "mid-chunglu-n50k": dict(kind="chung_lu", n=50_000, m=2_000_000, gamma=2.3, T=100_000,
                             times="pareto", gseed=1002, pseed=2002, opt="sfm", r=20_000),
    "big-chunglu-n1m": dict(kind="chung_lu", n=1_000_000, m=20_000_000, gamma=2.1, T=1_000_000,
                            times="uniform", gseed=1003, pseed=2003, opt="pfm", eps=0.005,
                            delta=0.1, c=16, s1=4096),
    "packed-256": dict(kind="packed", G=256, gseed=1004, pseed=2004, opt="sh", r_per_graph=2000),
    "serve-chunglu-n2m": dict(kind="chung_lu", n=2_000_000, m=50_000_000, gamma=2.3, T=1_000_000,
                              times="pareto", gseed=1005, pseed=2005, rseed=4005, rate=50.0,
                              n_req=1000),
}


def workload(name: str, scale: float = 1.0):
    """Build the graph of a named workload.  ``scale`` < 1 shrinks n and |E|
    proportionally (same recipe) for quick tests."""
    w = dict(WORKLOADS[name])
    if w["kind"] == "packed":
        return packed_uniform_graphs(w["G"], w["gseed"])
    n = max(8, int(round(w["n"] * scale)))
    m = max(8, int(round(w["m"] * scale)))
    if w["kind"] == "uniform":
        return uniform_graph(n, m, w["T"], w["gseed"], name=name)
    return chung_lu_graph(n, m, w["gamma"], w["T"], w["gseed"], times=w["times"], name=name)
