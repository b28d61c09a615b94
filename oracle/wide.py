"""Exact pair counts beyond 64 bits -- TEST INFRASTRUCTURE ONLY.

The per-pair quantities of Definition 1 and of the estimator of Section 4.1
(sigma_sz, N(v) = sigma_sz(v), N(e), the record), computed on the explicit
appearance DAG with Python's unbounded integers, so that nothing saturates.
The paper counts with 128-bit and arbitrary-precision integers where 64 bits
do not suffice (Table 1); this is the check for the library's multiword
path.  Only for small graphs (pure Python).

Pinned by brute-force walk enumeration (equal integers on random tiny
graphs), by agreement with the 64-bit oracle wherever its counts did not
saturate, and by closed forms whose counts exceed 2^64: a line of k hops with
p parallel edges per hop has sigma = p^k and every internal node on every
walk; complete layered graphs of widths w_1..w_L have sigma = prod w_i and
N(v) = sigma / w_i for a node of layer i.
"""
from __future__ import annotations

from collections import defaultdict

T_MAX = 2**31 - 1


def pair_exact(n, src, dst, t, opt, s, z, t0=0, t1=T_MAX):
    """(record dict with exact sigma, N(v) list of ints, N(e) dict edge id -> int)."""
    m = len(src)
    win = sorted((int(t[k]), k) for k in range(m) if t0 <= int(t[k]) <= t1)
    # appearances (v, time) of the heads, per node in time order
    apps = defaultdict(list)  # v -> [times]
    head_of = {}
    for tk, k in win:
        v = int(dst[k])
        if not apps[v] or apps[v][-1] != tk:
            apps[v].append(tk)
        head_of[k] = (v, tk)
    reach, dist, sig_t, sig_w = {}, {}, {}, {}
    # forward, tick by tick: heads read the state strictly before their time
    ticks = defaultdict(list)
    for tk, k in win:
        ticks[tk].append(k)
    for tk in sorted(ticks):
        for k in ticks[tk]:
            u = int(src[k])
            a = head_of[k]
            cands = []  # (dist, level count, walk count) of counted tail appearances
            if u == s:
                cands.append((0, 1, 1))
            for tb in apps.get(u, []):
                if tb >= tk:
                    break
                b = (u, tb)
                if reach.get(b):
                    cands.append((dist[b], sig_t[b], sig_w[b]))
            if not cands:
                continue
            reach[a] = True
            d = min(c[0] for c in cands) + 1
            st = sum(c[1] for c in cands if c[0] + 1 == d)
            sw = sum(c[2] for c in cands)
            if a not in dist or d < dist[a]:
                dist[a], sig_t[a] = d, st
            elif d == dist[a]:
                sig_t[a] += st
            sig_w[a] = sig_w.get(a, 0) + sw
    # first (earliest) reached appearance of every node
    first = {}
    for v, ts in apps.items():
        for tb in ts:
            if reach.get((v, tb)):
                first[v] = (v, tb)
                break

    def pfm_app(a):
        return a[0] != s and first.get(a[0]) == a

    # prefix-foremost counts: only first appearances, fed by first appearances
    sig_p, hop_p = {}, {}
    for tk, k in win:
        u, a = int(src[k]), head_of[k]
        if not pfm_app(a):
            continue
        if u == s:
            sig_p[a] = sig_p.get(a, 0) + 1
            hop_p[a] = min(hop_p.get(a, 1 << 30), 1)
        elif u in first and first[u][1] < tk and pfm_app(first[u]):
            b = first[u]
            sig_p[a] = sig_p.get(a, 0) + sig_p.get(b, 0)
            hop_p[a] = min(hop_p.get(a, 1 << 30), hop_p.get(b, 1 << 30) + 1)

    def sig(a):
        if opt == "fm":
            return sig_w.get(a, 0) if reach.get(a) else 0
        if opt == "pfm":
            return sig_p.get(a, 0) if pfm_app(a) else 0
        return sig_t.get(a, 0) if reach.get(a) else 0

    def counted(b, h):  # b = None: the origin
        if opt == "fm":
            return b is None or bool(reach.get(b))
        if opt == "pfm":
            return pfm_app(h) and (b is None or pfm_app(b))
        if b is None:
            return dist.get(h) == 1
        return bool(reach.get(b)) and dist[b] + 1 == dist.get(h)

    rec = {"reachable": 0, "t_arr": -1, "hops": -1, "sigma": 0}
    Nv = [0] * n
    Ne = {}
    if z not in first:
        return rec, Nv, Ne
    if opt == "sh":
        d = min(dist[(z, tb)] for tb in apps[z] if reach.get((z, tb)))
        term = [(z, tb) for tb in apps[z] if reach.get((z, tb)) and dist[(z, tb)] == d]
        rec.update(reachable=1, t_arr=min(a[1] for a in term), hops=d, sigma=sum(sig_t[a] for a in term))
    else:
        a = first[z]
        term = [a]
        hops = hop_p.get(a, -1) if opt == "pfm" else dist[a]
        rec.update(reachable=1, t_arr=a[1], hops=hops, sigma=sig(a))
    termset = set(term)
    # backward: B(a) = counted continuations from a to a terminal appearance
    B = {}
    all_apps = sorted(((tb, v) for v, ts in apps.items() for tb in ts), reverse=True)
    out_edges = defaultdict(list)
    for tk, k in win:
        out_edges[int(src[k])].append(k)
    for tb, v in all_apps:
        a = (v, tb)
        if a in termset:
            B[a] = 1
            continue
        if not (pfm_app(a) if opt == "pfm" else reach.get(a)):
            continue
        total = 0
        for k in out_edges[v]:
            if int(t[k]) <= tb:
                continue
            h = head_of[k]
            if counted(a, h):
                total += B.get(h, 0)
        B[a] = total
    for v, ts in apps.items():
        if v in (s, z):
            continue
        Nv[v] = sum(sig((v, tb)) * B.get((v, tb), 0) for tb in ts)
    for tk, k in win:
        h = head_of[k]
        if not B.get(h):
            continue
        u = int(src[k])
        ts_sum = 1 if (u == s and counted(None, h)) else 0
        for tb in apps.get(u, []):
            if tb >= tk:
                break
            if counted((u, tb), h):
                ts_sum += sig((u, tb))
        if ts_sum:
            Ne[k] = ts_sum * B[h]
    return rec, Nv, Ne


def f_rows(n, m, rec, Nv, Ne):
    """f(v) and f(e) as the library forms them: the IEEE quotient of the two
    integers, each rounded to double (nearest, ties to even)."""
    import numpy as np
    fv = np.zeros(n)
    fe = np.zeros(m)
    if not rec["reachable"]:
        return fv, fe
    sg = float(rec["sigma"])
    for v, x in enumerate(Nv):
        if x:
            fv[v] = float(x) / sg
    for k, x in Ne.items():
        fe[k] = float(x) / sg
    return fv, fe
