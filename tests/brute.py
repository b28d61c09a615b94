"""Brute-force enumeration of temporal walks (a pin for the oracle).

Every walk from s is listed explicitly (depth-first, each step takes an edge
leaving the current node strictly later than the previous edge), and the
optimal ones are selected straight from Definition 1 of the paper:

* sh  : fewest hops to z;
* sfm : earliest arrival t*(z) first, then fewest hops among those;
* pfm : every prefix ending at v_i arrives at t*(v_i) (a prefix that returns
        to s is never foremost: s is reached at the origin);
* fm  : every walk arriving at t*(z) (walks, visits counted with multiplicity).

Counts are Python integers (no overflow).  Only for tiny graphs.
"""
from __future__ import annotations

from collections import defaultdict

OPTS = ("sh", "fm", "sfm", "pfm")


def all_walks(src, dst, t, s, t0=0, t1=2**31 - 1, max_walks=2_000_000):
    """All non-empty temporal walks from s as tuples of edge ids."""
    out = defaultdict(list)
    for e in range(len(src)):
        if t0 <= t[e] <= t1:
            out[int(src[e])].append(e)
    walks = []
    stack = [(s, None, ())]
    while stack:
        node, last, path = stack.pop()
        for e in out[node]:
            if last is None or t[e] > last:
                p = path + (e,)
                walks.append(p)
                if len(walks) > max_walks:
                    raise RuntimeError("graph too large for brute force")
                stack.append((int(dst[e]), int(t[e]), p))
    return walks


def pair_brute(n, src, dst, t, s, z, opt, t0=0, t1=2**31 - 1, walks=None):
    """(record, N(v) list, N(e) dict) for one pair, from explicit walks."""
    if walks is None:
        walks = all_walks(src, dst, t, s, t0, t1)
    arr = {}  # t*(v): earliest arrival at v over all walks from s
    for w in walks:
        v = int(dst[w[-1]])
        a = int(t[w[-1]])
        if v not in arr or a < arr[v]:
            arr[v] = a
    to_z = [w for w in walks if int(dst[w[-1]]) == z]
    rec = {"reachable": 0, "t_arr": -1, "hops": -1, "sigma": 0}
    Nv = [0] * n
    Ne = defaultdict(int)
    if not to_z:
        return rec, Nv, Ne
    tz = arr[z]
    if opt == "sh":
        k = min(len(w) for w in to_z)
        opt_w = [w for w in to_z if len(w) == k]
    elif opt == "sfm":
        fore = [w for w in to_z if int(t[w[-1]]) == tz]
        k = min(len(w) for w in fore)
        opt_w = [w for w in fore if len(w) == k]
    elif opt == "fm":
        opt_w = [w for w in to_z if int(t[w[-1]]) == tz]
    elif opt == "pfm":
        opt_w = []
        for w in to_z:
            ok = True
            for e in w:
                v = int(dst[e])
                if v == s or int(t[e]) != arr[v]:
                    ok = False
                    break
            if ok:
                opt_w.append(w)
    else:
        raise ValueError(opt)
    if not opt_w:
        return rec, Nv, Ne
    rec = {"reachable": 1, "t_arr": min(int(t[w[-1]]) for w in opt_w),
           "hops": min(len(w) for w in opt_w), "sigma": len(opt_w)}
    for w in opt_w:
        for e in w[:-1]:
            v = int(dst[e])
            if v != s and v != z:
                Nv[v] += 1
        for e in w:
            Ne[e] += 1
    return rec, Nv, Ne


def is_simple(w, src, dst):
    nodes = [int(src[w[0]])] + [int(dst[e]) for e in w]
    return len(nodes) == len(set(nodes))
