"""Helpers of the GPU parity tests: run the HIP library and the oracle on the
same pairs and compare element by element."""
from __future__ import annotations

import numpy as np

import oracle

OPTS = ("sh", "fm", "sfm", "pfm")
U64MAX = 2**64 - 1


def oracle_pairs(og, opt, S, Z, t0=0, t1=2**31 - 1, mode=None, edges=True):
    """Per-pair oracle records, f(v) rows and f(e) rows (input edge order)."""
    recs, nf, ef = [], [], []
    for s, z in zip(S, Z):
        md = mode if mode is not None else (0 if og.m <= 20_000 else 1)
        rec, nN, eN = oracle.pair(og, opt, int(s), int(z), t0, t1, mode=md, edges=edges)
        recs.append(rec)
        ok = rec["reachable"] and not (rec["flags"] & oracle.REC_OVERFLOW)
        sg = float(rec["sigma"]) if ok else 1.0
        nf.append(nN.astype(np.float64) / sg if ok else np.zeros(og.n))
        if edges:
            ef.append(eN.astype(np.float64) / sg if ok else np.zeros(og.m))
    return recs, np.array(nf), (np.array(ef) if edges else None)


def compare_pairs(gg, og, opt, S, Z, t0=0, t1=2**31 - 1, edges=True, mode=None, ctx=""):
    """Bit-exact comparison of records and per-pair f between GPU and oracle."""
    S = np.asarray(S, dtype=np.int32)
    Z = np.asarray(Z, dtype=np.int32)
    rec, nf, ef = gg.count_pairs(opt, S, Z, t0, t1, node_f=True, edge_f=edges)
    orecs, onf, oef = oracle_pairs(og, opt, S, Z, t0, t1, mode=mode, edges=edges)
    for q, want in enumerate(orecs):
        got = {k: int(rec[k][q]) for k in ("reachable", "t_arr", "hops", "flags", "sigma")}
        assert got["flags"] & 2 == 0, ("flow conservation", ctx, opt, S[q], Z[q])
        if want["flags"] & oracle.REC_OVERFLOW:
            # beyond the 64-bit oracle: the library counted the pair in wider
            # words (its exact checks are in test_gpu_wide); the record agrees
            assert (got["reachable"], got["t_arr"], got["hops"]) == (
                want["reachable"], want["t_arr"], want["hops"]), (ctx, opt, int(S[q]), int(Z[q]), got, want)
            assert got["sigma"] == want["sigma"] or got["flags"] & 16, (ctx, opt, got, want)
            nf[q] = onf[q]
            if edges:
                ef[q] = oef[q]
            continue
        assert (got["reachable"], got["t_arr"], got["hops"], got["sigma"], got["flags"] & 1) == (
            want["reachable"], want["t_arr"], want["hops"], want["sigma"], 0), (
            ctx, opt, int(S[q]), int(Z[q]), got, want)
    # f(v|s,z) and f(e|s,z): the same IEEE division of the same exact integers
    bad = np.nonzero(nf != onf)
    assert bad[0].size == 0, (ctx, opt, "node f differs", [(int(S[i]), int(Z[i]), int(v), nf[i, v], onf[i, v])
                                                           for i, v in zip(*bad)][:5])
    if edges:
        bad = np.nonzero(ef != oef)
        assert bad[0].size == 0, (ctx, opt, "edge f differs", [(int(S[i]), int(Z[i]), int(e), ef[i, e], oef[i, e])
                                                               for i, e in zip(*bad)][:5])
    return rec


def rel_close(a, b, rel=1e-12, abs_floor=0.0):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    tol = rel * np.maximum(np.abs(a), np.abs(b)) + abs_floor
    return np.all(np.abs(a - b) <= tol), float(np.max(np.abs(a - b) - tol)) if a.size else 0.0
