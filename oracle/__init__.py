"""The oracle -- TEST INFRASTRUCTURE ONLY.

A plain, slow CPU statement of MANTRA's hot path (per-pair temporal path
counting, dependency accumulation, the MCERA bound and the progressive
sampling loop), written from the paper.  Only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import it;
the product package never does, and the two share no code.

Parity status per function (the tests that pin each one are named there):

* ``pair`` / ``accumulate`` (oracle.c): pinned by brute-force walk
  enumeration, the hand-worked example of the appendix figure, layered-DAG
  reductions to static Brandes counts, closed forms on lines and single-tick
  graphs, and the exact integer invariants of Lemma 1 and Lemma 6.
* ``draw_pairs`` / ``word``: pinned to published SplitMix64 outputs and to
  uniformity of the pair distribution.
* ``mantra.round_stats`` and the f, f^2 and lambda f sums of
  ``accumulate``: pinned by the same statistics computed from brute-force
  walk enumeration in exact fractions, and by the closed forms of all-plus
  and all-minus sign words and of the time-increasing line.
* ``bounds``: Theorem 3's size with rho = v is Bernstein's sample size for
  one function (pinned); the closed forms of Theorem 1 and Hoeffding's bound
  are checked by limit and monotonicity properties and by the statistical
  guarantee (SD <= xi in at least a 1 - delta fraction of runs).  "Parity
  unpinned": the constants of Theorem 1's Eqs. (1)-(3) and Theorem 3's
  ln(2 rho / v) factor beyond rho = v (no independent source for them
  exists).
* ``mantra.estimate`` (Algorithm 1): pinned through its parts and by the
  statistical guarantee of Theorem 5; fm has no guarantee ("parity unpinned"
  beyond its counts).
* ``distances`` (Algorithm 2): per-source distances pinned by brute force,
  the closing formulas by closed forms and the all-sources definitions.
* ``trk`` (the TRK estimator's path sampler): pinned by brute-force optimal
  walks, the 1/sigma distribution of the drawn walks and unbiasedness.
* ``rtb`` (the RTB estimator): pinned by brute force, the line's closed form
  and the mean over all sources.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_build", "liboracle.so")

OPT = {"sh": 0, "fm": 1, "sfm": 2, "pfm": 3}
OPT_NAMES = {v: k for k, v in OPT.items()}
REC_OVERFLOW = 1
REC_SELFCHECK = 2
STREAM_PAIR = 0
STREAM_BOOT = 1
STREAM_RADE = 2
T_MAX = 2**31 - 1


class Record(ctypes.Structure):
    _fields_ = [("reachable", ctypes.c_int32), ("t_arr", ctypes.c_int32),
                ("hops", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("sigma", ctypes.c_uint64)]


REC_DTYPE = np.dtype([("reachable", np.int32), ("t_arr", np.int32), ("hops", np.int32),
                      ("flags", np.int32), ("sigma", np.uint64)])

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.orc_graph_new.restype = P
        L.orc_graph_new.argtypes = [ctypes.c_int32, ctypes.c_int64, P, P, P]
        L.orc_graph_free.argtypes = [P]
        L.orc_pair.restype = ctypes.c_int
        L.orc_pair.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                               ctypes.c_int32, ctypes.c_int32, P, P, P]
        L.orc_accumulate.restype = ctypes.c_int64
        L.orc_accumulate.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_int64, P, P, ctypes.c_int32, P,
                                     P, P, P, P, P, P, P, P, P, ctypes.c_int32]
        L.orc_word.restype = ctypes.c_uint64
        L.orc_word.argtypes = [ctypes.c_uint64] * 4
        L.orc_splitmix_nth.restype = ctypes.c_uint64
        L.orc_splitmix_nth.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.orc_draw_pairs.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32,
                                     ctypes.c_int64, ctypes.c_int64, P, P]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class Graph:
    """The oracle's copy of a temporal graph (edges sorted by time once)."""

    def __init__(self, n, src, dst, t):
        self.n = int(n)
        self.src = np.ascontiguousarray(src, dtype=np.int32)
        self.dst = np.ascontiguousarray(dst, dtype=np.int32)
        self.t = np.ascontiguousarray(t, dtype=np.int32)
        self.m = int(self.src.shape[0])
        self._h = lib().orc_graph_new(self.n, self.m, _p(self.src), _p(self.dst), _p(self.t))

    @classmethod
    def of(cls, g):
        return cls(g.n, g.src, g.dst, g.t)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_graph_free(self._h)
            self._h = None


def _opt(opt):
    return OPT[opt] if isinstance(opt, str) else int(opt)


def pair(g: Graph, opt, s: int, z: int, t0: int = 0, t1: int = T_MAX, mode: int = 0,
         nodes: bool = True, edges: bool = True):
    """Exact counts for one pair: (record dict, N(v) uint64[n], N(e) uint64[m])."""
    rec = Record()
    nN = np.zeros(g.n, dtype=np.uint64) if nodes else None
    eN = np.zeros(g.m, dtype=np.uint64) if edges else None
    rc = lib().orc_pair(g._h, _opt(opt), int(t0), int(t1), int(s), int(z), int(mode),
                        ctypes.byref(rec), _p(nN) if nodes else None, _p(eN) if edges else None)
    if rc != 0:
        raise ValueError("oracle: bad pair arguments")
    r = {"reachable": rec.reachable, "t_arr": rec.t_arr, "hops": rec.hops, "flags": rec.flags,
         "sigma": int(rec.sigma)}
    return r, nN, eN


def word(seed: int, stream: int, i: int, j: int) -> int:
    return int(lib().orc_word(seed, stream, i, j))


def splitmix_nth(x: int, k: int) -> int:
    return int(lib().orc_splitmix_nth(x, k))


def draw_pairs(seed: int, stream: int, n: int, i0: int, k: int):
    S = np.empty(k, dtype=np.int32)
    Z = np.empty(k, dtype=np.int32)
    lib().orc_draw_pairs(seed, stream, n, i0, k, _p(S), _p(Z))
    return S, Z


def rade_words(seed: int, i0: int, k: int) -> np.ndarray:
    return np.array([word(seed, STREAM_RADE, i0 + q, 0) for q in range(k)], dtype=np.uint64)


class Sums:
    """Double-double running sums of f, f^2, lambda f and f(e) (Algorithm 1's
    arrays B, W, the Rademacher sums, and the temporal-edge sums)."""

    def __init__(self, n, m, c, edges):
        self.n, self.m, self.c = n, m, c
        self.bhi = np.zeros(n); self.blo = np.zeros(n)
        self.whi = np.zeros(n); self.wlo = np.zeros(n)
        self.rhi = np.zeros(n * max(c, 1)); self.rlo = np.zeros(n * max(c, 1))
        self.edges = edges
        self.ehi = np.zeros(m) if edges else None
        self.elo = np.zeros(m) if edges else None
        self.r = 0
        self.n_overflow = 0

    @property
    def B(self):
        return self.bhi + self.blo

    @property
    def W(self):
        return self.whi + self.wlo

    @property
    def R(self):
        return (self.rhi + self.rlo).reshape(self.n, max(self.c, 1))[:, : self.c]

    @property
    def E(self):
        return None if self.ehi is None else self.ehi + self.elo


def accumulate(g: Graph, opt, S, Z, lam=None, c: int = 0, sums: Sums = None, t0: int = 0,
               t1: int = T_MAX, mode: int = 0, edges: bool = False, nthreads: int = 0):
    """Add the pairs (S[q], Z[q]) into ``sums`` (created if None); returns
    (sums, records)."""
    S = np.ascontiguousarray(S, dtype=np.int32)
    Z = np.ascontiguousarray(Z, dtype=np.int32)
    npairs = int(S.shape[0])
    if lam is None:
        lam = np.zeros(npairs, dtype=np.uint64)
    lam = np.ascontiguousarray(lam, dtype=np.uint64)
    if sums is None:
        sums = Sums(g.n, g.m, c, edges)
    recs = np.zeros(npairs, dtype=REC_DTYPE)
    nov = lib().orc_accumulate(
        g._h, _opt(opt), int(t0), int(t1), int(mode), npairs, _p(S), _p(Z), int(sums.c), _p(lam),
        _p(sums.bhi), _p(sums.blo), _p(sums.whi), _p(sums.wlo), _p(sums.rhi), _p(sums.rlo),
        _p(sums.ehi) if sums.edges else None, _p(sums.elo) if sums.edges else None,
        _p(recs), int(nthreads))
    sums.r += npairs
    sums.n_overflow += int(nov)
    return sums, recs
