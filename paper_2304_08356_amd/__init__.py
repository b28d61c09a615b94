"""MI355X-native temporal betweenness estimation (MANTRA hot path).

A thin Python binding over the C ABI of ``libmantra.so`` (include/mantra.h):
every computation runs in the library's HIP kernels; this module only
marshals numpy arrays and results.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import (OPT, F_EDGE_BC, F_RTB, F_TRK, MantraError, PairRecord, Request, Result,  # noqa: F401
                   REC_OVERFLOW, REC_HOPS_LIMIT, RES_NO_GUARANTEE, RES_STOP_OMEGA, RES_STOP_XI)

REC_DTYPE = np.dtype([("reachable", np.int32), ("t_arr", np.int32), ("hops", np.int32),
                      ("flags", np.int32), ("sigma", np.uint64)])
T_MAX = 2**31 - 1


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _opt(o):
    return OPT[o] if isinstance(o, str) else int(o)


class Graph:
    """A device-resident temporal graph (mantra_graph)."""

    def __init__(self, n, src, dst, t, _packed=None):
        L = _lib.load()
        self._h = ctypes.c_void_p()
        if _packed is None:
            src = np.ascontiguousarray(src, dtype=np.int32)
            dst = np.ascontiguousarray(dst, dtype=np.int32)
            t = np.ascontiguousarray(t, dtype=np.int32)
            _lib.check(L.mantra_graph_create(_p(src), _p(dst), _p(t), int(src.shape[0]), int(n), 0,
                                             ctypes.byref(self._h)))
            self.m_input = int(src.shape[0])
        else:
            nc, eo = _packed
            _lib.check(L.mantra_graph_create_packed(int(nc.shape[0]), _p(nc), _p(eo), _p(src), _p(dst),
                                                    _p(t), 0, ctypes.byref(self._h)))
            self.m_input = int(src.shape[0])
        info = self.info()
        self.n = info["n"]
        self.m = info["m_unique"]
        self.n_graphs = info["n_graphs"]

    @classmethod
    def of(cls, g):
        return cls(g.n, g.src, g.dst, g.t)

    @classmethod
    def packed(cls, graphs):
        """One device graph holding independent graphs (local node ids)."""
        nc = np.array([g.n for g in graphs], dtype=np.int32)
        eo = np.zeros(len(graphs) + 1, dtype=np.int64)
        eo[1:] = np.cumsum([g.m for g in graphs])
        src = np.ascontiguousarray(np.concatenate([g.src for g in graphs]), dtype=np.int32)
        dst = np.ascontiguousarray(np.concatenate([g.dst for g in graphs]), dtype=np.int32)
        t = np.ascontiguousarray(np.concatenate([g.t for g in graphs]), dtype=np.int32)
        obj = cls(None, src, dst, t, _packed=(nc, eo))
        obj.node_counts = nc
        obj.edge_offsets = eo
        return obj

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib._lib.mantra_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        n = ctypes.c_int32(); mu = ctypes.c_int64(); nd = ctypes.c_int64()
        t0 = ctypes.c_int32(); t1 = ctypes.c_int32(); G = ctypes.c_int32()
        _lib.check(_lib._lib.mantra_graph_info(self._h, ctypes.byref(n), ctypes.byref(mu), ctypes.byref(nd),
                                               ctypes.byref(t0), ctypes.byref(t1), ctypes.byref(G)))
        return {"n": n.value, "m_unique": mu.value, "n_duplicates": nd.value, "t_min": t0.value,
                "t_max": t1.value, "n_graphs": G.value}

    def set_launch(self, n_slabs=0, arc_cap=0, order="longest", graph_rounds=False, per_pair_launch=False,
                   hub_nodes=0, wide_counts=1, no_arc_chunks=False, arc_chunks=0):
        """Launch configuration: scheduling (results do not change), and which
        saturated pairs are counted again in 256-bit words (wide_counts: 0
        none, 1 all but fm, 2 all)."""
        cfg = _lib.LaunchConfig(n_slabs=int(n_slabs), arc_cap=int(arc_cap),
                                order=_lib.ORDER[order] if isinstance(order, str) else int(order),
                                graph_rounds=1 if graph_rounds else 0,
                                per_pair_launch=1 if per_pair_launch else 0, hub_nodes=int(hub_nodes),
                                wide_counts=int(wide_counts), no_arc_chunks=1 if no_arc_chunks else 0,
                                arc_chunks=int(arc_chunks))
        _lib.check(_lib._lib.mantra_set_launch(self._h, ctypes.byref(cfg)))

    def autotune(self, opt, sample_pairs=0, seed=0):
        """Pick the launch configuration by timing candidates on a
        calibration sample; returns the configuration kept."""
        cfg = _lib.LaunchConfig()
        _lib.check(_lib._lib.mantra_autotune(self._h, _opt(opt), int(sample_pairs), int(seed), ctypes.byref(cfg)))
        return cfg.to_dict()

    def get_launch(self):
        cfg = _lib.LaunchConfig()
        _lib.check(_lib._lib.mantra_get_launch(self._h, ctypes.byref(cfg)))
        return cfg.to_dict()

    def last_timing(self):
        ms = ctypes.c_double(); nl = ctypes.c_int64(); w = ctypes.c_int64(); a = ctypes.c_int64()
        tn = ctypes.c_int64(); te = ctypes.c_int64(); bal = ctypes.c_double()
        lv = ctypes.c_int64(); sk = ctypes.c_int64(); fs = ctypes.c_double()
        _lib.check(_lib._lib.mantra_last_timing(self._h, ctypes.byref(ms), ctypes.byref(nl), ctypes.byref(w),
                                                ctypes.byref(a), ctypes.byref(tn), ctypes.byref(te),
                                                ctypes.byref(bal), ctypes.byref(lv), ctypes.byref(sk),
                                                ctypes.byref(fs)))
        return {"sweep_ms": ms.value, "launches": nl.value, "window_edges": w.value, "arcs": a.value,
                "touched_nodes": tn.value, "touched_edges": te.value, "balance": bal.value,
                "live_batches": lv.value, "skipped_batches": sk.value, "forward_share": fs.value}

    def count_pairs(self, opt, s, z, t0=0, t1=T_MAX, graph=None, node_f=False, edge_f=False):
        """Records (and optionally dense per-pair f over nodes / input edges)
        for explicit pairs."""
        s = np.ascontiguousarray(s, dtype=np.int32)
        z = np.ascontiguousarray(z, dtype=np.int32)
        r = int(s.shape[0])
        g = None if graph is None else np.ascontiguousarray(graph, dtype=np.int32)
        rec = np.zeros(r, dtype=REC_DTYPE)
        nf = np.zeros((r, self.n), dtype=np.float64) if node_f else None
        ef = np.zeros((r, self.m_input), dtype=np.float64) if edge_f else None
        _lib.check(_lib._lib.mantra_count_pairs(self._h, _opt(opt), int(t0), int(t1), r, _p(g), _p(s), _p(z),
                                                _p(rec), _p(nf), _p(ef)))
        return rec, nf, ef

    def sample_paths(self, opt, s, z, seed=0, t0=0, t1=T_MAX, graph=None, node_f=True, edge_f=True):
        """The TRK estimator's walk of each explicit pair: records, and per
        pair the walk's internal visits per node and uses per input edge."""
        s = np.ascontiguousarray(s, dtype=np.int32)
        z = np.ascontiguousarray(z, dtype=np.int32)
        r = int(s.shape[0])
        g = None if graph is None else np.ascontiguousarray(graph, dtype=np.int32)
        rec = np.zeros(r, dtype=REC_DTYPE)
        nf = np.zeros((r, self.n), dtype=np.float64) if node_f else None
        ef = np.zeros((r, self.m_input), dtype=np.float64) if edge_f else None
        _lib.check(_lib._lib.mantra_sample_paths(self._h, _opt(opt), int(t0), int(t1), r, _p(g), _p(s), _p(z),
                                                 int(seed), _p(rec), _p(nf), _p(ef)))
        return rec, nf, ef

    def source_dependencies(self, opt, s, t0=0, t1=T_MAX, graph=None, node_f=True, edge_f=True):
        """The RTB estimator's f of explicit sources: records, and per source
        f(v|s) per node and f(e|s) per input edge."""
        s = np.ascontiguousarray(s, dtype=np.int32)
        r = int(s.shape[0])
        g = None if graph is None else np.ascontiguousarray(graph, dtype=np.int32)
        rec = np.zeros(r, dtype=REC_DTYPE)
        nf = np.zeros((r, self.n), dtype=np.float64) if node_f else None
        ef = np.zeros((r, self.m_input), dtype=np.float64) if edge_f else None
        _lib.check(_lib._lib.mantra_source_dependencies(self._h, _opt(opt), int(t0), int(t1), r, _p(g), _p(s),
                                                        _p(rec), _p(nf), _p(ef)))
        return rec, nf, ef

    @staticmethod
    def _out_array(a, size, what):
        if a is None:
            return np.zeros(size, dtype=np.float64)
        if not (isinstance(a, np.ndarray) and a.dtype == np.float64 and a.ndim == 1 and a.size == size
                and a.flags.c_contiguous and a.flags.writeable):
            raise ValueError("%s must be a writeable contiguous float64 array of %d values" % (what, size))
        return a

    def _request(self, opt, eps, delta, seed, c, t0, t1, s1, max_samples, fixed_r, edges, trk=False, rtb=False,
                 out=None):
        node_out, edge_out = out if out is not None else (None, None)
        node_bc = self._out_array(node_out, self.n, "node output")
        edge_bc = self._out_array(edge_out, self.m_input, "edge output") if edges else None
        flags = (F_EDGE_BC if edges else 0) | (F_TRK if trk else 0) | (F_RTB if rtb else 0)
        rq = Request(opt=_opt(opt), t0=int(t0), t1=int(t1), eps=float(eps), delta=float(delta),
                     seed=int(seed), c=int(c), s1=int(s1), max_samples=int(max_samples), fixed_r=int(fixed_r),
                     flags=flags, node_bc=_p(node_bc), edge_bc=_p(edge_bc))
        return rq, node_bc, edge_bc

    def run(self, opt, eps=0.01, delta=0.1, seed=0, c=25, t0=0, t1=T_MAX, s1=0, max_samples=0, fixed_r=0,
            edges=False, raise_on_error=True, trk=False, rtb=False, out=None):
        """Algorithm 1 (or a fixed sample of ``fixed_r`` pairs), with the ob
        estimator, the TRK estimator (trk=True) or the RTB estimator
        (rtb=True, samples are sources): returns (node_bc, edge_bc or None,
        result dict).  ``out = (node_array, edge_array or None)`` gives the
        float64 arrays the estimates are written to (reused across calls;
        a call that fails other than by overflow leaves them as they were);
        by default fresh ones are allocated."""
        rq, node_bc, edge_bc = self._request(opt, eps, delta, seed, c, t0, t1, s1, max_samples, fixed_r, edges,
                                             trk, rtb, out)
        res = Result()
        rc = _lib._lib.mantra_run(self._h, ctypes.byref(rq), ctypes.byref(res))
        if raise_on_error:
            _lib.check(rc)
        out = res.to_dict()
        out["rc"] = rc
        return node_bc, edge_bc, out

    def estimate(self, opt, eps, delta, seed, edges=False):
        """Algorithm 1 with the paper's defaults (whole span, c = 25): returns
        (node_bc, edge_bc or None, result dict)."""
        node_bc = np.zeros(self.n, dtype=np.float64)
        edge_bc = np.zeros(self.m_input, dtype=np.float64) if edges else None
        res = Result(node_bc=_p(node_bc), edge_bc=_p(edge_bc))
        _lib.check(_lib._lib.mantra_estimate(self._h, _opt(opt), float(eps), float(delta), int(seed),
                                             ctypes.byref(res)))
        return node_bc, edge_bc, res.to_dict()

    def distances(self, opt, r, seed=0, tau=0.9, t0=0, t1=T_MAX, hist_len=64):
        """Algorithm 2 from r sampled sources: returns (hist[hist_len] of
        sampled pairs per distance, the last bin taking larger ones; result
        dict with d_lb, d_tau, zeta, psi, rho)."""
        hist = np.zeros(max(int(hist_len), 0), dtype=np.uint64)
        res = _lib.DistanceResult()
        _lib.check(_lib._lib.mantra_distances(self._h, _opt(opt), int(t0), int(t1), int(r), int(seed), float(tau),
                                              _p(hist) if hist.size else None, int(hist.size), ctypes.byref(res)))
        return hist, res.to_dict()

    # serving
    def serve_config(self, mem_budget_bytes=0, max_active=0):
        _lib.check(_lib._lib.mantra_serve_config(self._h, int(mem_budget_bytes), int(max_active)))

    def submit(self, opt, eps=0.01, delta=0.1, seed=0, c=25, t0=0, t1=T_MAX, s1=0, max_samples=0, fixed_r=0,
               edges=False, trk=False, rtb=False):
        rq, node_bc, edge_bc = self._request(opt, eps, delta, seed, c, t0, t1, s1, max_samples, fixed_r, edges,
                                             trk, rtb)
        tk = ctypes.c_uint64()
        _lib.check(_lib._lib.mantra_submit(self._h, ctypes.byref(rq), ctypes.byref(tk)))
        return Ticket(tk.value, node_bc, edge_bc)


class Ticket:
    def __init__(self, tk, node_bc, edge_bc):
        self.id = tk
        self.node_bc = node_bc  # filled by the library when the ticket finishes
        self.edge_bc = edge_bc
        self.result = None

    def poll(self, timeout_ms=0):
        res = Result()
        rc = _lib._lib.mantra_poll(self.id, ctypes.byref(res), int(timeout_ms))
        if rc == _lib.PENDING:
            return None
        if rc != _lib.E_INVALID:  # the ticket finished (and is consumed)
            self.result = res.to_dict()
            self.result["rc"] = rc
        _lib.check(rc)
        return self.result


def symbols():
    """Names of the exported C entry points (for checks without a GPU)."""
    return sorted(_lib.SIGNATURES)
