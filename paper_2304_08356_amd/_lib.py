"""ctypes declarations of the C ABI in include/mantra.h (marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmantra.so")

P = ctypes.c_void_p
I32 = ctypes.c_int32
I64 = ctypes.c_int64
U32 = ctypes.c_uint32
U64 = ctypes.c_uint64
F64 = ctypes.c_double

SH, FM, SFM, PFM = 0, 1, 2, 3
OPT = {"sh": SH, "fm": FM, "sfm": SFM, "pfm": PFM}

OK, PENDING = 0, 1
E_INVALID = -1
STATUS = {0: "OK", 1: "PENDING", -1: "E_INVALID", -2: "E_NODEV", -3: "E_OOM", -4: "E_OVERFLOW",
          -5: "E_TOO_LARGE", -6: "E_INTERNAL", -7: "E_LIMIT"}

REC_OVERFLOW = 1
REC_HOPS_LIMIT = 4
F_EDGE_BC = 1
F_TRK = 2
F_RTB = 4
RES_NO_GUARANTEE = 1
RES_STOP_XI = 2
RES_STOP_OMEGA = 4


class PairRecord(ctypes.Structure):
    _fields_ = [("reachable", I32), ("t_arr", I32), ("hops", I32), ("flags", I32), ("sigma", U64)]


class Request(ctypes.Structure):
    _fields_ = [("opt", I32), ("t0", I32), ("t1", I32), ("eps", F64), ("delta", F64), ("seed", U64),
                ("c", I32), ("s1", I64), ("max_samples", I64), ("fixed_r", I64), ("flags", U32),
                ("node_bc", P), ("edge_bc", P)]


class LaunchConfig(ctypes.Structure):
    _fields_ = [("n_slabs", I32), ("arc_cap", I64), ("order", I32), ("graph_rounds", I32), ("per_pair_launch", I32),
                ("hub_nodes", I32), ("wide_counts", I32), ("no_arc_chunks", I32), ("arc_chunks", I64)]

    def to_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


ORDER = {"longest": 0, "drawn": 1}


class Result(ctypes.Structure):
    _fields_ = [("node_bc", P), ("edge_bc", P), ("status", I32), ("flags", U32), ("samples", I64), ("rounds", I64), ("omega", I64),
                ("s_boot", I64), ("s1", I64), ("n_overflow", I64), ("n_reachable", I64),
                ("window_edges", I64), ("arcs", I64), ("xi", F64), ("rho_hat", F64), ("v_hat", F64),
                ("wimpy", F64), ("mcera", F64), ("gpu_ms", F64), ("latency_ms", F64)]

    def to_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k not in ("node_bc", "edge_bc")}


class DistanceResult(ctypes.Structure):
    _fields_ = [("sources", I64), ("reached_pairs", I64), ("d_lb", I32), ("d_tau", I32), ("zeta", F64),
                ("psi", F64), ("rho", F64), ("window_edges", I64), ("gpu_ms", F64)]

    def to_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# every symbol include/mantra.h declares, with (restype, argtypes)
SIGNATURES = {
    "mantra_graph_create": (I32, [P, P, P, I64, I32, U32, P]),
    "mantra_graph_create_packed": (I32, [I32, P, P, P, P, P, U32, P]),
    "mantra_graph_destroy": (None, [P]),
    "mantra_graph_info": (I32, [P, P, P, P, P, P, P]),
    "mantra_count_pairs": (I32, [P, I32, I32, I32, I64, P, P, P, P, P, P]),
    "mantra_count_pairs_static": (I32, [P, I32, I32, I32, I64, P, P, P, P]),
    "mantra_sample_paths": (I32, [P, I32, I32, I32, I64, P, P, P, U64, P, P, P]),
    "mantra_source_dependencies": (I32, [P, I32, I32, I32, I64, P, P, P, P, P]),
    "mantra_estimate": (I32, [P, I32, F64, F64, U64, P]),
    "mantra_run": (I32, [P, P, P]),
    "mantra_distances": (I32, [P, I32, I32, I32, I64, U64, F64, P, I32, P]),
    "mantra_submit": (I32, [P, P, P]),
    "mantra_poll": (I32, [U64, P, I32]),
    "mantra_serve_config": (I32, [P, U64, I32]),
    "mantra_set_launch": (I32, [P, P]),
    "mantra_get_launch": (I32, [P, P]),
    "mantra_autotune": (I32, [P, I32, I64, U64, P]),
    "mantra_last_timing": (I32, [P, P, P, P, P, P, P, P, P, P, P]),
    "mantra_debug_stamps": (I32, [P, U32]),
    "mantra_last_error": (ctypes.c_char_p, []),
}

_lib = None


class MantraError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


def load(path: str = LIB_PATH):
    """Load the HIP library.  There is no fallback: a missing or broken
    library is an error."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libmantra.so is not built (python -m paper_2304_08356_amd.build): " + path)
    L = ctypes.CDLL(path)
    for name, (rt, at) in SIGNATURES.items():
        f = getattr(L, name)
        f.restype = rt
        f.argtypes = at
    _lib = L
    return L


def check(code):
    if code < 0:
        msg = _lib.mantra_last_error().decode(errors="replace") if _lib else ""
        raise MantraError(code, msg)
    return code
