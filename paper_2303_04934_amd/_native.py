"""ctypes declarations of the C ABI in include/hipscc.h (marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhipscc.so")

SCC_OK, SCC_EINVAL, SCC_EGRAPH, SCC_ENOMEM, SCC_ECAPACITY, SCC_EHIP, SCC_EPOLICY, SCC_EINTERNAL = 0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "SCC_OK", -1: "SCC_EINVAL", -2: "SCC_EGRAPH", -3: "SCC_ENOMEM", -4: "SCC_ECAPACITY",
                -5: "SCC_EHIP", -6: "SCC_EPOLICY", -7: "SCC_EINTERNAL"}

POLICY_FLOATS = 32 * 5 + 32 + 32 * 32 + 32 + 8 * 32 + 8


class Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32),
                ("out_off", ctypes.c_void_p), ("out_adj", ctypes.c_void_p),
                ("in_off", ctypes.c_void_p), ("in_adj", ctypes.c_void_p)]


# frontier kernels timed with options.timing (SCC_KERNEL_* in hipscc.h)
KERNEL_NAMES = ["k_expand<0, 1>", "k_expand<1, 1>", "k_pull", "k_expand_heavy<0>", "k_expand_heavy<1>", "k_bag_extract",
                "k_cc_union"]
KERNELS = len(KERNEL_NAMES)


class Options(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_int32), ("beta", ctypes.c_float), ("lambda_log2", ctypes.c_int32),
                ("sigma", ctypes.c_int32), ("kappa", ctypes.c_int32), ("alpha", ctypes.c_float),
                ("seed", ctypes.c_uint64), ("policy", ctypes.c_int32), ("dense", ctypes.c_int32),
                ("validate", ctypes.c_int32), ("trim", ctypes.c_int32), ("table_init", ctypes.c_int64),
                ("seeds_per_wave", ctypes.c_int32), ("timing", ctypes.c_int32), ("trace", ctypes.c_int32),
                ("arcs_per_lane", ctypes.c_int32), ("vgc_fill", ctypes.c_float),
                ("beta_fast", ctypes.c_float), ("table_floor", ctypes.c_float), ("union_arcs_max", ctypes.c_int32),
                ("first_slot", ctypes.c_int32), ("vgc_measure", ctypes.c_int32), ("ldd_beta", ctypes.c_float),
                ("graph_rounds", ctypes.c_int32), ("packed", ctypes.c_int32),
                ("union_streams", ctypes.c_int32), ("tau_single", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_double) for f in ("ms_total", "ms_trim", "ms_first", "ms_multi", "ms_resize",
                                                "ms_label")] + \
               [(f, ctypes.c_int64) for f in ("n", "m", "batches", "rounds_first", "rounds_multi", "dense_rounds",
                                               "entries_expanded", "arcs_scanned", "claim_attempts", "claims", "claims_table",
                                               "bag_inserts", "bag_chunk_advances", "table_restarts", "restart_rounds", "trimmed",
                                               "n_scc", "policy_calls", "policy_fallbacks", "bytes_alg")] + \
               [("ms_kernel", ctypes.c_double * KERNELS), ("launches_kernel", ctypes.c_int64 * KERNELS),
                ("bytes_kernel", ctypes.c_int64 * KERNELS)]

    def as_dict(self):
        d = {}
        for f, _ in self._fields_:
            v = getattr(self, f)
            d[f] = list(v) if hasattr(v, "__len__") else v
        return d


EXPORTS = ["scc_version", "scc_default_options", "scc_create", "scc_destroy", "scc_last_error", "scc_labels",
           "scc_reach", "scc_labels_batched", "scc_policy_load", "scc_policy_eval", "scc_bag_selftest",
           "scc_trace_read", "scc_bag_stats", "scc_labels_static", "scc_cc", "scc_le_lists"]
TRACE_FIELDS = 12

_lib = None


def load():
    """Load libhipscc.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libhipscc.so is not built: run paper_2303_04934_amd/build.py (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    P = ctypes.POINTER
    lib.scc_version.restype = ctypes.c_char_p
    lib.scc_default_options.argtypes = [P(Options)]
    lib.scc_create.argtypes = [P(vp), ctypes.c_int, vp]
    lib.scc_destroy.argtypes = [vp]
    lib.scc_destroy.restype = None
    lib.scc_last_error.argtypes = [vp]
    lib.scc_last_error.restype = ctypes.c_char_p
    lib.scc_labels.argtypes = [vp, P(Graph), vp, P(Options), P(Stats)]
    lib.scc_labels_static.argtypes = [vp, P(Graph), vp, P(Options), P(Stats)]
    lib.scc_cc.argtypes = [vp, P(Graph), vp, P(Options), P(Stats)]
    lib.scc_le_lists.argtypes = [vp, P(Graph), vp, vp, vp, vp, i64, P(i64), P(Options), P(Stats)]
    lib.scc_reach.argtypes = [vp, P(Graph), i32, vp, i32, vp, vp, i64, P(i64), P(Options), P(Stats)]
    lib.scc_labels_batched.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, P(Options), P(Stats)]
    lib.scc_policy_load.argtypes = [vp, vp, i64]
    lib.scc_policy_eval.argtypes = [vp, vp, i32, vp]
    lib.scc_bag_selftest.argtypes = [vp, vp, i64, i32, vp, P(i64), P(Options), P(Stats)]
    lib.scc_trace_read.argtypes = [vp, vp, i64, P(i64)]
    lib.scc_bag_stats.argtypes = [vp, vp, i64, P(i64), vp, i64, P(i64)]
    for name in EXPORTS:
        if name not in ("scc_version", "scc_destroy", "scc_last_error"):
            getattr(lib, name).restype = ctypes.c_int32
    _lib = lib
    return lib
