"""ctypes declarations for libcfc.so (mirror of include/cfc.h).

Loading fails loudly when the library has not been built: there is no other
implementation of these calls.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# CFC_LIB_PATH selects another build of the same sources (the sanitized
# host build that tests/test_host_sanitized.py runs)
LIB_PATH = os.environ.get("CFC_LIB_PATH") or os.path.join(HERE, "libcfc.so")

CFC_OK = 0
ERRORS = {
    -1: "CFC_E_INVALID", -2: "CFC_E_DISCONNECTED", -3: "CFC_E_NOMEM", -4: "CFC_E_DEVICE",
    -5: "CFC_E_NOT_CONVERGED", -6: "CFC_E_STATE", -7: "CFC_E_BUSY", -8: "CFC_E_CANCELLED",
    -9: "CFC_E_INTERNAL",
}
COL_OK, COL_NOT_CONVERGED, COL_DIVERGED, COL_SKIPPED = 0, 1, 2, 3
LCC_ONLY, REJECT_PARALLEL = 1, 2
PREC_MIXED, PREC_FP64 = 0, 1
MAX_LEVELS = 32
ELIM_MAX_DEGREE = 4  # neighbour slots of an eliminated row (CFC_ELIM_MAX_DEGREE)
QUERY_SAMPLING, QUERY_JL = 0, 1

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class CtxOpts(C.Structure):
    _fields_ = [("device", C.c_int32), ("stream", C.c_void_p), ("alloc", ALLOC_FN),
                ("free", FREE_FN), ("user", C.c_void_p), ("hbm_budget", C.c_uint64)]


class GraphInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("m", C.c_int64), ("input_n", C.c_int64), ("levels", C.c_int32),
                ("unit_weights", C.c_int32), ("level_n", C.c_int64 * MAX_LEVELS),
                ("level_nnz", C.c_int64 * MAX_LEVELS), ("operator_complexity", C.c_double),
                ("setup_ms", C.c_double), ("device_bytes", C.c_uint64), ("max_degree", C.c_int32),
                ("eliminated", C.c_int32), ("cycle_complexity", C.c_double)]


class SetupParams(C.Structure):
    _fields_ = [("coarsest_max", C.c_int32), ("agg_cap", C.c_int32), ("test_vectors", C.c_int32),
                ("relax_sweeps", C.c_int32), ("omega", C.c_double), ("mu", C.c_double),
                ("seed", C.c_uint64), ("eliminate", C.c_int32), ("device", C.c_int32),
                ("order", C.c_int32), ("max_complexity_pct", C.c_int32),
                ("elim_degree", C.c_int32), ("nest", C.c_int32)]


class SolveParams(C.Structure):
    _fields_ = [("tol", C.c_double), ("precision", C.c_int32), ("block", C.c_int32),
                ("max_refine", C.c_int32), ("max_inner", C.c_int32), ("inner_tol", C.c_double),
                ("use_graph", C.c_int32), ("check_every", C.c_int32), ("levels", C.c_int32),
                ("pad", C.c_int32)]


class SolveStats(C.Structure):
    _fields_ = [("columns", C.c_int64), ("converged", C.c_int64), ("inner_iters", C.c_int64),
                ("refine_steps", C.c_int64), ("blocks", C.c_int64), ("block_width", C.c_int32),
                ("precision", C.c_int32), ("levels_used", C.c_int32), ("z_format", C.c_int32),
                ("max_rel_residual", C.c_double), ("solve_ms", C.c_double),
                ("model_bytes", C.c_double), ("kernel_ms", C.c_double * 3),
                ("kernel_bytes", C.c_double * 3), ("kernel_launches", C.c_int64 * 3)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        for f in ("kernel_ms", "kernel_bytes", "kernel_launches"):
            d[f] = list(d[f])
        return d


class LevelView(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("n_coarse", C.c_int64),
                ("row_ptr", C.POINTER(C.c_int32)), ("col", C.POINTER(C.c_int32)),
                ("w", C.POINTER(C.c_double)), ("deg", C.POINTER(C.c_double)),
                ("agg", C.POINTER(C.c_int32)), ("agg_ptr", C.POINTER(C.c_int32)),
                ("perm", C.POINTER(C.c_int32)), ("coarse_pinv", C.POINTER(C.c_double)),
                ("elimination", C.c_int32), ("pad", C.c_int32), ("elim_nb", C.POINTER(C.c_int32))]


class ServerOpts(C.Structure):
    _fields_ = [("slots", C.c_int32), ("max_queue", C.c_int32), ("jl_k", C.c_int32),
                ("sampling_k", C.c_int32), ("seed", C.c_uint64), ("tol", C.c_double),
                ("hbm_budget", C.c_uint64)]


class Query(C.Structure):
    _fields_ = [("graph", C.c_int32), ("kind", C.c_int32), ("nnodes", C.c_int32), ("k", C.c_int32),
                ("nodes", C.POINTER(C.c_int64)), ("seed", C.c_uint64)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("nnodes", C.c_int32), ("far", C.POINTER(C.c_double)),
                ("clo", C.POINTER(C.c_double)), ("latency_ms", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("queued", C.c_int64),
                ("in_flight", C.c_int64), ("p50_ms", C.c_double), ("p99_ms", C.c_double),
                ("mean_ms", C.c_double), ("queries_per_s", C.c_double), ("device_bytes", C.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


vp = C.c_void_p
i64p = C.POINTER(C.c_int64)
f64p = C.POINTER(C.c_double)
i32p = C.POINTER(C.c_int32)

# name -> (restype, argtypes): every entry point of include/cfc.h
SIGNATURES = {
    "cfc_ctx_create": (C.c_int, [C.POINTER(CtxOpts), C.POINTER(vp)]),
    "cfc_ctx_destroy": (None, [vp]),
    "cfc_last_error": (C.c_char_p, []),
    "cfc_version": (C.c_char_p, []),
    "cfc_graph_load": (C.c_int, [vp, C.c_int64, C.c_int64, i64p, i64p, f64p, C.c_uint32, C.POINTER(vp)]),
    "cfc_graph_get_info": (C.c_int, [vp, C.POINTER(GraphInfo)]),
    "cfc_graph_node_map": (C.c_int, [vp, i64p]),
    "cfc_graph_destroy": (None, [vp]),
    "cfc_hierarchy_build": (C.c_int, [vp, C.POINTER(SetupParams)]),
    "cfc_hierarchy_level": (C.c_int, [vp, C.c_int32, C.POINTER(LevelView)]),
    "cfc_solve": (C.c_int, [vp, C.c_int64, vp, vp, C.POINTER(SolveParams), C.POINTER(SolveStats), i32p]),
    "cfc_resistance": (C.c_int, [vp, C.c_int64, i64p, i64p, f64p, C.POINTER(SolveParams), C.POINTER(SolveStats)]),
    "cfc_farness_exact": (C.c_int, [vp, C.c_int64, i64p, f64p, f64p, C.POINTER(SolveParams), C.POINTER(SolveStats)]),
    "cfc_farness_sampling": (C.c_int, [vp, C.c_int64, i64p, C.c_int64, C.c_uint64, f64p, f64p,
                                       C.POINTER(SolveParams), C.POINTER(SolveStats)]),
    "cfc_jl_sketch": (C.c_int, [vp, C.c_int64, C.c_uint64, C.POINTER(SolveParams), C.POINTER(SolveStats)]),
    "cfc_farness_jl": (C.c_int, [vp, C.c_int64, i64p, f64p, f64p]),
    "cfc_device_copy": (C.c_int, [vp, vp, vp, C.c_size_t]),
    "cfc_farness_jl_static": (C.c_int, [vp, C.c_int64, vp, vp, vp]),
    "cfc_sampling_pivots": (C.c_int, [C.c_uint64, C.c_int64, C.c_int64, C.c_int64, i64p]),
    "cfc_jl_sign_word": (C.c_uint64, [C.c_uint64, C.c_uint64, C.c_int64, C.c_int64]),
    "cfc_farness_sampling_shared": (C.c_int, [vp, C.c_int64, i64p, C.c_int64, C.c_uint64, f64p, f64p,
                                              C.POINTER(SolveParams), C.POINTER(SolveStats)]),
    "cfc_spanning_edge": (C.c_int, [vp, C.c_int64, i64p, i64p, f64p, C.POINTER(SolveParams),
                                    C.POINTER(SolveStats)]),
    "cfc_spanning_edge_jl": (C.c_int, [vp, C.c_int64, i64p, i64p, C.c_int64, C.c_uint64, f64p,
                                       C.POINTER(SolveParams), C.POINTER(SolveStats)]),
    "cfc_current_throughput": (C.c_int, [vp, C.c_int64, i64p, i64p, f64p, C.POINTER(SolveParams),
                                         C.POINTER(SolveStats)]),
    "cfc_cfb_exact": (C.c_int, [vp, f64p, C.POINTER(SolveParams), C.POINTER(SolveStats)]),
    "cfc_cfb_sampled": (C.c_int, [vp, C.c_int64, C.c_uint64, f64p, C.POINTER(SolveParams),
                                  C.POINTER(SolveStats)]),
    "cfc_shared_pivots": (C.c_int, [C.c_uint64, C.c_int64, C.c_int64, i64p]),
    "cfc_random_pairs": (C.c_int, [C.c_uint64, C.c_int64, C.c_int64, i64p, i64p]),
    "cfc_server_create": (C.c_int, [vp, C.POINTER(ServerOpts), C.POINTER(vp)]),
    "cfc_server_add_graph": (C.c_int, [vp, vp, i32p]),
    "cfc_server_submit": (C.c_int, [vp, C.POINTER(Query), C.POINTER(C.c_uint64)]),
    "cfc_server_poll": (C.c_int, [vp, C.c_uint64, C.POINTER(Result)]),
    "cfc_server_wait": (C.c_int, [vp, C.c_uint64, C.c_double, C.POINTER(Result)]),
    "cfc_server_get_stats": (C.c_int, [vp, C.POINTER(ServerStats)]),
    "cfc_server_destroy": (None, [vp]),
}

_lib = None


def lib():
    """The loaded libcfc (raises if it is missing or incomplete)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libcfc.so not built at {LIB_PATH}; run python -m paper_1607_02955_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)  # AttributeError if a symbol is missing
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class CfcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def check(code):
    if code != CFC_OK:
        raise CfcError(code, lib().cfc_last_error().decode(errors="replace"))
    return code
