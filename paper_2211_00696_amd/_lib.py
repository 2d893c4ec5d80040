"""ctypes declarations of libphiq.so (mirrors include/phiq.h)."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_size_t, c_void_p

MAX_DIM = 4
MAX_P = 24

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libphiq.so")

STATUS = {
    0: "PHIQ_OK",
    -1: "PHIQ_ERR_INVALID_ARG",
    -2: "PHIQ_ERR_NONFINITE",
    -3: "PHIQ_ERR_NOT_CONVERGED",
    -4: "PHIQ_ERR_OOM",
    -5: "PHIQ_ERR_HIP",
    -6: "PHIQ_ERR_UNSUPPORTED",
}
RULE = {"gauss": 1, "cc": 2}
PROFILE_CLASSES = ["ttm_store", "ttm_accum", "ttm_square", "gemm", "taylor", "scale", "node_sum", "absdiff", "slice",
                   "ttm_slab"]
PRECISION = {"fp64": 0, "fp32": 1, "bf16x3": 2, "int8": 3}
SELECTOR = {"paper": 0, "mlp": 1, "mlp-empirical": 2}
CC_SCALING = {"realized": 0, "paper": 1}

# Every symbol include/phiq.h declares.
EXPORTS = [
    "phiq_status_string",
    "phiq_options_default",
    "phiq_norm_bound",
    "phiq_setup_quadrature",
    "phiq_cc_scaling",
    "phiq_log_quaderr",
    "phiq_quadnodes",
    "phiq_quadrature_rule",
    "phiq_create",
    "phiq_destroy",
    "phiq_plan_create",
    "phiq_plan_execute",
    "phiq_plan_execute_combo",
    "phiq_plan_destroy",
    "phiq_plan_execute_noalloc",
    "phiq_action",
    "phiq_action_batched",
    "phiq_batch_info",
    "phiq_etdrk4",
    "phiq_exprk",
    "phiq_mlp_forward",
    "phiq_mlp_grad",
    "phiq_mlp_train",
    "phiq_selector_set",
    "phiq_selector_load",
    "phiq_expm",
    "phiq_kron_apply",
    "phiq_profile_start",
    "phiq_profile_stop",
    "phiq_profile_enable",
    "phiq_tile_config",
    "phiq_autotune",
]


class KronOp(ctypes.Structure):
    _fields_ = [("dim", c_int), ("n", c_int * MAX_DIM), ("A", POINTER(c_double) * MAX_DIM)]


class Options(ctypes.Structure):
    _fields_ = [
        ("rule", c_int),
        ("precision", c_int),
        ("l", c_int),
        ("m", c_int),
        ("alpha", c_double),
        ("c1", c_double),
        ("c2", c_double),
        ("cc_max_doublings", c_int),
        ("workspace_cap", c_size_t),
        ("use_graphs", c_int),
        ("selector", c_int),
        ("slab_products", c_int),
        ("accept_floor", c_int),
        ("selector_slack", c_double),
        ("batch_persistent", c_int),
        ("rhs_per_launch", c_int),
        ("cc_scaling", c_int),
    ]


class Report(ctypes.Structure):
    _fields_ = [
        ("l", c_int),
        ("m", c_int),
        ("cc_doublings", c_int),
        ("ttm_chains", c_int),
        ("alpha", c_double),
        ("log10_bound", c_double),
        ("cc_err", c_double),
        ("workspace_bytes", c_size_t),
        ("selector", c_int),
        ("precision_floor", c_double),
        ("tol_met", c_int),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Problem(ctypes.Structure):
    _fields_ = [("op", KronOp), ("t", c_double), ("p", c_int), ("tol", c_double), ("nrhs", c_int),
                ("v", c_void_p), ("out", c_void_p), ("rep", POINTER(Report))]


class BatchStats(ctypes.Structure):
    _fields_ = [("persistent", c_int), ("separate", c_int), ("stages", ctypes.c_longlong),
                ("tiles", ctypes.c_longlong), ("depth", c_int), ("launches", c_int), ("groups", c_int),
                ("arena_bytes", ctypes.c_size_t), ("upload_bytes", ctypes.c_size_t)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class EtdReport(ctypes.Structure):
    _fields_ = [("steps_eager", c_int), ("steps_graph", c_int), ("graph_nodes", c_int),
                ("ttm_chains_per_step", c_int), ("l_half", c_int), ("m_half", c_int),
                ("l_full", c_int), ("m_full", c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("launches", c_int), ("ms", c_double), ("flops", c_double),
                ("bytes", c_double)]


_lib = None


def load():
    """Load libphiq.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2211_00696_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P = POINTER
    sig = {
        "phiq_status_string": (c_char_p, [c_int]),
        "phiq_options_default": (c_int, [P(Options)]),
        "phiq_norm_bound": (c_int, [P(KronOp), c_double, P(c_double)]),
        "phiq_cc_scaling": (c_int, [c_double, c_int, c_double, c_double, c_double, c_int, c_int, POINTER(c_int)]),
        "phiq_setup_quadrature": (c_int, [c_double, c_int, c_double, c_double, c_int, c_double, c_double, c_int,
                                          P(c_int), P(c_int), P(c_double)]),
        "phiq_log_quaderr": (c_int, [c_double, c_int, c_double, c_double, c_int, P(c_double)]),
        "phiq_quadnodes": (c_int, [c_double, c_int, c_double, c_double, c_int, P(c_int)]),
        "phiq_quadrature_rule": (c_int, [c_int, c_int, P(c_double), P(c_double)]),
        "phiq_create": (c_int, [P(c_void_p), c_int]),
        "phiq_destroy": (c_int, [c_void_p]),
        "phiq_plan_create": (c_int, [c_void_p, P(KronOp), c_double, c_int, c_double, P(Options), P(c_void_p),
                                     P(Report), c_void_p]),
        "phiq_plan_execute": (c_int, [c_void_p, c_void_p, c_int, c_void_p, P(Report), c_void_p]),
        "phiq_plan_execute_combo": (c_int, [c_void_p, P(c_void_p), c_void_p, c_void_p]),
        "phiq_plan_destroy": (c_int, [c_void_p]),
        "phiq_plan_execute_noalloc": (c_int, [c_void_p, c_void_p, c_void_p, P(c_size_t), c_void_p]),
        "phiq_action": (c_int, [c_void_p, P(KronOp), c_double, c_int, c_void_p, c_double, P(Options), c_void_p,
                                P(Report), c_void_p]),
        "phiq_action_batched": (c_int, [c_void_p, c_int, P(Problem), P(Options), c_void_p]),
        "phiq_batch_info": (c_int, [c_int, P(Problem), P(Options), P(BatchStats)]),
        "phiq_etdrk4": (c_int, [c_void_p, P(KronOp), c_double, c_int, c_double, c_double, c_double, c_int,
                                c_int, c_void_p, P(EtdReport), c_void_p]),
        "phiq_exprk": (c_int, [c_void_p, P(KronOp), c_int, c_double, c_int, c_double, c_double, P(Options), c_int,
                               c_void_p, P(Report), c_void_p]),
        "phiq_mlp_forward": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p]),
        "phiq_mlp_grad": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p, P(c_double), c_void_p]),
        "phiq_mlp_train": (c_int, [c_void_p, c_int, P(ctypes.c_float), P(ctypes.c_float), P(ctypes.c_float), c_int,
                                   ctypes.c_float, P(ctypes.c_float)]),
        "phiq_selector_set": (c_int, [c_void_p, P(ctypes.c_float)]),
        "phiq_selector_load": (c_int, [c_void_p, ctypes.c_char_p]),
        "phiq_expm": (c_int, [c_void_p, c_int, c_int, c_void_p, P(c_double), c_void_p, c_void_p]),
        "phiq_kron_apply": (c_int, [c_void_p, c_int, P(c_int), P(c_void_p), c_void_p, c_void_p, c_int, c_int,
                                    c_void_p]),
        "phiq_profile_start": (c_int, [c_void_p, ctypes.c_uint]),
        "phiq_profile_stop": (c_int, [c_void_p, P(KernelStat), c_int, P(c_int)]),
        "phiq_profile_enable": (c_int, [c_void_p, c_int]),
        "phiq_tile_config": (c_int, [c_void_p, c_int, c_int, P(c_int)]),
        "phiq_autotune": (c_int, [c_void_p, c_int, P(c_int), c_int, c_int, P(c_double), c_void_p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
