"""ctypes declarations of the C ABI in include/mnbab.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmnbab.so")

MNB_OK, MNB_PENDING = 0, 1
MNB_EINVAL, MNB_ENOMEM, MNB_EDEVICE, MNB_ETIMEOUT, MNB_ESTATE = -1, -2, -3, -4, -5
MNB_INPUT, MNB_FC, MNB_CONV, MNB_RELU, MNB_ADD, MNB_BN, MNB_AVGPOOL = 0, 1, 2, 3, 4, 5, 6
MNB_VERIFIED, MNB_FALSIFIED, MNB_UNKNOWN, MNB_TIMEOUT = 1, 2, 3, 4

fp = C.POINTER(C.c_float)
ip32 = C.POINTER(C.c_int32)
ip64 = C.POINTER(C.c_int64)


class Layer(C.Structure):
    _fields_ = [("kind", C.c_int), ("src", C.c_int), ("src2", C.c_int),
                ("in_chw", C.c_int * 3), ("out_chw", C.c_int * 3),
                ("k", C.c_int), ("stride", C.c_int), ("pad", C.c_int),
                ("W", fp), ("b", fp), ("eps", C.c_float)]


class Mnc(C.Structure):
    _fields_ = [("layer", C.c_int), ("e", C.c_int), ("row_ptr", ip32), ("col", ip32),
                ("P", fp), ("Phat", fp), ("p", fp)]


class OptCfg(C.Structure):
    _fields_ = [("steps", C.c_int), ("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float), ("recompute_intermediate", C.c_int), ("ckpt_stride", C.c_int),
                ("mem_budget", C.c_size_t)]


class Query(C.Structure):
    _fields_ = [("net_index", C.c_int), ("x_lo", fp), ("x_hi", fp), ("C", fp), ("c0", fp),
                ("n_spec", C.c_int), ("mnc", C.POINTER(Mnc)), ("n_mnc", C.c_int),
                ("timeout_s", C.c_double), ("mnc_cap", C.c_int)]


class Result(C.Structure):
    _fields_ = [("verdict", C.c_int), ("lb", C.c_float), ("subproblems", C.c_int64),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
                ("reason", C.c_int), ("restarts", C.c_int)]


class ServerCfg(C.Structure):
    _fields_ = [("opt", OptCfg), ("max_batch", C.c_int), ("queue_cap", C.c_int64),
                ("mem_budget", C.c_size_t), ("max_slots", C.c_int64)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

_SIGS = {
    "mnb_last_error": (C.c_char_p, []),
    "mnb_set_allocator": (C.c_int, [ALLOC_FN, FREE_FN, C.c_void_p]),
    "mnb_set_stream": (C.c_int, [C.c_void_p]),
    "mnb_net_create": (C.c_int, [C.POINTER(Layer), C.c_int, C.POINTER(C.c_void_p)]),
    "mnb_net_destroy": (None, [C.c_void_p]),
    "mnb_net_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                               C.POINTER(C.c_int)]),
    "mnb_problem_create": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_int, C.POINTER(C.c_void_p)]),
    "mnb_problem_destroy": (None, [C.c_void_p]),
    "bound_init": (C.c_int, [C.c_void_p, fp, fp, fp, fp, C.POINTER(Mnc), C.c_int, ip64, fp, fp]),
    "branch_split": (C.c_int, [C.c_void_p, ip64, ip32, ip32, C.c_int, ip64]),
    "mnb_opt_cfg_default": (None, [C.POINTER(OptCfg)]),
    "bound_optimize": (C.c_int, [C.c_void_p, ip64, C.c_int, C.POINTER(OptCfg), fp, fp, ip32, ip32]),
    "bound_optimize_begin": (C.c_int, [C.c_void_p, ip64, C.c_int, C.POINTER(OptCfg), C.POINTER(C.c_void_p)]),
    "bound_optimize_step": (C.c_int, [C.c_void_p]),
    "bound_optimize_end": (C.c_int, [C.c_void_p, fp, fp, ip32, ip32]),
    "mnb_opt_session_destroy": (None, [C.c_void_p]),
    "mnb_get_bounds": (C.c_int, [C.c_void_p, C.c_int64, C.c_int, fp, fp, C.POINTER(C.c_int8)]),
    "mnb_get_params": (C.c_int, [C.c_void_p, C.c_int64, C.c_int, fp, fp, fp]),
    "mnb_set_params": (C.c_int, [C.c_void_p, C.c_int64, C.c_int, fp, fp, fp]),
    "mnb_bound_grad": (C.c_int, [C.c_void_p, C.c_int64, C.c_int, C.POINTER(C.c_int), fp, fp, fp, fp]),
    "mnb_set_params_device": (C.c_int, [C.c_void_p, C.c_int64, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mnb_bound_grad_device": (C.c_int, [C.c_void_p, C.c_int64, C.c_int, C.POINTER(C.c_int), C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_void_p]),
    "mnb_branch_scores": (C.c_int, [C.c_void_p, ip64, C.c_int, fp, fp, ip32, ip32]),
    "mnb_branch_scores_noalloc": (C.c_int, [C.c_void_p, ip64, C.c_int, fp, fp, ip32, ip32]),
    "mnb_contribution_scores": (C.c_int, [C.c_void_p, ip64, C.c_int, fp, ip32, ip32]),
    "mnb_split_costs": (C.c_int, [C.POINTER(Layer), C.c_int, ip32, C.POINTER(C.c_double)]),
    "mnb_octahedral_bounds": (C.c_int, [C.c_void_p, C.c_int64, C.c_int, ip32, C.c_int, fp]),
    "mnb_mnc_generate": (C.c_int, [C.c_void_p, C.c_int64, C.c_int, ip32]),
    "mnb_get_mnc": (C.c_int, [C.c_void_p, C.c_int64, C.c_int, C.POINTER(C.c_int), ip32, ip32, fp, fp, fp]),
    "mnb_relu_hull": (C.c_int, [C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int)]),
    "mnb_release": (C.c_int, [C.c_void_p, ip64, C.c_int]),
    "mnb_problem_usage": (C.c_int, [C.c_void_p, ip64, ip64]),
    "mnb_kernel_fc_backsub": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_int]),
    "mnb_kernel_conv_backsub": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_int]),
    "mnb_kernel_fc_forward": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int]),
    "mnb_kernel_conv_forward": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int]),
    "mnb_sync": (C.c_int, []),
    "mnb_timer_begin": (C.c_int, [C.c_int, C.c_int]),
    "mnb_set_kernel_variants": (C.c_int, [C.c_int]),
    "mnb_get_kernel_variants": (C.c_int, []),
    "mnb_timer_end": (C.c_int, [ip64, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "mnb_server_cfg_default": (None, [C.POINTER(ServerCfg)]),
    "mnb_server_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.POINTER(ServerCfg), C.POINTER(C.c_void_p)]),
    "mnb_server_destroy": (None, [C.c_void_p]),
    "query_submit": (C.c_int, [C.c_void_p, C.POINTER(Query), C.POINTER(C.c_uint64)]),
    "query_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(Result)]),
}

_lib = None


def lib():
    """The loaded engine.  Raises if the HIP library has not been built: there is no fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2205_00263_amd/build.py "
                               "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name, None)
            if fn is None:
                continue
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    """Names of the ABI functions the binding declares (for the export test)."""
    return list(_SIGS)


class MnbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mnbab error {code}: {msg}")
        self.code = code


def check(code):
    if code < 0:
        raise MnbError(code, lib().mnb_last_error().decode(errors="replace"))
    return code
