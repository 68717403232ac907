"""ctypes view of the C ABI declared in include/fc.h.

This module only loads ``libfc.so`` and mirrors the header's structs and
signatures; it performs no computation.  Loading fails loudly when the
library has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfc.so")

# enums of fc.h
FC_OK, FC_ERR_INVALID_ARG, FC_ERR_UNSUPPORTED, FC_ERR_OUT_OF_MEMORY = 0, 1, 2, 3
FC_ERR_DEVICE, FC_ERR_NONFINITE, FC_ERR_STEP, FC_ERR_NOT_SYMMETRIC = 4, 5, 6, 7
FC_F64, FC_F32, FC_F16, FC_BF16 = 0, 1, 2, 3
FC_PREC_FP64, FC_PREC_FP32, FC_PREC_MIXED = 0, 1, 2
FC_DIAG_STORED, FC_DIAG_UNIT = 0, 1
FC_STEP_FIXED, FC_STEP_BACKTRACK = 0, 1
FC_REORDER_NONE, FC_REORDER_DEGREE, FC_REORDER_GIVEN = 0, 1, 2
FC_STOP_NONE, FC_STOP_MAXITER, FC_STOP_LOSS, FC_STOP_PGRAD, FC_STOP_ERROR = 0, 1, 2, 3, 4

STATUS_NAMES = {0: "FC_OK", 1: "FC_ERR_INVALID_ARG", 2: "FC_ERR_UNSUPPORTED",
                3: "FC_ERR_OUT_OF_MEMORY", 4: "FC_ERR_DEVICE", 5: "FC_ERR_NONFINITE",
                6: "FC_ERR_STEP", 7: "FC_ERR_NOT_SYMMETRIC", 8: "FC_ERR_CANCELLED"}
STATUS_CODES = {name: code for code, name in STATUS_NAMES.items()}

EXPORTED = [
    "fc_options_default", "fc_create", "fc_step", "fc_step_profiled", "fc_solve", "fc_get_u", "fc_get_history",
    "fc_get_state", "fc_set_state", "fc_destroy", "fc_objective", "fc_project", "fc_spmm",
    "fc_gram", "fc_spectral_norm", "fc_last_error",
    "fc_server_opts_default", "fc_server_clock", "fc_server_create", "fc_server_submit",
    "fc_server_poll", "fc_server_get_u", "fc_server_release", "fc_server_stats",
    "fc_server_destroy", "fc_server_tune", "fc_hessian_vector", "fc_curvature",
    "fc_gram_noalloc", "fc_gather_probe", "fc_server_cancel", "fc_debug_fail_allocations",
]


class CSR(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("values", ctypes.c_void_p), ("values_dtype", ctypes.c_int)]


class Options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("c", ctypes.c_int32),
                ("precision", ctypes.c_int), ("diag", ctypes.c_int),
                ("accelerate", ctypes.c_int32), ("step_rule", ctypes.c_int),
                ("step", ctypes.c_double), ("L0", ctypes.c_double), ("eta", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("tol_loss", ctypes.c_double), ("tol_pgrad", ctypes.c_double),
                ("validate", ctypes.c_int32), ("norm_estimate", ctypes.c_int32),
                ("step_schedule", ctypes.POINTER(ctypes.c_double)),
                ("step_schedule_len", ctypes.c_int32), ("reorder", ctypes.c_int32),
                ("defer_loss", ctypes.c_int32), ("single_pass", ctypes.c_int32),
                ("perm", ctypes.POINTER(ctypes.c_int32))]


class Info(ctypes.Structure):
    _fields_ = [("iter", ctypes.c_int32), ("trials", ctypes.c_int32),
                ("stop_reason", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("f", ctypes.c_double), ("f_prev", ctypes.c_double), ("L", ctypes.c_double),
                ("t", ctypes.c_double), ("beta", ctypes.c_double), ("pgrad", ctypes.c_double),
                ("pgrad_rel", ctypes.c_double)]


class KernelTimes(ctypes.Structure):
    _fields_ = [("fused_ms", ctypes.c_double), ("spmm_ms", ctypes.c_double),
                ("reduce_ms", ctypes.c_double), ("control_ms", ctypes.c_double),
                ("launches", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("max_active", ctypes.c_int32),
                ("hbm_budget", ctypes.c_double), ("ticks_per_poll", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("grid_fused", ctypes.c_int32 * 5),
                ("grid_spmm", ctypes.c_int32 * 5), ("solo_max", ctypes.c_int32),
                ("spmm_depth", ctypes.c_int32 * 5), ("reserved", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("req_id", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("iter", ctypes.c_int32), ("trials", ctypes.c_int32),
                ("stop_reason", ctypes.c_int32), ("f", ctypes.c_double),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_finish", ctypes.c_double), ("t_setup", ctypes.c_double),
                ("t_start", ctypes.c_double)]


_lib = None


def load() -> ctypes.CDLL:
    """Load libfc.so (built by paper_2506_04045_amd.build); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2506_04045_amd.build` "
            "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    st = ctypes.c_int
    lib.fc_options_default.argtypes = [P]
    lib.fc_options_default.restype = None
    lib.fc_create.argtypes = [ctypes.POINTER(CSR), ctypes.POINTER(Options), P, ctypes.c_int, P,
                              ctypes.POINTER(P)]
    lib.fc_create.restype = st
    lib.fc_step.argtypes = [P, i32, ctypes.POINTER(Info)]
    lib.fc_step.restype = st
    lib.fc_step_profiled.argtypes = [P, i32, ctypes.POINTER(Info), ctypes.POINTER(KernelTimes)]
    lib.fc_step_profiled.restype = st
    lib.fc_solve.argtypes = [P, ctypes.POINTER(Info)]
    lib.fc_solve.restype = st
    lib.fc_get_u.argtypes = [P, P, ctypes.c_int]
    lib.fc_get_u.restype = st
    lib.fc_get_history.argtypes = [P, i32, P, P, P, P, ctypes.POINTER(i32)]
    lib.fc_get_history.restype = st
    lib.fc_get_state.argtypes = [P, P, ctypes.POINTER(ctypes.c_size_t)]
    lib.fc_get_state.restype = st
    lib.fc_set_state.argtypes = [P, P, ctypes.c_size_t]
    lib.fc_set_state.restype = st
    lib.fc_destroy.argtypes = [P]
    lib.fc_destroy.restype = None
    lib.fc_objective.argtypes = [ctypes.POINTER(CSR), ctypes.c_int, P, ctypes.c_int, i32, P,
                                 ctypes.POINTER(f64)]
    lib.fc_objective.restype = st
    lib.fc_project.argtypes = [P, P, ctypes.c_int, i64, i32, i64, P]
    lib.fc_project.restype = st
    lib.fc_spmm.argtypes = [ctypes.POINTER(CSR), ctypes.c_int, P, P, ctypes.c_int, i32, P]
    lib.fc_spmm.restype = st
    lib.fc_gram.argtypes = [P, ctypes.c_int, i64, i32, P, P]
    lib.fc_gram.restype = st
    lib.fc_gram_noalloc.argtypes = [P, ctypes.c_int, i64, i32, i64, P, P]
    lib.fc_gram_noalloc.restype = st
    lib.fc_gather_probe.argtypes = [P, i64, P, i64, i32, i32, i32, P, ctypes.POINTER(f64)]
    lib.fc_gather_probe.restype = st
    lib.fc_debug_fail_allocations.argtypes = [i64]
    lib.fc_debug_fail_allocations.restype = None
    lib.fc_spectral_norm.argtypes = [ctypes.POINTER(CSR), ctypes.c_int, i32, f64, P,
                                     ctypes.POINTER(f64), ctypes.POINTER(i32)]
    lib.fc_spectral_norm.restype = st
    lib.fc_last_error.argtypes = []
    lib.fc_last_error.restype = ctypes.c_char_p
    lib.fc_server_opts_default.argtypes = [P]
    lib.fc_server_opts_default.restype = None
    lib.fc_server_clock.argtypes = []
    lib.fc_server_clock.restype = f64
    lib.fc_server_create.argtypes = [ctypes.POINTER(ServerOpts), P, ctypes.POINTER(P)]
    lib.fc_server_create.restype = st
    lib.fc_server_submit.argtypes = [P, ctypes.POINTER(CSR), ctypes.POINTER(Options), P,
                                     ctypes.c_int, ctypes.c_uint64]
    lib.fc_server_submit.restype = st
    lib.fc_server_poll.argtypes = [P, ctypes.POINTER(Result), i32, i32, ctypes.POINTER(i32)]
    lib.fc_server_poll.restype = st
    lib.fc_server_get_u.argtypes = [P, ctypes.c_uint64, P, ctypes.c_int]
    lib.fc_server_get_u.restype = st
    lib.fc_server_release.argtypes = [P, ctypes.c_uint64]
    lib.fc_server_release.restype = st
    lib.fc_server_cancel.argtypes = [P, ctypes.c_uint64]
    lib.fc_server_cancel.restype = st
    lib.fc_server_tune.argtypes = [ctypes.POINTER(ServerOpts), i32, ctypes.POINTER(CSR),
                                   ctypes.POINTER(Options), ctypes.POINTER(P), ctypes.c_int, P,
                                   ctypes.POINTER(ServerOpts), ctypes.POINTER(f64),
                                   ctypes.POINTER(i32)]
    lib.fc_server_tune.restype = st
    lib.fc_server_stats.argtypes = [P, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                    ctypes.POINTER(i64), ctypes.POINTER(f64)]
    lib.fc_server_stats.restype = st
    lib.fc_server_destroy.argtypes = [P]
    lib.fc_server_destroy.restype = None
    lib.fc_hessian_vector.argtypes = [ctypes.POINTER(CSR), ctypes.c_int, P, P, P, ctypes.c_int,
                                      i32, P]
    lib.fc_hessian_vector.restype = st
    lib.fc_curvature.argtypes = [ctypes.POINTER(CSR), ctypes.c_int, P, P, ctypes.c_int, i32, i32,
                                 f64, ctypes.POINTER(ctypes.c_double), P,
                                 ctypes.POINTER(ctypes.c_int32), P]
    lib.fc_curvature.restype = st
    _lib = lib
    return lib


class FcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def check(status: int) -> None:
    if status != FC_OK:
        msg = load().fc_last_error()
        raise FcError(status, msg.decode() if msg else "")


def default_server_options() -> ServerOpts:
    lib = load()
    raw = (ctypes.c_char * 256)()
    lib.fc_server_opts_default(ctypes.cast(raw, ctypes.c_void_p))
    size = ctypes.c_uint32.from_buffer(raw).value
    if size != ctypes.sizeof(ServerOpts):
        raise RuntimeError(f"fc_server_opts layout mismatch: C {size} vs ctypes "
                           f"{ctypes.sizeof(ServerOpts)}")
    return ServerOpts.from_buffer_copy(bytes(raw[:size]))


def default_options() -> Options:
    """fc_options_default into a buffer larger than the struct, then checked
    against this module's layout."""
    lib = load()
    raw = (ctypes.c_char * 512)()
    lib.fc_options_default(ctypes.cast(raw, ctypes.c_void_p))
    size = ctypes.c_uint32.from_buffer(raw).value
    if size != ctypes.sizeof(Options):
        raise RuntimeError(f"fc_options layout mismatch: C {size} vs ctypes {ctypes.sizeof(Options)}")
    return Options.from_buffer_copy(bytes(raw[:size]))
