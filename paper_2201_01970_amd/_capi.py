"""ctypes declarations of the C ABI in include/cpr.h and include/cpr_inspect.h.

Argument marshalling only: every step of the solve runs in the HIP library.
Importing this module does not load the library; ``lib()`` does, and raises
if it has not been built (there is no fallback path).
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcpr_mi355x.so")

CPR_OK = 0
CPR_NOT_CONVERGED = 1
CPR_ERR_INVALID_ARG = -1
CPR_ERR_PATTERN_MISMATCH = -2
CPR_ERR_SIZE_MISMATCH = -3
CPR_ERR_SINGULAR_BLOCK = -4
CPR_ERR_SINGULAR_COARSE = -5
CPR_ERR_NAN = -6
CPR_ERR_OOM = -7
CPR_ERR_HIP = -8

CPR_MEM_HOST = 0
CPR_MEM_DEVICE = 1

CPR_KSTAT_SPMV = 0
CPR_KSTAT_SMOOTH_L0 = 1
CPR_KSTAT_TRANSFER_L0 = 2
CPR_KSTAT_STAGE2 = 3
CPR_KSTAT_SMOOTH_COARSE = 4
CPR_KSTAT_TRANSFER_COARSE = 5
CPR_KSTAT_TAIL = 6
CPR_KSTAT_COUNT = 7


class cpr_bsr(C.Structure):
    _fields_ = [
        ("n_block_rows", C.c_int32),
        ("nnz_blocks", C.c_int32),
        ("block_dim", C.c_int32),
        ("row_ptr", C.c_void_p),
        ("col_idx", C.c_void_p),
        ("values", C.c_void_p),
        ("location", C.c_int32),
    ]


class cpr_params(C.Structure):
    _fields_ = [
        ("restart", C.c_int32),
        ("max_restarts", C.c_int32),
        ("theta_rs", C.c_double),
        ("theta_color", C.c_double),
        ("coarse_max", C.c_int32),
        ("max_levels", C.c_int32),
        ("pre_sweeps", C.c_int32),
        ("post_sweeps", C.c_int32),
        ("precond_fp32", C.c_int32),
        ("reuse_mode", C.c_int32),
        ("mu", C.c_int32),
        ("reuse_factor", C.c_double),
        ("use_graphs", C.c_int32),
        ("tail_nnz", C.c_int32),
        ("row_layout", C.c_int32),
        ("second_stage", C.c_int32),
        ("decoupling", C.c_int32),
        ("smoother", C.c_int32),
        ("smoother_chunks", C.c_int32),
        ("amg_kind", C.c_int32),
        ("amli_inner", C.c_int32),
        ("npair", C.c_int32),
        ("pair_beta", C.c_double),
        ("coarse_solver", C.c_int32),
    ]


class cpr_solve_info(C.Structure):
    _fields_ = [
        ("iterations", C.c_int32),
        ("restarts", C.c_int32),
        ("rebuilt", C.c_int32),
        ("n_levels", C.c_int32),
        ("relres_true", C.c_double),
        ("relres_est", C.c_double),
        ("setup_ms", C.c_double),
        ("solve_ms", C.c_double),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class cpr_request(C.Structure):
    _fields_ = [
        ("case_id", C.c_int64),
        ("A", cpr_bsr),
        ("b", C.c_void_p),
        ("x", C.c_void_p),
        ("tol", C.c_double),
    ]


class cpr_server_stats(C.Structure):
    _fields_ = [(name, C.c_int64) for name in (
        "submitted", "completed", "rejected", "setups", "reuses", "evictions",
        "resident_cases", "bytes_in_use", "bytes_peak", "budget_bytes")]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


_P = C.c_void_p
_I32 = C.c_int32
_I64 = C.c_int64
_D = C.c_double

# name -> (restype, argtypes)
SIGNATURES = {
    "cpr_params_default": (None, [C.POINTER(cpr_params)]),
    "cpr_setup": (_I32, [C.POINTER(cpr_bsr), C.POINTER(cpr_params), _P, C.POINTER(_P)]),
    "cpr_update_values": (_I32, [_P, C.POINTER(cpr_bsr)]),
    "cpr_solve": (_I32, [_P, _P, _P, _D, C.POINTER(cpr_solve_info)]),
    "cpr_second_stage": (_I32, [_P, _P, _P, _P]),
    "cpr_bilu_factors": (_I32, [_P, _P, _P, _P, _P, _P]),
    "cpr_solve_noalloc": (_I32, [_P, _P, _P, _D, C.POINTER(cpr_solve_info)]),
    "cpr_set_stream": (_I32, [_P, _P]),
    "cpr_destroy": (None, [_P]),
    "cpr_status_string": (C.c_char_p, [_I32]),
    "cpr_last_error": (C.c_char_p, [_P]),
    "cpr_device_bytes": (_I64, [_P]),
    "cpr_spmv": (_I32, [_P, _P, _P]),
    "cpr_precond_apply": (_I32, [_P, _P, _P]),
    "cpr_vcycle": (_I32, [_P, _P, _P]),
    "cpr_smooth": (_I32, [_P, _I32, _P, _P, _I32, _I32]),
    "cpr_level_info": (_I32, [_P, _I32, _P]),
    "cpr_level_arrays": (_I32, [_P, _I32, _P, _P, _P, _P, _P, _P, _P]),
    "cpr_level_interp": (_I32, [_P, _I32, _P, _P, _P]),
    "cpr_block_colours": (_I32, [_P, _P]),
    "cpr_level_aggregates": (_I32, [_P, _I32, _P]),
    "cpr_host_grouping": (_I32, [_I32, _P, _P, _P, _P]),
    "cpr_host_rs_split": (_I32, [_I32, _P, _P, _P]),
    "cpr_host_interpolation": (_I32, [_I32, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "cpr_host_bilu0": (_I32, [_I32, _P, _P, _P, _P, _P, _P, _P]),
    "cpr_host_aggregates": (_I32, [_I32, _P, _P, _P, _D, _I32, _P, _P]),
    "cpr_host_galerkin": (_I32, [_I32, _I32, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "cpr_profile_enable": (_I32, [_P, _I32]),
    "cpr_profile_read": (_I32, [_P, _I32, _P, _P, _P]),
    "cpr_copy_kernel": (_I32, [_P, _P, _I64, _P]),
    "cpr_server_create": (_I32, [_I64, _I32, C.POINTER(cpr_params), C.POINTER(_P)]),
    "cpr_server_submit": (_I32, [_P, C.POINTER(cpr_request), C.POINTER(_I64)]),
    "cpr_server_wait": (_I32, [_P, _I64, C.POINTER(cpr_solve_info), C.POINTER(_D)]),
    "cpr_server_stats_get": (_I32, [_P, C.POINTER(cpr_server_stats)]),
    "cpr_server_destroy": (None, [_P]),
    "cpr_server_last_error": (C.c_char_p, [_P]),
}

_lib = None


def lib():
    """The loaded HIP library; raises RuntimeError if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2201_01970_amd.build` "
                "(there is no CPU fallback)")
        handle = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


class CprError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{status_name(status)}: {message}")
        self.status = status


def status_name(st):
    return lib().cpr_status_string(st).decode()


def check(st, handle=None, allow=(CPR_OK,)):
    if st in allow:
        return st
    msg = lib().cpr_last_error(handle).decode()
    raise CprError(st, msg)
