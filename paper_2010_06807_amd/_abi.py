"""ctypes declarations of the C ABI in include/spaqr.h (argument marshalling only)."""

from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspaqr.so")

OK, ENOCONV, PENDING = 0, 1, 2
EINVAL, ENOMEM, ESINGULAR, EDEVICE = -1, -2, -3, -4


class CSR(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("rowptr", C.POINTER(C.c_int64)),
                ("col", C.POINTER(C.c_int32)), ("val", C.POINTER(C.c_double))]


class CSRDev(C.Structure):
    _fields_ = [("rowptr", C.c_void_p), ("col", C.c_void_p), ("val", C.c_void_p)]


class Opts(C.Structure):
    _fields_ = [("eps", C.c_double), ("skip", C.c_int), ("scale", C.c_int), ("precision", C.c_int),
                ("restart", C.c_int), ("maxit", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("relres", C.c_double),
                ("seconds", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("levels", C.c_int32), ("precision", C.c_int32),
                ("factor_bytes", C.c_int64), ("top_separator", C.c_int64), ("fronts", C.c_int64),
                ("interfaces_sparsified", C.c_int64), ("flops_front", C.c_double),
                ("flops_scale", C.c_double), ("flops_sparsify", C.c_double),
                ("ms_symbolic", C.c_double), ("ms_factor", C.c_double), ("ms_phase", C.c_double * 4)]


_P = C.c_void_p
_I64P = C.POINTER(C.c_int64)
_I32P = C.POINTER(C.c_int32)
_DP = C.POINTER(C.c_double)

# name: (restype, argtypes)
SIGNATURES = {
    "spaqr_status_string": (C.c_char_p, [C.c_int]),
    "spaqr_last_error": (C.c_char_p, []),
    "spaqr_order_grid": (C.c_int, [C.c_int, _I32P, C.c_int, C.POINTER(_P)]),
    "spaqr_ordering_free": (None, [_P]),
    "spaqr_ordering_n": (C.c_int64, [_P]),
    "spaqr_ordering_levels": (C.c_int, [_P]),
    "spaqr_ordering_perm": (C.c_int, [_P, _I64P]),
    "spaqr_ordering_num_clusters": (C.c_int64, [_P, C.c_int]),
    "spaqr_ordering_clusters": (C.c_int, [_P, C.c_int, _I64P, _I64P, _I64P, _I32P]),
    "spaqr_ordering_merge_parents": (C.c_int, [_P, C.c_int, _I64P]),
    "spaqr_opts_default": (Opts, []),
    "spaqr_analyze": (C.c_int, [C.POINTER(CSR), _P, C.POINTER(Opts), C.POINTER(_P)]),
    "spaqr_symbolic_free": (None, [_P]),
    "spaqr_symbolic_stage_info": (C.c_int, [_P, C.c_int, C.c_int, _I32P, C.c_int64, _I64P]),
    "spaqr_factor": (C.c_int, [C.POINTER(CSR), _P, C.POINTER(Opts), _P, C.POINTER(_P)]),
    "spaqr_factor_symbolic": (C.c_int, [C.POINTER(CSR), _P, C.POINTER(Opts), _P, C.POINTER(_P)]),
    "spaqr_factor_device": (C.c_int, [C.POINTER(CSR), C.POINTER(CSRDev), _P, C.POINTER(Opts), _P,
                                      C.POINTER(_P)]),
    "spaqr_factor_batch": (C.c_int, [C.c_int, C.POINTER(C.POINTER(CSR)), C.POINTER(C.POINTER(CSRDev)),
                                     C.POINTER(_P), C.POINTER(Opts), _P, C.POINTER(_P)]),
    "spaqr_apply": (C.c_int, [_P, _P, _P, C.c_int64, C.c_int64, C.c_int]),
    "spaqr_solve": (C.c_int, [_P, _P, _P, C.c_int64, C.c_int64, C.c_int, C.c_double,
                              C.POINTER(SolveInfo)]),
    "spaqr_solve_batch": (C.c_int, [C.c_int, C.POINTER(_P), C.POINTER(_P), C.POINTER(_P), _I64P, C.c_int, _DP,
                                    C.POINTER(SolveInfo)]),
    "spaqr_stats": (C.c_int, [_P, C.POINTER(Stats)]),
    "spaqr_stage_sizes": (C.c_int, [_P, C.c_int, _I32P, C.c_int64, _I64P]),
    "spaqr_free": (None, [_P]),
    "spaqr_profile_enable": (C.c_int, [C.c_int, C.c_char_p]),
    "spaqr_profile_query": (C.c_int, [C.c_char_p, _I64P, _DP, _DP, _DP]),
    "spaqr_server_create": (C.c_int, [C.c_size_t, _P, C.POINTER(_P)]),
    "spaqr_submit": (C.c_int, [_P, C.POINTER(CSR), _P, C.POINTER(Opts), _P, C.c_int64, C.c_double,
                               C.POINTER(C.c_uint64)]),
    "spaqr_server_step": (C.c_int, [_P, C.POINTER(C.c_int)]),
    "spaqr_poll": (C.c_int, [_P, C.c_uint64, _P, C.POINTER(SolveInfo)]),
    "spaqr_server_destroy": (None, [_P]),
}

_lib = None


def load():
    """Load libspaqr.so; raise ImportError if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2010_06807_amd.build`")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class SpaqrError(RuntimeError):
    def __init__(self, status, where):
        lib = load()
        msg = lib.spaqr_status_string(status).decode()
        detail = lib.spaqr_last_error().decode()
        super().__init__(f"{where}: {msg} ({status}){': ' + detail if detail else ''}")
        self.status = status


def check(status, where):
    if status < 0:
        raise SpaqrError(status, where)
    return status
