"""ctypes declarations of the C ABI in include/spaqr.h (argument marshalling only)."""

from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

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


class StageStats(C.Structure):
    _fields_ = [("stage", C.c_int32), ("sparsified", C.c_int32), ("fronts", C.c_int32),
                ("max_front_rows", C.c_int32), ("max_front_pivots", C.c_int32), ("interfaces", C.c_int32),
                ("max_nbr_cols", C.c_int32), ("iface_size_q1", C.c_int32), ("iface_size_median", C.c_int32),
                ("iface_size_q3", C.c_int32), ("iface_size_max", C.c_int32), ("pad", C.c_int32),
                ("front_pivots", C.c_int64), ("iface_unknowns_in", C.c_int64), ("iface_unknowns_out", C.c_int64),
                ("nbr_cols", C.c_int64), ("top_separator", C.c_int64), ("factor_bytes", C.c_int64),
                ("flops_front", C.c_double), ("flops_scale", C.c_double), ("flops_sparsify", C.c_double),
                ("ms_front", C.c_double), ("ms_scale", C.c_double), ("ms_sparsify", C.c_double),
                ("ms_merge", C.c_double)]


class Tuning(C.Structure):
    _fields_ = [("qr_reg_max_rows", C.c_int), ("split_rows", C.c_int), ("split_cols", C.c_int),
                ("cpqr_reg", C.c_int), ("cpqr_coop", C.c_int), ("scale_small", C.c_int), ("iface_dense", C.c_int),
                ("trail_mfma", C.c_int), ("cpqr_dd", C.c_int),
                ("cpqr_team", C.c_int)]


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
    "spaqr_order_graph": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(_P)]),
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
    "spaqr_finalize": (None, []),
    "spaqr_stage_stats": (C.c_int, [_P, C.c_int, C.POINTER(StageStats)]),
    "spaqr_stage_interfaces": (C.c_int, [_P, C.c_int, _I32P, C.c_int64, _I64P]),
    "spaqr_solve_history": (C.c_int, [_P, _DP, C.c_int64, _I64P]),
    "spaqr_apply_noalloc": (C.c_int, [_P, _P, _P, C.c_int64, C.c_int64]),
    "spaqr_apply_noalloc_max": (C.c_int64, []),
    "spaqr_set_tuning": (C.c_int, [C.POINTER(Tuning)]),
    "spaqr_get_tuning": (C.c_int, [C.POINTER(Tuning)]),
    "spaqr_kernel_launches": (C.c_int, [C.c_char_p, _I64P]),
    "spaqr_server_status": (C.c_int, [_P, _I64P, _I64P, C.POINTER(C.c_size_t)]),
    "spaqr_estimate_bytes": (C.c_int, [_P, C.POINTER(Opts), C.c_int64, C.POINTER(C.c_size_t)]),
}

_lib = None

# Library objects alive in this process, by kind, in the order the exit hook
# releases them (a factorization reads its analysis, so it goes first).
_KINDS = ("factor", "server", "symbolic", "ordering")
_live = {k: weakref.WeakSet() for k in _KINDS}
_closed = False


def track(kind, obj):
    _live[kind].add(obj)


def released():
    """True once the exit hook has run: handles were freed there, and later
    destructors must not call into the library."""
    return _closed


def _exit_hook():
    """Frees every live handle and then the library's caches while the HIP
    runtime is still fully up (Python's exit hooks run before C++ static
    destruction and before the runtime unloads)."""
    global _closed
    if _closed or _lib is None:
        return
    for kind in _KINDS:
        for obj in list(_live[kind]):
            try:
                obj.close()
            except Exception:
                pass
    _lib.spaqr_finalize()
    _closed = True


def load():
    """Load libspaqr.so; raise ImportError if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2010_06807_amd.build`")
    try:
        # registered after torch's own hooks, so it runs before them
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    atexit.register(_exit_hook)
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
