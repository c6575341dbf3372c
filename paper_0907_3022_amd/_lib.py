"""ctypes binding of libchebtd.so (the C ABI in include/chebtd.h).

Argument marshalling only: every step of the propagation runs in the HIP
kernels of the library.  If the library has not been built this module
raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

# CHEBTD_LIB names another build of the same library (the host-sanitizer
# build of the tests); by default the in-tree one
LIB_PATH = os.environ.get("CHEBTD_LIB") or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                        "libchebtd.so")

OK = 0
E_ARG, E_HIP, E_DIVERGED, E_OOM, E_STATE, E_TIMEOUT = -1, -2, -3, -4, -5, -6
ZIGZAG, ARMCHAIR = 0, 1
KEEP_CHECKPOINTS, NO_CHECK, GRAPH, NO_PERSISTENT, SINGLE_ORDER = 1, 2, 4, 8, 16
SCHED_LEVELS, SCHED_PERSISTENT, SCHED_PAIRS, SCHED_DEEP = 0, 1, 2, 3
ADJ_STEP, ADJ_SQRTM, ADJ_REVERSE = 0, 1, 2

_ERRNAMES = {E_ARG: "CHEBTD_E_ARG", E_HIP: "CHEBTD_E_HIP", E_DIVERGED: "CHEBTD_E_DIVERGED",
             E_OOM: "CHEBTD_E_OOM", E_STATE: "CHEBTD_E_STATE", E_TIMEOUT: "CHEBTD_E_TIMEOUT"}


class ChebError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class SysDesc(C.Structure):
    _fields_ = [("width", C.c_int64), ("length", C.c_int64), ("edge", C.c_int),
                ("t_hop", C.c_double), ("eps_dev", C.c_void_p), ("emin", C.c_double),
                ("emax", C.c_double), ("psi_dev", C.c_void_p)]


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "chebtd_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_void_p]),
    "chebtd_destroy": (C.c_int, [C.c_void_p]),
    "chebtd_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "chebtd_last_error": (C.c_char_p, [C.c_void_p]),
    "chebtd_version": (C.c_int, []),
    "chebtd_h_chain1d": (C.c_int, [C.c_void_p, C.c_int64, C.c_double, C.c_void_p]),
    "chebtd_h_honeycomb": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.c_int, C.c_double,
                                     C.c_void_p]),
    "chebtd_h_csr": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p,
                               C.c_void_p]),
    "chebtd_h_holstein": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_double, C.c_double,
                                    C.c_void_p, C.c_void_p, C.c_int]),
    "chebtd_holstein_csr_host": (C.c_int, [C.c_int, C.c_int, C.c_double, C.c_double, C.c_void_p,
                                           C.c_void_p, C.c_int, C.POINTER(C.c_int64),
                                           C.POINTER(C.c_int64), C.c_void_p, C.c_void_p,
                                           C.c_void_p]),
    "chebtd_holstein_occupations": (C.c_int, [C.c_int, C.c_int, C.POINTER(C.c_int64), C.c_void_p]),
    "chebtd_dim": (C.c_int64, [C.c_void_p]),
    "chebtd_gershgorin": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "chebtd_set_bounds": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_double]),
    "chebtd_plan": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.POINTER(C.c_int)]),
    "chebtd_plan_order": (C.c_int, [C.c_void_p, C.c_double, C.c_int]),
    "chebtd_get_plan": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_double),
                                  C.POINTER(C.c_double), C.POINTER(C.c_double),
                                  C.POINTER(C.c_int)]),
    "chebtd_plan_passes": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.POINTER(C.c_int)]),
    "chebtd_propagate": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                   C.c_uint]),
    "chebtd_propagate_td": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                                      C.c_void_p, C.c_void_p, C.c_uint]),
    "chebtd_crank_nicolson": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_int64]),
    "chebtd_set_check_tol": (C.c_int, [C.c_void_p, C.c_double]),
    "chebtd_density": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "chebtd_region_sum": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "chebtd_region_sum_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "chebtd_norm_energy": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "chebtd_holstein_obs": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p]),
    "chebtd_batch_create": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(SysDesc), C.c_double,
                                      C.c_double, C.c_double]),
    "chebtd_batch_set_schedule": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int]),
    "chebtd_batch_autotune": (C.c_int, [C.c_void_p, C.c_char_p, C.POINTER(C.c_int)]),
    "chebtd_batch_propagate": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_uint]),
    "chebtd_batch_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.c_void_p]),
    "chebtd_reserve_adjoint": (C.c_int, [C.c_void_p, C.c_int64, C.c_int]),
    "chebtd_adjoint": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "chebtd_checkpoint_run": (C.c_int, [C.c_void_p, C.c_void_p]),
    "chebtd_adjoint_run": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "chebtd_time_recursion_kernel": (C.c_int, [C.c_void_p, C.c_int, C.c_uint, C.POINTER(C.c_double),
                                               C.POINTER(C.c_char_p), C.POINTER(C.c_int)]),
}


def exported_names():
    return list(_SIGS)


def lib():
    """Load libchebtd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ChebError(E_STATE, f"{LIB_PATH} is missing; build it with "
                                 "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def last_error(handle=None) -> str:
    msg = lib().chebtd_last_error(handle)
    return msg.decode() if msg else ""


def check(rc: int, handle=None):
    if rc != OK:
        raise ChebError(rc, last_error(handle))
