"""ctypes declarations of the C ABI in include/ddelm.h (argument marshalling only)."""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libddelm.so")

c_double_p = ctypes.POINTER(ctypes.c_double)
c_int_p = ctypes.POINTER(ctypes.c_int)

DDELM_OK = 0
DDELM_WARN_NOCONV = 1
STATUS_NAMES = {
    0: "DDELM_OK", 1: "DDELM_WARN_NOCONV", -1: "DDELM_E_ARG", -2: "DDELM_E_SHAPE", -3: "DDELM_E_STATE",
    -4: "DDELM_E_HIP", -5: "DDELM_E_NOMEM", -6: "DDELM_E_CHOLESKY", -7: "DDELM_E_NONFINITE",
}


class Problem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("lo", ctypes.c_double * 2), ("hi", ctypes.c_double * 2),
        ("p", ctypes.c_int), ("edge_s", c_double_p),
        ("n_extra", ctypes.c_int), ("extra_s", c_double_p),
        ("n_int", ctypes.c_int), ("x_int", ctypes.c_void_p),
        ("M", ctypes.c_int), ("W", ctypes.c_void_p), ("b", ctypes.c_void_p),
    ]


class Options(ctypes.Structure):
    _fields_ = [
        ("theta", ctypes.c_double), ("coarse", ctypes.c_int), ("precision", ctypes.c_int),
        ("tol", ctypes.c_double), ("maxit", ctypes.c_int), ("max_nrhs", ctypes.c_int),
        ("cg_mode", ctypes.c_int), ("refine_maxit", ctypes.c_int), ("refine_tol", ctypes.c_double),
        ("inner_tol", ctypes.c_double),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int), ("refine_steps", ctypes.c_int), ("rel_res", ctypes.c_double),
        ("ms_rhs", ctypes.c_double), ("ms_cg", ctypes.c_double), ("ms_recover", ctypes.c_double),
        ("cg_blocks", ctypes.c_int), ("cg_slices", ctypes.c_int), ("cg_coarse_dist", ctypes.c_int),
        ("cg_restarts", ctypes.c_int), ("true_rel_res", ctypes.c_double), ("refine_corr", ctypes.c_double),
        ("kappa_est_max", ctypes.c_double), ("start_rel_res", ctypes.c_double),
    ]


class Sizes(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int), ("M", ctypes.c_int), ("n_pi", ctypes.c_int), ("n_dl", ctypes.c_int),
        ("n_int", ctypes.c_int), ("max_m", ctypes.c_int), ("sum_nB", ctypes.c_longlong),
        ("sum_nG", ctypes.c_longlong),
    ]


# name -> (restype, argtypes)
SIGNATURES = {
    "ddelm_default_options": (None, [ctypes.POINTER(Options)]),
    "ddelm_setup": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(Problem),
                                   ctypes.POINTER(Options), ctypes.c_void_p]),
    "ddelm_factor": (ctypes.c_int, [ctypes.c_void_p]),
    "ddelm_set_coefficient": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "ddelm_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.POINTER(Stats)]),
    "ddelm_solve_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(Stats)]),
    "ddelm_solve_general": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(Stats)]),
    "ddelm_evaluate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_longlong,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "ddelm_solve_adjoint": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.POINTER(Stats)]),
    "ddelm_solve_adjoint_general": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                   ctypes.POINTER(Stats)]),
    "ddelm_evaluate_adjoint": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_longlong, ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "ddelm_get_sizes": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Sizes)]),
    "ddelm_get_counts": (ctypes.c_int, [ctypes.c_void_p, c_int_p, c_int_p, c_int_p, c_int_p]),
    "ddelm_get_indexing": (ctypes.c_int, [ctypes.c_void_p, c_int_p, c_int_p]),
    "ddelm_get_boundary_points": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "ddelm_get_interface_points": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "ddelm_get_local_matrix": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                              c_int_p, c_int_p]),
    "ddelm_get_phase_times": (ctypes.c_int, [ctypes.c_void_p, c_double_p]),
    "ddelm_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "ddelm_destroy": (None, [ctypes.c_void_p]),
    "ddelm_release_cached_memory": (ctypes.c_int, []),
}

_lib = None
_live = weakref.WeakSet()     # objects holding a context (with a close() method)


def register(obj) -> None:
    """Track an object that owns a context, so that it is closed at exit."""
    _live.add(obj)


def _release_at_exit() -> None:
    # Contexts still alive at interpreter exit are destroyed, and the library's
    # idle memory, streams, events and pinned buffers are handed back, while
    # the HIP runtime (and any tool attached to it) is still fully up.
    if _lib is None:
        return
    for obj in list(_live):
        try:
            obj.close()
        except Exception:
            pass
    _lib.ddelm_release_cached_memory()


def load() -> ctypes.CDLL:
    """Load libddelm.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2503_10032_amd._build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    atexit.register(_release_at_exit)
    return lib
