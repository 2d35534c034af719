"""ctypes binding of libmlcr.so (argument marshalling only).

Loading fails loudly if the library has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmlcr.so")

c_int, c_ll, c_dbl_p, c_void_p = ctypes.c_int, ctypes.c_longlong, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p

# name -> (restype, argtypes)
SIGNATURES = {
    "mlcr_last_error": (ctypes.c_char_p, []),
    "mlcr_version": (ctypes.c_char_p, []),
    "mlcr_geom_create": (c_int, [c_int, c_int, ctypes.POINTER(c_void_p)]),
    "mlcr_geom_create_gl": (c_int, [c_int, c_int, c_int, ctypes.POINTER(c_void_p)]),
    "mlcr_geom_weights": (c_int, [c_void_p, c_void_p]),
    "mlcr_geom_set_tuning": (c_int, [c_void_p, c_int, c_int, c_int, c_int]),
    "mlcr_geom_get_tuning": (c_int, [c_void_p, c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_int),
                                     ctypes.POINTER(c_int)]),
    "mlcr_geom_destroy": (None, [c_void_p]),
    "mlcr_geom_info": (c_int, [c_void_p, ctypes.POINTER(c_int), ctypes.POINTER(c_int),
                               ctypes.POINTER(c_ll), ctypes.POINTER(c_int)]),
    "sht_synth": (c_int, [c_void_p, c_int, c_int, c_void_p, c_void_p, c_int, c_void_p]),
    "sht_adjoint": (c_int, [c_void_p, c_int, c_int, c_void_p, c_void_p, c_int, c_void_p]),
    "sht_synth_noalloc": (c_int, [c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p]),
    "mlcr_op_create": (c_int, [c_void_p, c_int, c_dbl_p, c_dbl_p, c_void_p, c_int,
                               ctypes.POINTER(c_void_p)]),
    "mlcr_op_destroy": (None, [c_void_p]),
    "mlcr_op_set_level": (c_int, [c_void_p, c_int, c_int, c_dbl_p]),
    "mlcr_op_set_level_gl": (c_int, [c_void_p, c_int, c_int, c_dbl_p]),
    "mlcr_op_level_lmax": (c_int, [c_void_p, c_int]),
    "apply_A": (c_int, [c_void_p, c_int, c_int, c_void_p, c_void_p, c_int, c_void_p]),
    "mlcr_solver_create": (c_int, [c_void_p, c_void_p, c_int, ctypes.POINTER(c_void_p)]),
    "mlcr_ladder_default": (c_int, [c_int, c_int, c_void_p, c_void_p]),
    "mlcr_ladder_check": (c_int, [c_int, c_int, c_void_p]),
    "mlcr_solver_set_profile": (c_int, [c_void_p, c_int]),
    "mlcr_solver_profile": (c_int, [c_void_p, c_int, c_void_p, c_void_p]),
    "mlcr_op_set_prior": (c_int, [c_void_p, c_dbl_p]),
    "mlcr_prior_band_grad": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_int, c_void_p,
                                     c_void_p, c_void_p]),
    "mlcr_solver_destroy": (None, [c_void_p]),
    "mlcr_solver_info": (c_int, [c_void_p, ctypes.POINTER(c_int), ctypes.POINTER(c_int),
                                 ctypes.POINTER(c_int), ctypes.POINTER(ctypes.c_float)]),
    "mlcr_solver_top_dinv": (c_int, [c_void_p, c_void_p, c_void_p]),
    "mlcr_solver_bottom": (c_int, [c_void_p, ctypes.POINTER(c_int), c_void_p, c_void_p]),
    "mlcr_solver_level_blocks": (c_int, [c_void_p, c_int, c_int, ctypes.POINTER(c_int),
                                         ctypes.POINTER(c_ll), c_void_p, c_void_p]),
    "wcycle_solve": (c_int, [c_void_p, c_int, c_void_p, c_void_p, ctypes.c_double, c_int, c_int,
                             c_void_p, c_void_p]),
    "mlcr_solver_set_graph": (c_int, [c_void_p, c_int]),
    "mlcr_solver_graph_stats": (c_int, [c_void_p, ctypes.POINTER(c_ll), ctypes.POINTER(c_ll)]),
    "pcg_solve": (c_int, [c_void_p, c_int, c_void_p, c_void_p, ctypes.c_double, c_int, c_int,
                          c_void_p, c_void_p]),
    "mlcr_cr_rhs": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "apply_A_grouped": (c_int, [c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_void_p]),
    "wcycle_solve_grouped": (c_int, [c_int, c_void_p, c_void_p, c_void_p, c_void_p, ctypes.c_double,
                                     c_int, c_int, c_void_p, c_void_p]),
    "mlcr_nest2ring": (c_int, [c_int, c_ll, c_void_p, c_void_p]),
    "mlcr_tile_graph": (c_int, [c_int, c_int, c_void_p, c_void_p, c_void_p, ctypes.POINTER(c_int),
                                ctypes.POINTER(c_int)]),
    "mlcr_ladder_plan": (c_int, [c_int, c_int, ctypes.POINTER(c_int), c_void_p, c_void_p, c_void_p,
                                 ctypes.POINTER(c_int), ctypes.POINTER(c_int)]),
    "mlcr_cycle_counts": (c_int, [c_int, c_void_p, c_int, c_int, c_void_p]),
    "mlcr_timing_enable": (c_int, [c_int]),
    "mlcr_timing_reset": (c_int, []),
    "mlcr_timing_count": (c_int, []),
    "mlcr_timing_get": (c_int, [c_int, ctypes.c_char_p, c_int, ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(c_ll)]),
}

_lib = None


class LadderDesc(ctypes.Structure):
    """mlcr_ladder_desc (include/mlcr.h)."""
    _fields_ = [("nlevels", ctypes.c_int), ("nside", ctypes.c_int * 8), ("lmax", ctypes.c_int * 8),
                ("nrec", ctypes.c_int * 8), ("nrec_top", ctypes.c_int), ("lmax_dense", ctypes.c_int),
                ("filter", c_dbl_p * 8), ("highpass", c_dbl_p), ("gl_levels", ctypes.c_int),
                ("smoother", ctypes.c_int), ("ridge_min", ctypes.c_double),
                ("ridge_max", ctypes.c_double), ("keep_blocks", ctypes.c_int)]


class SolveInfo(ctypes.Structure):
    """mlcr_solve_info (include/mlcr.h)."""
    _fields_ = [("cycles", ctypes.c_int), ("converged", ctypes.c_int), ("rho0", ctypes.c_double),
                ("rho", ctypes.c_double), ("s_half_res", ctypes.c_double)]


class MLCRError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mlcr error {code}: {msg}")
        self.code = code


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1308_5299_amd.build` "
            "(or __graft_entry__.build()); there is no non-HIP fallback")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(rc: int) -> None:
    if rc != 0:
        msg = load().mlcr_last_error().decode()
        raise MLCRError(rc, msg)
