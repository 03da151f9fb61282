"""ctypes declarations of the C ABI in include/sbm.h (argument marshalling only).

The library is loaded from this package directory; there is no fallback: if
``libsbm.so`` is missing the import of the solver fails loudly.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsbm.so")

SBM_OK = 0
SBM_NOT_CONVERGED = 1
STATUS_NAMES = {0: "SBM_OK", 1: "SBM_NOT_CONVERGED", -1: "SBM_E_ARG", -2: "SBM_E_SHAPE",
                -3: "SBM_E_HIP", -4: "SBM_E_NONFINITE", -5: "SBM_E_DIVERGED", -6: "SBM_E_DIAG",
                -7: "SBM_E_WORKSPACE"}
TRACTION = 0
DISPLACEMENT = 1
CHAIN_PSI, CHAIN_FLOOR, CHAIN_RHO3 = 0, 1, 2
PROF_CLASSES = ("smooth", "residual", "restrict", "prolong", "norm", "bottom", "ghost", "sweep0",
                "smooth_dot")


class SbmGrid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("ncell", ctypes.c_int64 * 3), ("h", ctypes.c_double * 3)]


class SbmBc(ctypes.Structure):
    _fields_ = [("kind", (ctypes.c_int * 3) * 6), ("value", (ctypes.c_double * 3) * 6)]


class SbmMaterial(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("mu", ctypes.c_double),
                ("psi_floor", ctypes.c_double)]


class SbmJ2(ctypes.Structure):
    _fields_ = [("sigma_y", ctypes.c_double), ("hbar", ctypes.c_double), ("theta", ctypes.c_double)]


class SbmPf(ctypes.Structure):
    _fields_ = [("Gc", ctypes.c_double), ("xi", ctypes.c_double), ("M", ctypes.c_double),
                ("dt", ctypes.c_double), ("eta", ctypes.c_double)]


class SbmOptions(ctypes.Structure):
    _fields_ = [("smoother", ctypes.c_int), ("omega", ctypes.c_double), ("nu_pre", ctypes.c_int),
                ("nu_post", ctypes.c_int), ("precision", ctypes.c_int), ("rtol", ctypes.c_double),
                ("max_cycles", ctypes.c_int), ("bottom_rtol", ctypes.c_double),
                ("bottom_max_iter", ctypes.c_int), ("use_graphs", ctypes.c_int),
                ("krylov", ctypes.c_int), ("fused_sweep", ctypes.c_int)]


_P = ctypes.c_void_p
_DP = ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int)
_I64P = ctypes.POINTER(ctypes.c_int64)

# name -> (restype, argtypes)
SIGNATURES = {
    "sbm_default_options": (None, [ctypes.POINTER(SbmOptions)]),
    "sbm_num_levels": (ctypes.c_int, [ctypes.POINTER(SbmGrid)]),
    "sbm_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(SbmGrid), ctypes.POINTER(SbmOptions)]),
    "sbm_create": (ctypes.c_int, [ctypes.POINTER(SbmGrid), ctypes.POINTER(SbmOptions), _P,
                                  ctypes.c_size_t, _P, ctypes.POINTER(_P)]),
    "sbm_set_options": (ctypes.c_int, [_P, ctypes.POINTER(SbmOptions)]),
    "sbm_set_problem": (ctypes.c_int, [_P, _P, ctypes.POINTER(SbmMaterial), ctypes.POINTER(SbmBc),
                                       _P]),
    "sbm_solve": (ctypes.c_int, [_P, _P, _DP, ctypes.c_int, _IP, _DP]),
    "sbm_solve_rhs": (ctypes.c_int, [_P, _P, _P, _DP, ctypes.c_int, _IP, _DP]),
    "sbm_apply": (ctypes.c_int, [_P, _P, _P]),
    "sbm_residual": (ctypes.c_int, [_P, _P, _P, _DP]),
    "sbm_rhs": (ctypes.c_int, [_P, _P, _P]),
    "sbm_sensitivity": (ctypes.c_int, [_P, _P, _P, ctypes.c_double, _P, ctypes.c_int, _P]),
    "sbm_set_problem_density": (ctypes.c_int, [_P, _P, ctypes.POINTER(SbmMaterial),
                                               ctypes.POINTER(SbmBc), _P]),
    "sbm_compliance": (ctypes.c_int, [_P, _P, _DP]),
    "sbm_plastic_source": (ctypes.c_int, [_P, _P, _P]),
    "sbm_return_map": (ctypes.c_int, [_P, _P, ctypes.POINTER(SbmJ2), _P, _P, _P, _I64P]),
    "sbm_diffuse_traction": (ctypes.c_int, [_P, _P, ctypes.c_double, _P, ctypes.c_double, _P]),
    "sbm_crack_drive": (ctypes.c_int, [_P, _P, _P, _P]),
    "sbm_phase_step": (ctypes.c_int, [_P, _P, _P, _P, ctypes.POINTER(SbmPf), _P, _P]),
    "sbm_profile": (ctypes.c_int, [_P, ctypes.c_int]),
    "sbm_graph_info": (ctypes.c_int, [_P, _I64P, _I64P]),
    "sbm_residual_static": (ctypes.c_int, [ctypes.POINTER(SbmGrid), ctypes.POINTER(SbmMaterial),
                                           ctypes.POINTER(SbmBc), _P, _P, _P, _P, _DP, _P]),
    "sbm_stream_triad": (ctypes.c_int, [_P, _P, _P, ctypes.c_int64, ctypes.c_double, _P]),
    "sbm_profile_read": (ctypes.c_int, [_P, _DP, _I64P]),
    "sbm_destroy": (None, [_P]),
    "sbm_last_error": (ctypes.c_char_p, []),
    "sbm_level_shape": (ctypes.c_int, [_P, ctypes.c_int, _I64P]),
    "sbm_level_psi": (ctypes.c_int, [_P, ctypes.c_int, _P]),
    "sbm_level_apply": (ctypes.c_int, [_P, ctypes.c_int, _P, _P]),
    "sbm_level_apply_f32": (ctypes.c_int, [_P, ctypes.c_int, _P, _P]),
    "sbm_level_smooth": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_double, _P, _P,
                                        _P]),
    "sbm_level_sweep": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_double, _P, _P,
                                       _P]),
    "sbm_level_sweep_f32": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_double, _P,
                                           _P, _P]),
    "sbm_level_residual": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P]),
    "sbm_level_restrict": (ctypes.c_int, [_P, ctypes.c_int, _P, _P]),
    "sbm_level_prolong_add": (ctypes.c_int, [_P, ctypes.c_int, _P, _P]),
    "sbm_bottom_solve": (ctypes.c_int, [_P, _P, _P, _IP]),
    # block-structured adaptive composite solve; per-level pointer arrays are
    # host arrays of device pointers
    "sbm_amr_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(SbmGrid), ctypes.c_int,
                                                  ctypes.c_int, ctypes.POINTER(SbmOptions)]),
    "sbm_amr_create": (ctypes.c_int, [ctypes.POINTER(SbmGrid), ctypes.c_int, ctypes.c_int,
                                      ctypes.POINTER(SbmOptions), _P, ctypes.c_size_t, _P,
                                      ctypes.POINTER(_P)]),
    "sbm_amr_set_options": (ctypes.c_int, [_P, ctypes.POINTER(SbmOptions)]),
    "sbm_amr_set_clustering": (ctypes.c_int, [_P, ctypes.c_double]),
    "sbm_amr_cluster": (ctypes.c_int, [ctypes.c_int, _P, _P, ctypes.c_double, _P]),
    "sbm_amr_set_problem": (ctypes.c_int, [_P, ctypes.POINTER(_P), ctypes.POINTER(SbmMaterial),
                                           ctypes.POINTER(SbmBc), ctypes.c_double,
                                           ctypes.POINTER(_P)]),
    "sbm_amr_level_info": (ctypes.c_int, [_P, ctypes.c_int, _I64P, _I64P, _P, _P, _P]),
    "sbm_amr_stats": (ctypes.c_int, [_P, _I64P, _DP]),
    "sbm_amr_ghost_fill": (ctypes.c_int, [_P, ctypes.c_int, _P, _P]),
    "sbm_amr_residual": (ctypes.c_int, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), _DP]),
    "sbm_amr_solve": (ctypes.c_int, [_P, ctypes.POINTER(_P), _DP, ctypes.c_int, _IP, _DP]),
    "sbm_amr_profile": (ctypes.c_int, [_P, ctypes.c_int]),
    "sbm_amr_profile_read": (ctypes.c_int, [_P, _DP, _I64P]),
    "sbm_amr_destroy": (None, [_P]),
}

_lib = None


class SbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def lib():
    """Loads libsbm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status, allow=(SBM_OK,)):
    if status in allow:
        return status
    raise SbmError(status, lib().sbm_last_error().decode())
