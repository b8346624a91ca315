"""ctypes declarations of the C ABI in include/mlbm.h.

Loading fails loudly if the in-tree library has not been built; there is no
fallback implementation.  The environment variable MLBM_LIBRARY may name
another build of the same library (the tests use a build whose host code is
compiled with AddressSanitizer and UndefinedBehaviorSanitizer).
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MLBM_LIBRARY") or os.path.join(HERE, "lib", "libmlbm.so")

# enums mirrored from include/mlbm.h
D2Q9, D3Q19, D3Q27 = 0, 1, 2
F64, F32, F16S = 0, 1, 2
FACE = {"periodic": 0, "eq": 1, "copy": 2, "wall": 3}
NBR_MISSING, NBR_BOUNCE, NBR_EQ, NBR_COPY = -1, -2, -3, -4
E_ARG, E_MESH, E_STATE, E_HIP, E_OOM = -1, -2, -3, -4, -5
DIAG_MASS, DIAG_KE, DIAG_FORCE = 1, 2, 4
STATUS_NONFINITE, STATUS_F16_OVERFLOW, STATUS_GRAPH_FALLBACK = 1, 2, 4
TABLE_TREEID, TABLE_COORDS, TABLE_NBR, TABLE_GFC_SRC, TABLE_GFF_SRC, \
    TABLE_CAPTURE, TABLE_BOUNCE, TABLE_NBR16, TABLE_NBASE, TABLE_NBR_WIDE, \
    TABLE_NBR_HDR, TABLE_WALL, TABLE_WALL_Q = range(13)
STATE_PDF_POST, STATE_MOMENTS, STATE_PDF_PRE, STATE_STRAIN, STATE_PDF_PREV = range(5)
INFO_FIELDS = ("level", "n", "n_fluid", "n_gfc_inner", "n_gfc_outer", "n_gff",
               "n_cap_fluid", "n_cap", "n_gfc_groups", "n_bounce", "n_wall")

_p = C.c_void_p
_i32, _i64, _u32, _sz = C.c_int32, C.c_int64, C.c_uint32, C.c_size_t
_pi32, _pi64, _pu64 = C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_uint64)
_pd, _pu32, _psz = C.POINTER(C.c_double), C.POINTER(C.c_uint32), C.POINTER(C.c_size_t)

# name: (restype, argtypes)
SIGNATURES = {
    "mlbm_error_string": (C.c_char_p, [_i32]),
    "mlbm_last_error": (C.c_char_p, []),
    "mlbm_lattice": (_i32, [_i32, _pi32, _pi32, _pd]),
    "mlbm_plan_create": (_i32, [_i32, _i32, _pi32, _pi32, _pi32, _pu64, _i64, _pu64, _i64,
                                C.POINTER(_p)]),
    "mlbm_plan_destroy": (None, [_p]),
    "mlbm_set_morton_policy": (_i32, [C.c_double, _i32]),
    "mlbm_plan_set_walls": (_i32, [_p, _pu64, _pi32, _pd, _i64]),
    "mlbm_set_gfc_layers": (_i32, [_i32]),
    "mlbm_plan_gfc_layers": (_i32, [_p, _pi32]),
    "mlbm_plan_levels": (_i32, [_p, _pi32, _pi32]),
    "mlbm_plan_level_info": (_i32, [_p, _i32, _pi64]),
    "mlbm_plan_export": (_i32, [_p, _i32, _i32, _p, _psz]),
    "mlbm_sim_workspace_bytes": (_i32, [_p, _i32, _psz]),
    "mlbm_sim_create": (_i32, [_p, _i32, C.c_double, C.c_double, _pd, _pi32, _p, _p, _sz,
                               C.POINTER(_p)]),
    "mlbm_sim_destroy": (None, [_p]),
    "mlbm_init": (_i32, [_p, _i32, _p, _p, _p]),
    "mlbm_fill_ghosts": (_i32, [_p]),
    "mlbm_step": (_i32, [_p, _i64]),
    "mlbm_diagnostics": (_i32, [_p, _u32, _p]),
    "mlbm_diagnostics_noalloc": (_i32, [_p, _u32, _p]),
    "mlbm_get_state": (_i32, [_p, _i32, _i32, _p]),
    "mlbm_set_state": (_i32, [_p, _i32, _i32, _p]),
    "mlbm_status": (_i32, [_p, _pu32]),
    "mlbm_time": (_i32, [_p, _pi64]),
    "mlbm_checkpoint_bytes": (_i32, [_p, _psz]),
    "mlbm_save_checkpoint": (_i32, [_p, _p, _sz]),
    "mlbm_load_checkpoint": (_i32, [_p, _p, _sz]),
    "mlbm_launches_per_step": (_i32, [_p, _pi64]),
    "mlbm_profile": (_i32, [_p, _i32]),
    "mlbm_use_graphs": (_i32, [_p, _i32]),
    "mlbm_profile_read": (_i32, [_p, _i32, _pd, _pi64, _pi64]),
    "mlbm_profile_read_kind": (_i32, [_p, _i32, _i32, _pd, _pi64, _pi64]),
    "mlbm_adjoint_workspace_bytes": (_i32, [_p, _p, _psz]),
    "mlbm_adjoint_attach": (_i32, [_p, _p, _p, _sz]),
    "mlbm_adjoint_seed": (_i32, [_p, _i32]),
    "mlbm_adjoint_step": (_i32, [_p, _p, _sz]),
    "mlbm_adjoint_init": (_i32, [_p, C.POINTER(_p), C.POINTER(_p), C.POINTER(_p),
                                 C.POINTER(_p), C.POINTER(_p), C.POINTER(_p)]),
    "mlbm_adjoint_params": (_i32, [_p, _pd, _pd, _pd]),
    "mlbm_adjoint_get_lambda": (_i32, [_p, _i32, _p]),
}
OBJ_KE, OBJ_DRAG_X = 0, 1

_LIB = None


class MLBMError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{message} (code {code})")
        self.code = code


def lib():
    """The loaded library; raises if it is missing (never falls back)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "paper_1601_06984_amd/build.py first")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def check(code: int):
    if code != 0:
        msg = lib().mlbm_last_error().decode(errors="replace")
        raise MLBMError(code, msg or lib().mlbm_error_string(code).decode())
    return code
