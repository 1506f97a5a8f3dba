"""ctypes declarations of the C ABI in ``include/lbf.h``.

Loading fails loudly when ``liblbf.so`` has not been built: there is no
fallback path."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbf.so")

OK, EINVAL, ENOMEM, EHIP, ENOTCONV, EDIVERGED, ESTATE = 0, -1, -2, -3, -4, -5, -6


class LbfParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("real_bytes", ctypes.c_int), ("nspecies", ctypes.c_int),
        ("reaction_mode", ctypes.c_int),
        ("tau_f", ctypes.c_double), ("u0", ctypes.c_double),
        ("tau_g", ctypes.c_double), ("c_in", ctypes.c_double),
        ("vel_scale", ctypes.c_double),
        ("flux_col", ctypes.c_int), ("tile_x", ctypes.c_int), ("tile_y", ctypes.c_int),
        ("variant", ctypes.c_int), ("flags", ctypes.c_int),
        ("boundary", ctypes.c_int),
    ]


class Lbf3Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("real_bytes", ctypes.c_int), ("nspecies", ctypes.c_int),
        ("tau_f", ctypes.c_double), ("force_x", ctypes.c_double),
        ("tau_g", ctypes.c_double), ("c_in", ctypes.c_double),
        ("vel_scale", ctypes.c_double),
        ("flux_col", ctypes.c_int), ("tile_x", ctypes.c_int), ("tile_y", ctypes.c_int),
        ("flags", ctypes.c_int),
    ]


class LbfRwParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nspecies", ctypes.c_int),
        ("xf", ctypes.c_int), ("wall_mode", ctypes.c_int),
        ("D", ctypes.c_double), ("dt", ctypes.c_double), ("zone", ctypes.c_double),
        ("rate_w", ctypes.c_double), ("density", ctypes.c_double),
        ("vel_scale", ctypes.c_double), ("seed", ctypes.c_uint64), ("capacity", ctypes.c_long),
    ]


# name -> (restype, argtypes)
_P, _I, _L, _D, _S = ctypes.c_void_p, ctypes.c_int, ctypes.c_long, ctypes.c_double, ctypes.c_size_t
_PP = ctypes.POINTER(LbfParams)
_PD = ctypes.POINTER(ctypes.c_double)
_PL = ctypes.POINTER(ctypes.c_long)
_PS = ctypes.POINTER(ctypes.c_size_t)
SIGNATURES = {
    "lbf_params_default": (_I, [_PP, _I, _I]),
    "lbf_create": (_I, [_PP, ctypes.POINTER(_P)]),
    "lbf_workspace_bytes": (_I, [_P, _PS]),
    "lbf_bind": (_I, [_P, _P, _S, _P]),
    "lbf_set_geometry": (_I, [_P, _P]),
    "lbf_set_rates": (_I, [_P, _P]),
    "lbf_flow_init": (_I, [_P]),
    "lbf_flow_run": (_I, [_P, _L]),
    "lbf_flow_steady": (_I, [_P, _L, _I, _D, _PL, _PD]),
    "lbf_get_velocity": (_I, [_P, _P, _P]),
    "lbf_set_velocity": (_I, [_P, _P, _P]),
    "lbf_adr_init": (_I, [_P]),
    "lbf_adr_run": (_I, [_P, _L, _I, _D, _PL]),
    "lbf_efficiency": (_I, [_P, _PD, _PD, _PD]),
    "lbf_get_concentration": (_I, [_P, _I, _P]),
    "lbf_adr_totals": (_I, [_P, _PD]),
    "lbf_adr_production": (_I, [_P, _PD]),
    "lbf_adr_steps": (_I, [_P, _PL]),
    "lbf_adjoint_workspace_bytes": (_I, [_P, _L, _I, _I, _PS]),
    "lbf_adr_adjoint": (_I, [_P, _L, _I, _I, _P, _S, _PD, _P]),
    "lbf_adr_adjoint_steady": (_I, [_P, _L, _I, _D, _P, _S, _PD, _P, _PL]),
    "lbf_state_bytes": (_I, [_P, _PS]),
    "lbf_get_state": (_I, [_P, _P]),
    "lbf_set_state": (_I, [_P, _P]),
    "lbf_prepare_adr_steps": (_I, [_P, _L]),
    "lbf_efficiency_noalloc": (_I, [_PP, _P, _P, _P, _PD, _PD, _PD]),
    "lbf_time_adr_steps": (_I, [_P, _L, _PD]),
    "lbf_time_flow_steps": (_I, [_P, _L, _PD]),
    "lbf_status_str": (ctypes.c_char_p, [_I]),
    "lbf_last_error": (ctypes.c_char_p, [_P]),
    "lbf_destroy": (None, [_P]),
    "lbf_version": (_I, []),
    "lbf_probe_copy": (_I, [_P, _P, _S, _P, _PD]),
    "lbf_batch_create": (_I, [_I, _PP, ctypes.POINTER(_P)]),
    "lbf_batch_workspace_bytes": (_I, [_P, _PS]),
    "lbf_batch_bind": (_I, [_P, _P, _S, _P]),
    "lbf_batch_set_geometry": (_I, [_P, _P, _P]),
    "lbf_batch_flow": (_I, [_P, _L, _I, _D]),
    "lbf_batch_run": (_I, [_P, _L, _I, _D, _PD, _PD, _PL]),
    "lbf_batch_resume": (_I, [_P, _L, _I, _D, _PD, _PD, _PL]),
    "lbf_batch_get_concentration": (_I, [_P, _I, _I, _P]),
    "lbf_batch_time_steps": (_I, [_P, _L, _PD]),
    "lbf_batch_last_error": (ctypes.c_char_p, [_P]),
    "lbf_batch_destroy": (None, [_P]),
    # 3D path (include/lbf3d.h)
    "lbf3_params_default": (_I, [ctypes.POINTER(Lbf3Params), _I, _I, _I]),
    "lbf3_create": (_I, [ctypes.POINTER(Lbf3Params), ctypes.POINTER(_P)]),
    "lbf3_workspace_bytes": (_I, [_P, _PS]),
    "lbf3_bind": (_I, [_P, _P, _S, _P]),
    "lbf3_set_geometry": (_I, [_P, _P]),
    "lbf3_set_rates": (_I, [_P, _P]),
    "lbf3_flow_init": (_I, [_P]),
    "lbf3_flow_run": (_I, [_P, _L]),
    "lbf3_flow_steady": (_I, [_P, _L, _I, _D, _PL, _PD]),
    "lbf3_get_velocity": (_I, [_P, _P, _P, _P]),
    "lbf3_set_velocity": (_I, [_P, _P, _P, _P]),
    "lbf3_adr_init": (_I, [_P]),
    "lbf3_adr_run": (_I, [_P, _L, _I, _D, _PL]),
    "lbf3_efficiency": (_I, [_P, _PD, _PD, _PD]),
    "lbf3_get_concentration": (_I, [_P, _I, _P]),
    "lbf3_adr_totals": (_I, [_P, _PD]),
    "lbf3_time_adr_steps": (_I, [_P, _L, _PD]),
    "lbf3_time_flow_steps": (_I, [_P, _L, _PD]),
    "lbf3_last_error": (ctypes.c_char_p, [_P]),
    "lbf3_destroy": (None, [_P]),
    # random-walk tracker (include/lbf_rw.h)
    "lbf_rw_params_default": (_I, [ctypes.POINTER(LbfRwParams), _I, _I]),
    "lbf_rw_create": (_I, [ctypes.POINTER(LbfRwParams), ctypes.POINTER(_P)]),
    "lbf_rw_workspace_bytes": (_I, [_P, _PS]),
    "lbf_rw_bind": (_I, [_P, _P, _S, _P]),
    "lbf_rw_set_fields": (_I, [_P, _P, _P, _P, _P]),
    "lbf_rw_fill": (_I, [_P]),
    "lbf_rw_run": (_I, [_P, _L, _I]),
    "lbf_rw_counts": (_I, [_P, _PD, _PL, _PL]),
    "lbf_rw_walk": (_I, [_P, _L, _P, _P, _P, _P, _L, _L]),
    "lbf_rw_time_steps": (_I, [_P, _L, _I, _PD]),
    "lbf_rw_last_error": (ctypes.c_char_p, [_P]),
    "lbf_rw_destroy": (None, [_P]),
}

_lib = None


def load():
    """Load ``liblbf.so`` and declare every entry point."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with "
                "`python -c 'import __graft_entry__ as g; g.build()'` (or "
                "paper_2109_04455_amd/build.py); there is no non-HIP fallback")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib
