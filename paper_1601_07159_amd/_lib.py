"""ctypes declarations of libace's C ABI (include/ace.h).  Marshalling only."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libace.so")

(ACE_OK, ACE_E_ARG, ACE_E_NOT_PD, ACE_E_NOMEM, ACE_E_HIP, ACE_E_UNSUPPORTED,
 ACE_E_CAPTURE) = range(7)
ACE_FP64, ACE_FP32, ACE_MIXED, ACE_REAL64, ACE_REAL32 = 0, 1, 2, 3, 4
ACE_COULOMB, ACE_ERFC = 0, 1

EXPORTED = [
    "ace_create", "ace_destroy", "ace_set_stream", "ace_reserve", "ace_build_W", "ace_compress",
    "ace_apply", "ace_apply_noalloc", "ace_exchange_energy", "ace_exchange_energy_grad", "ace_orthonormalize",
    "ace_supported_n", "ace_build_W_batched", "ace_autotune", "ace_tune_load",
    "ace_profile_enable", "ace_profile_reset", "ace_profile_count", "ace_profile_get",
    "ace_set_pair_budget", "ace_set_tuning", "ace_get_tuning", "ace_status_string",
    "ace_last_error", "ace_apply_h", "ace_combine", "ace_rayleigh_ritz",
]
(ACE_TUNE_PAIR_BUDGET, ACE_TUNE_JBLOCK, ACE_TUNE_SYMMETRY, ACE_TUNE_FFT_SHAPE,
 ACE_TUNE_ACCUM_SHAPE, ACE_TUNE_BRANCHES, ACE_TUNE_BATCH_FORM) = 0, 1, 2, 3, 4, 5, 6


class AceGrid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("L", ctypes.c_double * 3), ("kind", ctypes.c_int),
                ("mu", ctypes.c_double), ("g0", ctypes.c_double)]


class AceInstance(ctypes.Structure):
    _fields_ = [("grid", AceGrid), ("prec", ctypes.c_int),
                ("phi", ctypes.c_void_p), ("n_occ", ctypes.c_int), ("ld_phi", ctypes.c_long),
                ("psi", ctypes.c_void_p), ("n_band", ctypes.c_int), ("ld_psi", ctypes.c_long),
                ("W", ctypes.c_void_p), ("ld_W", ctypes.c_long),
                ("xi", ctypes.c_void_p), ("ld_xi", ctypes.c_long),
                ("info_dev", ctypes.c_void_p), ("scale", ctypes.c_double)]


_vp = ctypes.c_void_p
_i = ctypes.c_int
_l = ctypes.c_long
_d = ctypes.c_double
_gp = ctypes.POINTER(AceGrid)

_PROTOS = {
    "ace_create": (_i, [ctypes.POINTER(_vp), _vp, ctypes.c_char_p]),
    "ace_destroy": (_i, [_vp]),
    "ace_set_stream": (_i, [_vp, _vp]),
    "ace_reserve": (_i, [_vp, _gp, _i, _i, _i, _i]),
    "ace_build_W": (_i, [_vp, _gp, _i, _vp, _i, _l, _vp, _i, _l, _vp, _l, _d]),
    "ace_compress": (_i, [_vp, _gp, _i, _vp, _l, _vp, _l, _i, _vp, _l, _vp, _vp]),
    "ace_apply": (_i, [_vp, _gp, _i, _vp, _i, _l, _vp, _i, _l, _vp, _l]),
    "ace_apply_noalloc": (_i, [_vp, _gp, _i, _vp, _i, _l, _vp, _i, _l, _vp, _l]),
    "ace_exchange_energy": (_i, [_vp, _gp, _i, _vp, _i, _l, _vp, _i, _l, _vp]),
    "ace_exchange_energy_grad": (_i, [_vp, _gp, _i, _vp, _i, _l, _vp, _vp, _l]),
    "ace_orthonormalize": (_i, [_vp, _gp, _i, _vp, _i, _l, _vp, _l, _vp]),
    "ace_supported_n": (_i, [ctypes.POINTER(_i), _i]),
    "ace_build_W_batched": (_i, [_vp, _i, ctypes.POINTER(AceInstance)]),
    "ace_autotune": (_i, [_vp, _gp, _i, _i, _i, ctypes.c_char_p, ctypes.POINTER(_l),
                          ctypes.POINTER(_l), ctypes.POINTER(_i), ctypes.POINTER(_i),
                          ctypes.POINTER(_d)]),
    "ace_tune_load": (_i, [_vp, ctypes.c_char_p]),
    "ace_profile_enable": (_i, [_vp, _i]),
    "ace_profile_reset": (_i, [_vp]),
    "ace_profile_count": (_i, [_vp]),
    "ace_profile_get": (_i, [_vp, _i, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(_l),
                             ctypes.POINTER(_d)]),
    "ace_set_pair_budget": (_i, [_vp, _l]),
    "ace_set_tuning": (_i, [_vp, _i, _l]),
    "ace_get_tuning": (_i, [_vp, _i, ctypes.POINTER(_l)]),
    "ace_apply_h": (_i, [_vp, _gp, _i, _vp, _vp, _i, _l, _vp, _i, _l, _d, _vp, _i, _l, _vp, _l]),
    "ace_combine": (_i, [_vp, _gp, _i, _i, _d, _vp, _l, _d, _vp, _l, _d, _vp, _l, _vp, _l]),
    "ace_rayleigh_ritz": (_i, [_vp, _gp, _i, _vp, _l, _vp, _l, _i, _vp, _vp, _l, _vp]),
    "ace_status_string": (ctypes.c_char_p, [_i]),
    "ace_last_error": (ctypes.c_char_p, [_vp]),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load the built library; raises if it has not been built (there is no
    fallback implementation)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libace.so not found at {LIB_PATH}; build it with "
                          "`python -m paper_1601_07159_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _PROTOS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
