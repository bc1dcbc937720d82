"""ctypes declarations of the C interface in include/syk.h.

Loads paper_2002_05725_amd/libsyk.so (built by build.py).  There is no
fallback: if the library is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsyk.so")

SYK_OK, SYK_EINVAL, SYK_ENOMEM, SYK_EHIP, SYK_EBREAKDOWN, SYK_ENOTCONVERGED, SYK_EUNSUPPORTED = range(7)
SYK_C128, SYK_C64 = 0, 1
STATUS_NAMES = {0: "SYK_OK", 1: "SYK_EINVAL", 2: "SYK_ENOMEM", 3: "SYK_EHIP", 4: "SYK_EBREAKDOWN",
                5: "SYK_ENOTCONVERGED", 6: "SYK_EUNSUPPORTED"}


class KrylovOpts(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int), ("dt", ctypes.c_double), ("tau_step", ctypes.c_double),
                ("tol", ctypes.c_double)]


class ChebOpts(ctypes.Structure):
    _fields_ = [("degree", ctypes.c_int), ("dt", ctypes.c_double), ("tau_steps", ctypes.c_int),
                ("checkpoint_every", ctypes.c_int), ("e_center", ctypes.c_double),
                ("e_halfwidth", ctypes.c_double), ("keep_segment", ctypes.c_int)]


class SykError(RuntimeError):
    def __init__(self, status: int, fn: str, msg: str):
        super().__init__(f"{fn}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None

_vp = ctypes.c_void_p
_i = ctypes.c_int
_i64 = ctypes.c_int64
_d = ctypes.c_double
_SIGS = {
    "syk_last_error": (ctypes.c_char_p, []),
    "syk_version": (_i, []),
    "syk_build_terms": (_i, [_i, _i, _vp, ctypes.POINTER(_vp)]),
    "syk_destroy_terms": (_i, [_vp]),
    "syk_terms_info": (_i, [_vp, ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i64),
                            ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    "syk_apply_H": (_i, [_vp, _i, _i, _vp, _vp, _vp, _vp]),
    "syk_apply_H_noalloc": (_i, [_vp, _i, _i, _vp, _vp, _vp, _vp]),
    "syk_set_apply_tuning": (_i, [_vp, _i, _i, _i]),
    "syk_set_workspace_limit": (_i, [_vp, ctypes.c_uint64]),
    "syk_timing_enable": (_i, [_i]),
    "syk_timing_read": (_i, [ctypes.POINTER(_i64), ctypes.POINTER(_d)]),
    "syk_timing_reset": (_i, []),
    "syk_apply_majorana": (_i, [_vp, _i, _i, _i, _vp, _vp, _vp]),
    "syk_dot": (_i, [_i, _i64, _i, _vp, _vp, _vp, _vp]),
    "syk_krylov_expmv": (_i, [_vp, _i, _i, _vp, _d, _d, _d, ctypes.POINTER(KrylovOpts), _vp, _vp, _vp]),
    "syk_two_point": (_i, [_vp, _i, _i, _d, _vp, _i, _i, _vp, _vp, ctypes.POINTER(KrylovOpts), _vp, _vp, _vp]),
    "syk_apply_H_sector": (_i, [_vp, _i, _i, _i, _vp, _vp, _vp, _vp]),
    "syk_apply_majorana_sector": (_i, [_vp, _i, _i, _i, _i, _vp, _vp, _vp]),
    "syk_krylov_expmv_sector": (_i, [_vp, _i, _i, _i, _vp, _d, _d, _d, ctypes.POINTER(KrylovOpts), _vp, _vp, _vp]),
    "syk_two_point_sector": (_i, [_vp, _i, _i, _i, _d, _vp, _i, _i, _vp, _vp, ctypes.POINTER(KrylovOpts), _vp, _vp,
                                  _vp]),
    "syk_otoc_sector": (_i, [_vp, _i, _i, _i, _i, _d, _vp, _i, _i, _vp, _vp, ctypes.POINTER(KrylovOpts), _vp, _vp,
                             _vp, _vp]),
    "syk_otoc_unregularized_sector": (_i, [_vp, _i, _i, _i, _i, _d, _vp, _i, _i, _vp, _vp, ctypes.POINTER(KrylovOpts),
                                           _vp, _vp, _vp, _vp]),
    "syk_imag_two_point_sector": (_i, [_vp, _i, _i, _i, _d, _vp, _i, _i, _vp, _vp, ctypes.POINTER(KrylovOpts), _vp,
                                       _vp, _vp]),
    "syk_lowest_eigenvalues": (_i, [_vp, _i, _i, _i, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_int), _vp]),
    "syk_otoc_unregularized": (_i, [_vp, _i, _i, _i, _d, _vp, _i, _i, _vp, _vp, ctypes.POINTER(KrylovOpts), _vp,
                                    _vp, _vp, _vp]),
    "syk_imag_two_point": (_i, [_vp, _i, _i, _d, _vp, _i, _i, _vp, _vp, ctypes.POINTER(KrylovOpts), _vp, _vp, _vp]),
    "syk_otoc": (_i, [_vp, _i, _i, _i, _d, _vp, _i, _i, _vp, _vp, ctypes.POINTER(KrylovOpts), _vp, _vp, _vp,
                      _vp]),
    "syk_spectrum_bounds": (_i, [_vp, _i, _i, _vp, ctypes.POINTER(_d), ctypes.POINTER(_d), _vp]),
    "syk_cheb_otoc": (_i, [_vp, _i, _i, _d, _d, ctypes.POINTER(ChebOpts), _vp, ctypes.POINTER(_d), _vp]),
    "syk_grad_couplings": (_i, [_vp, _i, _i, _d, _d, ctypes.POINTER(ChebOpts), _vp, ctypes.POINTER(_d), _vp, _vp]),
    "syk_coupling_overlaps": (_i, [_vp, _i, _vp, _vp, _vp, _vp, _vp]),
}


def lib():
    """The loaded library; raises if libsyk.so is absent (no CPU fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run __graft_entry__.build() or python paper_2002_05725_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def declared_symbols():
    return list(_SIGS)


def check(status: int, fn: str):
    if status != SYK_OK:
        raise SykError(status, fn, lib().syk_last_error().decode())
