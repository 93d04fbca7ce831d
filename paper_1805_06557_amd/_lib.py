"""ctypes loader for librexi_swe.so with the argument types of every entry
point declared in include/rexi_swe.h.  Loading fails loudly when the library
has not been built; there is no fallback implementation."""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librexi_swe.so")

_c_int, _c_double, _vp = ctypes.c_int, ctypes.c_double, ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


class RexiMember(ctypes.Structure):
    """rexi_member of include/rexi_swe.h."""
    _fields_ = [("ctx", _vp), ("alpha", _dp), ("beta", _dp), ("N", _c_int), ("dt", _c_double),
                ("U0", _vp), ("U1", _vp)]


# name -> (restype, argtypes); the stream argument is a hipStream_t (void*).
SIGNATURES = {
    "rexi_coefficients": (_c_int, [_c_int, _c_int, _c_double, _c_double, _dp, _dp, _dp, _dp]),
    "rexi_check_contour": (_c_int, [_c_int, _c_double, _c_double, _c_double, _c_double, _c_double, _dp, _dp,
                                    _c_int, _dp]),
    "rexi_spectral_radius": (_c_int, [_c_int, _c_double, _c_double, _c_double, _c_double, _c_double, _dp]),
    "rexi_contour_error": (_c_int, [_dp, _dp, _c_int, _c_double, _c_int, _dp, _dp]),
    "rexi_choose_contour": (_c_int, [_c_double, _c_double, _c_int, _c_int, _dp, _c_int, _c_int, _dp, _dp, _ip,
                                     _dp]),
    "swe_create": (_c_int, [_c_int, _c_int, _c_int, _c_double, _c_double, _c_double, _c_double, _c_int,
                            ctypes.POINTER(_vp)]),
    "swe_destroy": (_c_int, [_vp]),
    "rexi_linear_step": (_c_int, [_vp, _dp, _dp, _c_int, _c_double, _vp, _vp, _vp]),
    "rexi_lg_step": (_c_int, [_vp, _dp, _dp, _c_int, _c_double, _vp, _vp, _vp]),
    "rexi_lg_step_noalloc": (_c_int, [_vp, _dp, _dp, _c_int, _c_double, _vp, _vp, _vp]),
    "sh_synthesis": (_c_int, [_vp, _vp, _vp, _c_int, _vp]),
    "sh_analysis": (_c_int, [_vp, _vp, _vp, _c_int, _vp]),
    "swe_nonlinear_step": (_c_int, [_vp, _c_double, _vp, _vp, _vp]),
    "swe_strang_step": (_c_int, [_vp, _dp, _dp, _c_int, _c_double, _vp, _vp, _vp]),
    "swe_strang_steps": (_c_int, [_vp, _dp, _dp, _c_int, _c_double, _c_int, _vp, _vp, _vp]),
    "swe_etdrk2_step": (_c_int, [_vp, _dp, _dp, _dp, _dp, _c_int, _c_double, _vp, _vp, _vp]),
    "swe_cn_step": (_c_int, [_vp, _c_double, _vp, _vp, _vp]),
    "swe_split_step": (_c_int, [_vp, _c_int, _dp, _dp, _c_int, _c_double, _vp, _vp, _vp]),
    "swe_sync": (_c_int, [_vp]),
    "rexi_last_error": (ctypes.c_char_p, []),
    "swe_set_tuning": (_c_int, [_vp, _c_int, _c_int, _c_int, _c_int]),
    "swe_get_tuning": (_c_int, [_vp, _ip, _ip, _ip, _ip]),
    "swe_set_fusion": (_c_int, [_vp, _c_int]),
    "swe_get_fusion": (_c_int, [_vp, _ip]),
    "swe_autotune": (_c_int, [_vp, _dp, _dp, _c_int, _c_double, _vp, _vp, _c_int, _vp, _dp]),
    "rexi_linear_step_batched": (_c_int, [ctypes.POINTER(RexiMember), _c_int, _vp]),
    "swe_profile": (_c_int, [_vp, _c_int]),
    "swe_profile_kernels": (_c_int, [_vp, ctypes.c_uint]),
    "swe_profile_read": (_c_int, [_vp, _c_int, _dp, ctypes.POINTER(_c_int)]),
}

_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1805_06557_amd.build` "
                "(there is no CPU fallback)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib
