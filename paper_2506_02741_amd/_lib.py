"""ctypes binding of ``libvtgs.so`` (declared in ``include/vtgs.h``).

Argument marshalling only: every step of the renderer runs in the HIP
library.  Loading fails loudly if the library has not been built; there is
no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libvtgs.so")

VTGS_ABI_VERSION = 2  # the structures below follow this version of vtgs.h
VTGS_OK = 0
VTGS_E_ARG = -1
VTGS_E_HIP = -2
VTGS_E_WORKSPACE = -3
VTGS_E_CAPACITY = -4
VTGS_E_NONFINITE = -5
VTGS_N_STAGES = 10
VTGS_STATIC_SCRATCH_BYTES = 128 << 20


class vtgs_camera(C.Structure):
    _fields_ = [("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("width", C.c_int32), ("height", C.c_int32)]


class vtgs_keyframe(C.Structure):
    _fields_ = [("n", C.c_int32), ("pix", C.c_void_p), ("depth", C.c_void_p),
                ("color", C.c_void_p), ("opacity", C.c_void_p), ("radius", C.c_void_p),
                ("pose", C.c_void_p), ("cam", vtgs_camera), ("learnable", C.c_int32),
                ("g_color", C.c_void_p), ("g_opacity", C.c_void_p), ("g_radius", C.c_void_p),
                ("adam", C.c_void_p), ("g_depth", C.c_void_p), ("g_pose", C.c_void_p),
                ("depth_adam", C.c_void_p), ("pose_adam", C.c_void_p)]


class vtgs_view(C.Structure):
    _fields_ = [("cam", vtgs_camera), ("pose", C.c_void_p), ("kf_first", C.c_int32),
                ("kf_count", C.c_int32), ("obs_rgb", C.c_void_p), ("obs_depth", C.c_void_p),
                ("vis", C.c_void_p), ("pose_adam", C.c_void_p)]


class vtgs_frame_ref(C.Structure):
    _fields_ = [("depth", C.c_void_p), ("cam", vtgs_camera), ("pose", C.c_void_p)]


class vtgs_params(C.Structure):
    _fields_ = [("alpha_min", C.c_float), ("alpha_max", C.c_float), ("t_min", C.c_float),
                ("q_cut", C.c_float), ("z_near", C.c_float), ("lowpass", C.c_float),
                ("bg", C.c_float * 3), ("tile", C.c_int32), ("batch", C.c_int32)]


class vtgs_track_cfg(C.Structure):
    _fields_ = [("alpha", C.c_float), ("beta", C.c_float), ("lr_rot", C.c_float),
                ("lr_trans", C.c_float), ("sil_thr", C.c_float)]


class vtgs_map_cfg(C.Structure):
    _fields_ = [("rho", C.c_float), ("tau", C.c_float), ("sigma", C.c_float),
                ("lr_color", C.c_float), ("lr_opacity", C.c_float), ("lr_radius", C.c_float),
                ("lr_depth", C.c_float), ("lr_trans", C.c_float), ("lr_rot", C.c_float)]


_P = C.c_void_p
_I32 = C.c_int32
_I64 = C.c_int64
_F = C.c_float

# name -> (restype, argtypes); the same names as the C ABI
SIGNATURES = {
    "vtgs_abi_version": (_I32, []),
    "vtgs_last_error": (C.c_char_p, []),
    "vtgs_default_params": (None, [_P]),
    "vtgs_ingest_scratch_bytes": (_I64, [_I32, _I32, _I32]),
    "vtgs_ingest_count": (C.c_int, [_P, _P, _I32, _I32, _I32, _P, _I64, _P, _P]),
    "vtgs_ingest_fill": (C.c_int, [_P, _P, _P, _I32, _I32, _I32, _F, _F, _P, _I64, _I32, _P, _P,
                                   _P, _P, _P, _P]),
    "vtgs_uncovered_mask": (C.c_int, [_P, _P, _I64, _F, _P, _P]),
    "vtgs_plan_create": (C.c_int, [_P, _I32, _P, _I32, _P, _I64, _P]),
    "vtgs_plan_destroy": (None, [_P]),
    "vtgs_plan_workspace_bytes": (_I64, [_P]),
    "vtgs_plan_pixels": (_I64, [_P]),
    "vtgs_plan_view_offset": (_I64, [_P, _I32]),
    "vtgs_plan_records": (_I64, [_P]),
    "vtgs_plan_tiles": (_I64, [_P]),
    "vtgs_plan_pair_capacity": (_I64, [_P]),
    "vtgs_plan_bind": (C.c_int, [_P, _P, _I64, _P]),
    "vtgs_plan_status": (C.c_int, [_P, _P, _I32, _P]),
    "vtgs_render_fwd": (C.c_int, [_P, _P, _P, _P, _P]),
    "vtgs_render_fwd_static": (C.c_int, [_P, _P, _P, _P, _P]),
    "vtgs_render_bwd": (C.c_int, [_P, _P, _P, _P, _P, _P]),
    "vtgs_track_step": (C.c_int, [_P, _P, _I32, _P, _P]),
    "vtgs_map_step": (C.c_int, [_P, _P, _P, _P, _P]),
    "vtgs_debug_state": (C.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "vtgs_debug_images": (C.c_int, [_P, _P, _P, _P]),
    "vtgs_debug_gather": (C.c_int, [_P, _P]),
    "vtgs_visibility": (C.c_int, [_P, _P, _P, _P, _I32, _F, _F, _P, _P, _P]),
    "vtgs_stage_name": (C.c_char_p, [_I32]),
    "vtgs_plan_timing": (C.c_int, [_P, _I32, _P, _P]),
}

_lib = None


class VtgsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("vtgs error %d: %s" % (code, msg))
        self.code = code


def load():
    """Load libvtgs.so (built by ``__graft_entry__.build()``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libvtgs.so is not built (run __graft_entry__.build()); "
                              "the renderer has no fallback path")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        if L.vtgs_abi_version() != VTGS_ABI_VERSION:
            raise ImportError("libvtgs.so has ABI version %d, the binding expects %d (rebuild)"
                              % (L.vtgs_abi_version(), VTGS_ABI_VERSION))
        _lib = L
    return _lib


def last_error() -> str:
    return load().vtgs_last_error().decode()


def check(rc: int):
    if rc != VTGS_OK:
        raise VtgsError(rc, last_error())
    return rc


def default_params(**kw) -> vtgs_params:
    p = vtgs_params()
    load().vtgs_default_params(C.byref(p))
    for k, v in kw.items():
        if k == "bg":
            p.bg = (C.c_float * 3)(*v)
        else:
            setattr(p, k, v)
    return p
