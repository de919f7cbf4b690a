"""ctypes declarations of libsoftshadow.so (the C ABI in include/softshadow.h)."""
from __future__ import annotations

import ctypes as C
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsoftshadow.so")

SS_OK = 0
SS_ERR_INVALID_ARG = -1
SS_ERR_HIP = -2
SS_ERR_WORKSPACE = -3
SS_ERR_UNSUPPORTED = -4
SS_NOALLOC_SCRATCH_BYTES = 2 << 20
SS_MODE_DP = 0
SS_MODE_UNIFORM = 1
SS_MODE_EXACT = 2
SS_MODE_POINT = 3
SS_SCHED_GEOMETRIC = 0
SS_SCHED_EQUAL = 1
SS_SCHED_LIST = 2
SS_VIEW_HIER = 0
SS_VIEW_DENSE = 1
RAY_TILES = {"8x8": 1, "16x4": 2, "4x16": 3, "32x2": 4}


class SSSun(C.Structure):
    _fields_ = [("elev_rad", C.c_double), ("azim_rad", C.c_double), ("ang_radius_rad", C.c_double)]


class SSParams(C.Structure):
    _fields_ = [("body_radius_m", C.c_double), ("max_len_m", C.c_double), ("n_prime0", C.c_int32),
                ("schedule", C.c_int32), ("n_segments", C.c_int32), ("mode", C.c_int32),
                ("uniform_step", C.c_double), ("prune", C.c_int32), ("ray_tile", C.c_int32),
                ("n_prime_list", C.c_int32 * 16)]


class SSTile(C.Structure):
    _fields_ = [("height", C.c_void_p), ("maxmip", C.c_void_p), ("width", C.c_int32),
                ("rows", C.c_int32), ("texel_m", C.c_double), ("bound", C.c_void_p),
                ("ray_x0", C.c_int32), ("ray_y0", C.c_int32), ("ray_w", C.c_int32),
                ("ray_h", C.c_int32)]


class SSCamera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("eye_m", C.c_double * 3),
                ("fwd", C.c_double * 3), ("right", C.c_double * 3), ("up", C.c_double * 3),
                ("step_m", C.c_double), ("far_m", C.c_double), ("mode", C.c_int32)]


class SSFrame(C.Structure):
    _fields_ = [("width", C.c_int32), ("rows", C.c_int32), ("texel_m", C.c_double),
                ("centre", C.c_double * 3), ("ex", C.c_double * 3), ("ey", C.c_double * 3),
                ("origin_m", C.c_double * 2)]


# Every exported symbol with (restype, argtypes); the CPU tests check that this
# list matches include/softshadow.h.
SIGNATURES = {
    "ss_maxmip_levels": (C.c_int32, [C.c_int32, C.c_int32]),
    "ss_maxmip_level_offset": (C.c_int64, [C.c_int32, C.c_int32, C.c_int32]),
    "ss_maxmip_floats": (C.c_int64, [C.c_int32, C.c_int32]),
    "ss_maxmip_build": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_int32,
                                    C.c_void_p]),
    "ss_bound_floats": (C.c_int64, [C.c_int32, C.c_int32]),
    "ss_bound_level_offset": (C.c_int64, [C.c_int32, C.c_int32, C.c_int32]),
    "ss_bound_build": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]),
    "ss_shadow_cast": (C.c_int32, [C.POINTER(SSTile), C.POINTER(SSSun), C.POINTER(SSParams),
                                   C.c_void_p, C.c_void_p]),
    "ss_shadow_cast_counted": (C.c_int32, [C.POINTER(SSTile), C.POINTER(SSSun),
                                           C.POINTER(SSParams), C.c_void_p, C.c_void_p,
                                           C.c_void_p]),
    "ss_shadow_cast_backward": (C.c_int32, [C.POINTER(SSTile), C.POINTER(SSSun),
                                            C.POINTER(SSParams), C.c_void_p, C.c_void_p,
                                            C.c_void_p, C.c_void_p]),
    "ss_shadow_cast_backward_penumbra": (C.c_int32, [C.POINTER(SSTile), C.POINTER(SSSun),
                                                     C.POINTER(SSParams), C.c_void_p, C.c_void_p,
                                                     C.c_void_p, C.c_void_p, C.c_void_p]),
    "ss_shadow_cast_save": (C.c_int32, [C.POINTER(SSTile), C.POINTER(SSSun), C.POINTER(SSParams),
                                        C.c_void_p, C.c_void_p, C.c_void_p]),
    "ss_shadow_cast_backward_saved": (C.c_int32, [C.POINTER(SSTile), C.POINTER(SSSun),
                                                  C.POINTER(SSParams), C.c_void_p, C.c_void_p,
                                                  C.c_void_p, C.c_void_p, C.c_void_p]),
    "ss_batched_workspace_bytes": (C.c_int64, [C.c_int32, C.c_int32]),
    "ss_shadow_cast_batched": (C.c_int32, [C.POINTER(SSTile), C.c_int32, C.POINTER(SSSun),
                                           C.c_int32, C.POINTER(SSParams), C.c_void_p, C.c_void_p,
                                           C.c_int64, C.c_void_p]),
    "ss_shadow_cast_batched_noalloc": (C.c_int32, [C.POINTER(SSTile), C.c_int32,
                                                   C.POINTER(SSSun), C.c_int32,
                                                   C.POINTER(SSParams), C.c_void_p, C.c_void_p]),
    "ss_batched_plan_create": (C.c_int32, [C.POINTER(SSTile), C.c_int32, C.POINTER(SSSun),
                                           C.c_int32, C.POINTER(SSParams), C.c_void_p, C.c_void_p,
                                           C.c_int64, C.c_void_p, C.POINTER(C.c_void_p)]),
    "ss_batched_plan_launch": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "ss_batched_plan_config": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32),
                                           C.POINTER(C.c_int32)]),
    "ss_batched_plan_destroy": (C.c_int32, [C.c_void_p]),
    "ss_shadow_points": (C.c_int32, [C.POINTER(SSTile), C.POINTER(SSSun), C.POINTER(SSParams),
                                     C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "ss_shadow_points_backward": (C.c_int32, [C.POINTER(SSTile), C.POINTER(SSSun),
                                              C.POINTER(SSParams), C.c_void_p, C.c_int64,
                                              C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                              C.c_void_p]),
    "ss_shadow_points_image": (C.c_int32, [C.POINTER(SSTile), C.POINTER(SSSun), C.POINTER(SSParams),
                                           C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                                           C.c_void_p]),
    "ss_view_cast": (C.c_int32, [C.POINTER(SSTile), C.c_double, C.POINTER(SSCamera), C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_void_p]),
    "ss_resample": (C.c_int32, [C.c_void_p, C.POINTER(SSFrame), C.c_void_p, C.POINTER(SSFrame),
                                C.c_double, C.c_void_p]),
    "ss_probe_gather": (C.c_int32, [C.c_void_p, C.c_int64, C.c_int64, C.c_int32, C.c_void_p,
                                    C.c_int64, C.c_void_p]),
    "ss_probe_gather_tiles": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                          C.c_void_p, C.c_int64, C.c_void_p]),
    "ss_probe_valu": (C.c_int32, [C.c_int32, C.c_int64, C.c_void_p, C.c_void_p]),
    "ss_status_string": (C.c_char_p, [C.c_int32]),
}

_lock = threading.Lock()
_lib = None


class SoftShadowError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn} failed: {msg} ({status})")
        self.status = status


def lib() -> C.CDLL:
    """The loaded HIP library; raises if it has not been built (no fallback)."""
    global _lib
    with _lock:
        if _lib is None:
            how = ("build it with `python -c 'import __graft_entry__ as g; g.build()'` or "
                   "`python paper_2005_06671_amd/build.py`")
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"{LIB_PATH} is missing: {how}")
            from . import build as _build
            try:
                with open(_build.HASH_FILE) as f:
                    built = f.read().strip()
            except OSError:
                built = ""
            if built != _build.source_hash():
                raise ImportError(f"{LIB_PATH} was built from other sources than the ones next "
                                  f"to it (stale): {how}")
            L = C.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
            _lib = L
        return _lib


def check(fn: str, status: int) -> None:
    if status != SS_OK:
        msg = lib().ss_status_string(status).decode()
        raise SoftShadowError(fn, status, msg)
