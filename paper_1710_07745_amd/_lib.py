"""ctypes loader for libcanny.so (the HIP library built in-tree).

Only argument marshalling lives here.  If the shared library is missing the
first call raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcanny.so")
_lib = None

CANNY_OK = 0
CANNY_ERR_INVALID = 1
CANNY_ERR_WORKSPACE = 2
CANNY_ERR_HIP = 3
CANNY_ERR_UNSUPPORTED = 4
CANNY_ERR_TOO_LARGE = 5
CANNY_NOALLOC_SCRATCH_BYTES = 32 << 20  # include/canny.h

P = C.c_void_p
i32 = C.c_int32
i64 = C.c_int64
sz = C.c_size_t
f32 = C.c_float

# name -> (restype, argtypes); mirrors include/canny.h
SIGNATURES = {
    "canny_status_string": (C.c_char_p, [C.c_int]),
    "canny_abi_version": (C.c_int, []),
    "canny_class_pitch": (i64, [C.c_int]),
    "canny_u8_workspace_bytes": (sz, [C.c_int, C.c_int]),
    "canny_u8": (C.c_int, [P, i64, C.c_int, C.c_int, i32, i32, P, i64, P, P, sz, P]),
    "canny_u8_noalloc": (C.c_int, [P, i64, C.c_int, C.c_int, i32, i32, P, i64, P, P]),
    "canny_log_u8": (C.c_int, [P, i64, C.c_int, C.c_int, i32, P, i64, P, i64, P]),
    "canny_hysteresis_workspace_bytes": (sz, [C.c_int, C.c_int]),
    "canny_hysteresis": (C.c_int, [P, C.c_int, C.c_int, P, i64, P, sz, P]),
    "canny_f32_workspace_bytes": (sz, [C.c_int, C.c_int]),
    "canny_f32": (C.c_int, [P, i64, C.c_int, C.c_int, f32, C.c_int, f32, f32, C.c_int, P, i64, P,
                            P, P, P, sz, P]),
    "canny_f32_sector": (C.c_int, [P, i64, C.c_int, C.c_int, f32, C.c_int, f32, f32, P, i64, P, P,
                                   P, sz, P]),
    "canny_batch_plan_create": (C.c_int, [C.c_int, P, P, i32, i32, C.c_int, C.POINTER(P)]),
    "canny_batch_workspace_bytes": (sz, [P]),
    "canny_batch": (C.c_int, [P, P, P, P, P, P, sz, P]),
    "canny_batch_plan_info": (C.c_int, [P, P, P]),
    "canny_batch_plan_destroy": (None, [P]),
    "canny_video_create": (C.c_int, [C.c_int, C.c_int, i32, i32, C.c_int, C.POINTER(P)]),
    "canny_video_push": (C.c_int, [P, P, P]),
    "canny_video_sync": (C.c_int, [P]),
    "canny_video_destroy": (None, [P]),
    "canny_mag_forward": (C.c_int, [P, P, C.c_int, C.c_int, C.c_int, C.c_int, P, P]),
    "canny_mag_backward_workspace_bytes": (sz, [C.c_int, C.c_int, C.c_int, C.c_int]),
    "canny_mag_backward": (C.c_int, [P, P, P, C.c_int, C.c_int, C.c_int, C.c_int, P, P, P, sz, P]),
    "canny_timing_begin": (C.c_int, [C.c_int]),
    "canny_timing_read": (C.c_int, [C.c_int, C.POINTER(C.c_double), C.POINTER(i64)]),
    "canny_timing_end": (C.c_int, []),
}

# stage ids of canny_timing_read (include/canny.h)
STAGES = {"u8_forward": 0, "f32_clear": 1, "f32_walk": 2, "f32_classify": 3, "hysteresis": 4,
          "mag_forward": 5, "mag_backward": 6}


class CannyError(RuntimeError):
    def __init__(self, fn: str, status: int):
        super().__init__(f"{fn} failed: {status_string(status)} (status {status})")
        self.status = status


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libcanny.so not built ({LIB_PATH}); run __graft_entry__.build()")
        l = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(l, name, None)
            if f is None:
                continue
            f.restype = res
            f.argtypes = args
        _lib = l
    return _lib


def status_string(status: int) -> str:
    return lib().canny_status_string(int(status)).decode()


def check(fn: str, status: int) -> None:
    if status != CANNY_OK:
        raise CannyError(fn, status)
