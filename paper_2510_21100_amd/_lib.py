"""ctypes view of libhistretinex.so (the C ABI declared in include/histretinex.h).

Argument marshalling only: every step of the method runs in the HIP library.
Importing this module loads the library and raises if it is missing; there
is no fallback.
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhistretinex.so")

HR_OK = 0
HR_ERR_INVALID_ARG = 1
HR_ERR_UNSUPPORTED = 2
HR_ERR_WORKSPACE = 3
HR_ERR_DEVICE = 4
HR_FLAG_VALUE_CLAMPED = 0x1
HR_FLAG_HIST_MASS = 0x2
HR_NOALLOC_MAX_IMAGES = 4
HR_VARIANT_GRAD_L2 = 0x1
HR_VARIANT_GRAD_SOBEL = 0x2
HR_VARIANT_GRAD_CLIP = 0x4
HR_VARIANT_UPDATE_DIV = 0x8
HR_VARIANT_INIT_UNIFORM = 0x10
HR_VARIANT_GRAD_BITS = 0x7
HR_VARIANT_SOLVE_BITS = 0x18

#: every symbol the header declares
EXPORTS = (
    "hr_workspace_create", "hr_workspace_destroy", "hr_workspace_set_schedule", "hr_get_flags",
    "hr_build_hist", "hr_build_hist_variant", "hr_build_hist_batch", "hr_solve", "hr_match", "hr_equalize",
    "hr_enhance_batch",
    "hr_enhance_batch_noalloc",
    "hr_solve_ckpt", "hr_softmatch_loss_grad", "hr_solve_vjp",
    "hr_status_string", "hr_last_error", "hr_abi_version",
)


class HrImage(C.Structure):
    _fields_ = [("data", C.c_void_p), ("width", C.c_int32), ("height", C.c_int32),
                ("row_stride_bytes", C.c_int64)]


class HrParams(C.Structure):
    _fields_ = [("bins", C.c_int32), ("iters", C.c_int32), ("alpha", C.c_double),
                ("beta", C.c_double), ("gamma", C.c_double), ("eps", C.c_double),
                ("variant", C.c_uint32), ("reserved", C.c_int32)]


class HrSchedule(C.Structure):
    _fields_ = [("tile_steps", C.c_int32), ("wg_per_cu", C.c_int32), ("remap_steps", C.c_int32)]


class HistRetinexError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    u32p = C.POINTER(C.c_uint32)
    sig = {
        "hr_workspace_create": (C.c_int, [C.c_int32, C.c_int32, C.POINTER(P)]),
        "hr_workspace_destroy": (None, [P]),
        "hr_workspace_set_schedule": (C.c_int, [P, C.POINTER(HrSchedule)]),
        "hr_get_flags": (C.c_int, [P, u32p, C.c_int32]),
        "hr_build_hist": (C.c_int, [C.POINTER(HrImage), C.c_int32, P, P, P, P, P]),
        "hr_build_hist_variant": (C.c_int, [C.POINTER(HrImage), C.c_int32, C.c_uint32, P, P, P, P, P]),
        "hr_build_hist_batch": (C.c_int, [C.POINTER(HrImage), C.c_int32, C.c_int32, P, P, P, P]),
        "hr_solve": (C.c_int, [P, P, C.c_int64, C.POINTER(HrParams), P, P, P, P, P, P]),
        "hr_match": (C.c_int, [C.POINTER(HrImage), C.c_int32, P, P, P, C.c_int64, P, P, P]),
        "hr_equalize": (C.c_int, [C.POINTER(HrImage), C.c_int32, P, P, C.c_int64, P, P, P]),
        "hr_enhance_batch": (C.c_int, [C.POINTER(HrImage), C.POINTER(P), C.POINTER(C.c_int64), C.c_int32,
                                       C.c_int32, C.POINTER(HrParams), P, P, P, P, P, P, P]),
        "hr_enhance_batch_noalloc": (C.c_int, [C.POINTER(HrImage), C.POINTER(P), C.POINTER(C.c_int64), C.c_int32,
                                               C.c_int32, C.POINTER(HrParams), P, P, P, P, P, P, P]),
        "hr_solve_ckpt": (C.c_int, [P, P, C.c_int32, C.POINTER(HrParams), C.c_int32, P, P, P, P]),
        "hr_softmatch_loss_grad": (C.c_int, [C.POINTER(HrImage), C.POINTER(P), C.c_int32, P, P, P, P, P, P]),
        "hr_solve_vjp": (C.c_int, [P, P, C.c_int32, C.POINTER(HrParams), C.c_int32, P, P, P, P, P, P]),
        "hr_status_string": (C.c_char_p, [C.c_int]),
        "hr_last_error": (C.c_char_p, []),
        "hr_abi_version": (C.c_int32, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def check(status: int) -> None:
    if status != HR_OK:
        msg = lib.hr_last_error().decode(errors="replace")
        raise HistRetinexError(status, msg or lib.hr_status_string(status).decode())
