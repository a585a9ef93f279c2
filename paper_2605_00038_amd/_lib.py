"""ctypes binding of the C ABI declared in include/lbp.h.

Argument marshalling only: every step of decoding runs in the HIP kernels of
``liblbp.so``.  Importing this module fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbp.so")

LBP_OK, LBP_EINVAL, LBP_ENOMEM, LBP_EDEVICE, LBP_EBUSY, LBP_ENOTREADY, LBP_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
MSG_FP32, MSG_FP16, MSG_INT8 = 0, 1, 2


def msg_fixed(x: int, y: int) -> int:
    """lbp_params.msg for fixed point Int x.y (LBP_MSG_FIXED): sign, x integer and y fraction bits."""
    return 0x100 | (x << 4) | y
SCALE_PAPER, SCALE_CONST = 0, 1
FLIP_MSG, FLIP_LLR = 0, 1
OSD_NONE, OSD_0, OSD_CS = 0, 1, 2
CN_RANDOM, CN_WORST = 0, 1
VN_PROPOSED, VN_Q_FIRST, VN_UNRELIABLE, VN_RANDOM = 0, 1, 2, 3


def lottery_rule(cn: int = CN_RANDOM, vn: int = VN_PROPOSED) -> int:
    """lbp_params.lottery_rule for a check rule and a neighbour rule (LBP_LOTTERY_RULE)."""
    return cn | (vn << 4)
FLAG_CONVERGED, FLAG_OSD, FLAG_OSD_INCONSISTENT = 1, 2, 4
NOALLOC_SCRATCH_BYTES = 128 << 20   # LBP_NOALLOC_SCRATCH_BYTES

_STATUS = {0: "LBP_OK", -1: "LBP_EINVAL", -2: "LBP_ENOMEM", -3: "LBP_EDEVICE", -4: "LBP_EBUSY",
           -5: "LBP_ENOTREADY", -6: "LBP_EUNSUPPORTED"}


class LbpError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Group(ctypes.Structure):
    """lbp_group: one group of shots of a multi-group plan (device pointers)."""
    _fields_ = [
        ("dec", ctypes.c_void_p),
        ("n_shots", ctypes.c_int64),
        ("first_shot_id", ctypes.c_uint64),
        ("syndromes", ctypes.c_void_p),
        ("corrections", ctypes.c_void_p),
        ("flags", ctypes.c_void_p),
        ("iters", ctypes.c_void_p),
    ]


PLAN_AUTOTUNE = 1


class Params(ctypes.Structure):
    _fields_ = [
        ("max_iter", ctypes.c_int32),
        ("scale_mode", ctypes.c_int32),
        ("scale", ctypes.c_float),
        ("msg", ctypes.c_int32),
        ("lottery", ctypes.c_int32),
        ("lottery_skip", ctypes.c_int32),
        ("flip", ctypes.c_int32),
        ("osd", ctypes.c_int32),
        ("osd_order", ctypes.c_int32),
        ("lottery_rule", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
    ]


# Every exported symbol with (restype, argtypes).
_VP, _I32, _I64, _U64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
SIGNATURES = {
    "lbp_params_default": (None, [ctypes.POINTER(Params)]),
    "lbp_code_create": (_I32, [_I32, _I32, _VP, _VP, _VP, ctypes.POINTER(_VP)]),
    "lbp_code_destroy": (None, [_VP]),
    "lbp_code_rows": (_I32, [_VP]),
    "lbp_code_cols": (_I32, [_VP]),
    "lbp_decoder_create": (_I32, [_VP, ctypes.POINTER(Params), _I64, ctypes.POINTER(_VP)]),
    "lbp_decoder_destroy": (None, [_VP]),
    "lbp_decode": (_I32, [_VP, _I64, _U64, _VP, _VP, _VP, _VP, _VP, _VP]),
    "lbp_decode_host": (_I32, [_VP, _I64, _U64, _VP, _VP, _VP, _VP, _VP]),
    "lbp_decoder_osd_capacity": (_I64, [_VP]),
    "lbp_decoder_set_osd_capacity": (_I32, [_VP, _I64]),
    "lbp_decoder_set_timing": (_I32, [_VP, _I32]),
    "lbp_decoder_kernel_times": (_I32, [_VP, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I64),
                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I64)]),
    "lbp_decode_keyed": (_I32, [_VP, _I64, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "lbp_decode_noalloc": (_I32, [_VP, _I64, _U64, _VP, _VP, _VP, _VP, _VP, _VP]),
    "lbp_decode_baseline": (_I32, [_VP, _I64, _U64, _VP, _VP, _VP, _VP, _VP]),
    "lbp_decoder_shape": (_I32, [_VP] + [ctypes.POINTER(_I32)] * 6),
    "lbp_decoder_device_bytes": (_I64, [_VP]),
    "lbp_decoder_max_batch": (_I64, [_VP]),
    "lbp_plan_create": (_I32, [_I32, _VP, _I32, ctypes.POINTER(_VP)]),
    "lbp_plan_launch": (_I32, [_VP, _VP]),
    "lbp_plan_info": (_I32, [_VP, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                             ctypes.POINTER(ctypes.c_double)]),
    "lbp_plan_destroy": (None, [_VP]),
    "lbp_server_create": (_I32, [_I64, _I32, ctypes.POINTER(_VP)]),
    "lbp_server_add_code": (_I32, [_VP, _VP, ctypes.POINTER(Params), ctypes.POINTER(_I32)]),
    "lbp_server_submit": (_I32, [_VP, _I32, _I64, _U64, _U64, _VP, ctypes.POINTER(_U64)]),
    "lbp_server_poll": (_I32, [_VP, _U64, _VP, _VP, _VP]),
    "lbp_server_wait": (_I32, [_VP, _U64, _I64, _VP, _VP, _VP]),
    "lbp_server_cancel": (_I32, [_VP, _U64]),
    "lbp_server_slot_info": (_I32, [_VP, _I32] + [ctypes.POINTER(_I64)] * 5),
    "lbp_server_run_load": (_I32, [_VP, _I32, _VP, _VP, _VP, _I64, _I64, ctypes.c_double, _U64, _VP, _VP,
                                   ctypes.POINTER(ctypes.c_double)]),
    "lbp_server_destroy": (None, [_VP]),
    "lbp_last_error": (ctypes.c_char_p, []),
    "lbp_version": (_I32, []),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load liblbp.so (built by paper_2605_00038_amd.build); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2605_00038_amd.build` "
                              "(there is no CPU fallback)")
        # Bind to the HIP runtime torch already carries (same SONAME): a second HIP
        # runtime in the process could not open the device.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(status: int) -> None:
    if status != LBP_OK:
        raise LbpError(status, load().lbp_last_error().decode(errors="replace"))
