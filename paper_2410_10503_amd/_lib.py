"""ctypes declarations of include/mcr.h and the loader of libmcr.so."""
from __future__ import annotations

import ctypes
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmcr.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "mcr.h")

MCR_OK, MCR_ERR_ARG, MCR_ERR_HIP, MCR_ERR_NOMEM, MCR_ERR_NONFINITE, MCR_ERR_STATE = range(6)
STATUS_NAMES = ["MCR_OK", "MCR_ERR_ARG", "MCR_ERR_HIP", "MCR_ERR_NOMEM", "MCR_ERR_NONFINITE", "MCR_ERR_STATE"]
MCR_F32, MCR_F64 = 0, 1
MOTION_IDENTITY, MOTION_RIGID, MOTION_FIELD = 0, 1, 2


class McrError(RuntimeError):
    def __init__(self, status: int, message: str):
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{name}: {message}")
        self.status = status


class Geometry(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_angles", ctypes.c_int32), ("n_det", ctypes.c_int32)]


class Motion(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("rigid", ctypes.c_double * 3), ("field", ctypes.c_void_p)]


class State(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("z", ctypes.c_void_p), ("zbar", ctypes.c_void_p),
                ("y", ctypes.POINTER(ctypes.c_void_p))]


_P = ctypes.c_void_p
_I = ctypes.c_int32
_D = ctypes.c_double
_PD = ctypes.POINTER(ctypes.c_double)
_PI = ctypes.POINTER(ctypes.c_int32)
_PP = ctypes.POINTER(ctypes.c_void_p)

SIGNATURES = {
    "mcr_create": [ctypes.POINTER(Geometry), _I, ctypes.POINTER(Motion), _I, _P, ctypes.POINTER(_P)],
    "mcr_destroy": [_P],
    "mcr_set_stream": [_P, _P],
    "mcr_set_motion": [_P, _I, ctypes.POINTER(Motion)],
    "mcr_set_rigid_params": [_P, _PD],
    "mcr_get_info": [_P, ctypes.POINTER(Geometry), _PI, _PI, _PI],
    "mcr_warp": [_P, _I, _P, _P],
    "mcr_warp_adjoint": [_P, _I, _P, _P],
    "mcr_project": [_P, _P, _P],
    "mcr_backproject": [_P, _P, _P],
    "mcr_apply_Ai": [_P, _I, _P, _P],
    "mcr_apply_Ai_adjoint": [_P, _I, _P, _P],
    "mcr_spdhg_iterate": [_P, ctypes.POINTER(State), _PP, _D, _PD, _D, _D, _PD, _PI, _I],
    "mcr_spdhg_epoch": [_P, ctypes.POINTER(State), _PP, _D, _PD, _D, _D, _PD, _PI],
    "mcr_pdhg_epoch": [_P, ctypes.POINTER(State), _PP, _D, _PD, _D, _D],
    "mcr_power_norm_sq": [_P, _I, _P, _I, _D, _PD, _PI],
    "mcr_objective": [_P, _P, _PP, _D, _PD],
    "mcr_duality_gap": [_P, ctypes.POINTER(State), _PP, _D, _PD],
    "mcr_step_sizes": [_I, _I, _PD, _D, _PD, _PD, _PD, _PD],
    "mcr_set_subsets": [_P, _I],
    "mcr_set_subset_partition": [_P, _I, _I],
    "mcr_block_norm_sq": [_P, _I, _I, _P, _I, _D, _PD, _PI],
    "mcr_spdhg_blocks_iterate": [_P, ctypes.POINTER(State), _PP, _D, _PD, _D, _D, _PD, _PI, _I],
    "mcr_step_sizes_blocks": [_I, _I, _PD, _D, _PD, _PD, _PD, _PD],
    "mcr_spdhg_iterate_ckpt": [_P, ctypes.POINTER(State), _PP, _D, _PD, _D, _D, _PD, _PI, _I, _PP, _PP, _PP],
    "mcr_spdhg_step_backward": [_P, _I, _P, _P, _P, _D, _D, _D, _D, _D, _P, _P, _P, _P, _P, _P],
    "mcr_warp_motion_grad": [_P, _I, _P, _P, _P],
    "mcr_register_rigid": [_P, _I, _P, _P, _PD, _I, _D, _PD, _PI],
    "mcr_register_affine": [_P, _I, _P, _P, _PD, _I, _D, _PD, _PI],
    "mcr_register_field": [_P, _I, _P, _P, _P, _D, _PD, _I, _I, _D, _PD, _PI],
    "mcr_batch_create": [ctypes.POINTER(Geometry), _I, _PI, ctypes.POINTER(Motion), _I, _P, ctypes.POINTER(_P)],
    "mcr_batch_spdhg_epoch": [_P, _P, _P, _P, _P, _P, _PD, _PD, _PD, _PD, _PD, _PI, _I],
    "mcr_profile_enable": [_P, _I],
    "mcr_autotune": [_P, _I, _PI, _PI, _PI],
    "mcr_set_variant": [_P, _I, _I, _I],
    "mcr_profile_read": [_P, _PD, ctypes.POINTER(ctypes.c_int64)],
    "mcr_project_noalloc": [ctypes.POINTER(Geometry), _P, _P, _P],
}
KERNEL_CLASSES = ["warp", "project", "backproject", "twarp", "xstep", "other"]

_lib = None


def load() -> ctypes.CDLL:
    """Loads libmcr.so from the package directory (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2410_10503_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, args in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.mcr_last_error.argtypes = []
    lib.mcr_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != MCR_OK:
        msg = load().mcr_last_error()
        raise McrError(status, msg.decode() if msg else "")


def header_functions() -> list[str]:
    """Names of the functions declared in include/mcr.h."""
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(mcr_[A-Za-z0-9_]+)\s*\(", text)))
