"""ctypes view of libmechstep.so (the C ABI in include/mechstep.h).

Loading imports torch first so that the process holds a single HIP runtime
(torch's).  There is no fallback: if the library is missing or does not load,
this module raises.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (load torch's HIP runtime before ours)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmechstep.so")

MS_OK, MS_EINVAL, MS_ECAPACITY, MS_EDEVICE, MS_EINPUT = 0, 1, 2, 3, 4
MS_F32, MS_F64, MS_F32_POS64 = 0, 1, 2
MS_BOX_ORDER_AUTO, MS_BOX_ORDER_ROWS, MS_BOX_ORDER_TILES = 0, 1, 2
MS_WALK_LANES, MS_WALK_PLANES = 0, 1
STATUS_NAMES = {0: "MS_OK", 1: "MS_EINVAL", 2: "MS_ECAPACITY", 3: "MS_EDEVICE", 4: "MS_EINPUT"}

EXPORTS = (
    "ms_workspace_bytes", "ms_workspace_init", "ms_grid_build", "ms_mech_step",
    "ms_mech_step_backward", "ms_grid_build_batched", "ms_mech_step_batched",
    "ms_mech_step_backward_batched", "ms_mech_step_integrate", "ms_mech_step_batched_integrate",
    "ms_mech_step_backward_accumulate", "ms_mech_step_backward_batched_accumulate",
    "ms_mech_step_integrate_sorted", "ms_mech_step_batched_integrate_sorted",
    "ms_integrate", "ms_reorder", "ms_grid_get", "ms_neighbors",
    "ms_device_status", "ms_copy_probe", "ms_last_error", "ms_mech_step_noalloc",
)
# capacities of ms_mech_step_noalloc's static workspace (mechstep.h)
NOALLOC_MAX_AGENTS = 65536
NOALLOC_MAX_BOXES = 524288


class ms_params(ctypes.Structure):
    _fields_ = [("kappa", ctypes.c_double), ("gamma", ctypes.c_double), ("dt", ctypes.c_double),
                ("max_disp", ctypes.c_double), ("adherence", ctypes.c_double)]


class ms_grid_info(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_double * 3), ("edge", ctypes.c_double),
                ("dims", ctypes.c_int32 * 3), ("error", ctypes.c_int32),
                ("n_boxes", ctypes.c_int64), ("box_base", ctypes.c_int64),
                ("n_agents", ctypes.c_int64), ("tile_shift", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class ms_workspace(ctypes.Structure):
    _fields_ = [("base", ctypes.c_void_p), ("bytes", ctypes.c_size_t),
                ("max_agents", ctypes.c_int64), ("max_boxes", ctypes.c_int64),
                ("max_sims", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("n_agents", ctypes.c_int64), ("n_sims", ctypes.c_int32),
                ("built", ctypes.c_int32), ("keep_forces", ctypes.c_int32),
                ("gather_list", ctypes.c_int32), ("gather_block", ctypes.c_int32),
                ("sorted_input", ctypes.c_int32), ("box_order", ctypes.c_int32),
                ("gather_walk", ctypes.c_int32)]


class MechStepError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load():
    """Load and type the library (once)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2105_00039_amd.build` "
                          "(the HIP extension is required, there is no fallback)")
    L = ctypes.CDLL(LIB_PATH)
    P, I64, I32, D, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
    WS = ctypes.POINTER(ms_workspace)
    PAR = ctypes.POINTER(ms_params)
    sig = {
        "ms_workspace_bytes": (SZ, [I64, I64, I32, ctypes.c_int]),
        "ms_workspace_init": (ctypes.c_int, [WS, P, SZ, I64, I64, I32, ctypes.c_int, P]),
        "ms_grid_build": (ctypes.c_int, [WS, P, P, P, P, I64, D, P]),
        "ms_mech_step": (ctypes.c_int, [WS, PAR, P, P, P, P]),
        "ms_mech_step_backward": (ctypes.c_int, [WS, PAR, P, P, P, P, P, P, P, P, P]),
        "ms_grid_build_batched": (ctypes.c_int, [WS, P, P, P, P, P, I32, I64, P, P]),
        "ms_mech_step_batched": (ctypes.c_int, [WS, P, P, P, P, P]),
        "ms_mech_step_backward_batched": (ctypes.c_int, [WS, P, P, P, P, P, P, P, P, P, P]),
        "ms_mech_step_backward_accumulate": (ctypes.c_int, [WS, PAR, P, P, P, P, P, P]),
        "ms_mech_step_backward_batched_accumulate": (ctypes.c_int, [WS, P, P, P, P, P, P, P]),
        "ms_mech_step_integrate": (ctypes.c_int, [WS, PAR, P, P, P, P, P, P, P]),
        "ms_mech_step_integrate_sorted": (ctypes.c_int, [WS, PAR] + [P] * 12),
        "ms_mech_step_batched_integrate_sorted": (ctypes.c_int, [WS, P] + [P] * 12),
        "ms_mech_step_batched_integrate": (ctypes.c_int, [WS, P, P, P, P, P, P, P, P]),
        "ms_integrate": (ctypes.c_int, [P, P, P, P, P, P, I64, ctypes.c_int, P]),
        "ms_reorder": (ctypes.c_int, [WS, P, P, I32, P]),
        "ms_grid_get": (ctypes.c_int, [WS, ctypes.POINTER(ms_grid_info), P, P, P, P]),
        "ms_neighbors": (ctypes.c_int, [WS, P, P, P, I64, ctypes.POINTER(ctypes.c_int64), P]),
        "ms_device_status": (ctypes.c_int, [WS, P]),
        "ms_copy_probe": (ctypes.c_int, [P, P, SZ, P]),
        "ms_mech_step_noalloc": (ctypes.c_int, [P, P, P, P, I64, ctypes.c_int, D, PAR, P, P, P, P, P]),
        "ms_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def check(status: int):
    if status != MS_OK:
        msg = load().ms_last_error().decode(errors="replace")
        raise MechStepError(status, msg)
