"""ctypes binding of libdrr.so: same names as the C ABI in include/drr.h.

Argument marshalling only.  Device pointers are passed as integers
(``tensor.data_ptr()``), streams as the raw hipStream_t handle
(``torch.cuda.current_stream().cuda_stream``).  A missing or unloadable
library raises immediately: there is no fallback implementation.
"""

from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdrr.so")

DRR_OK = 0
DRR_EINVAL = -1
DRR_ENOMEM = -2
DRR_EHIP = -3
DRR_ENOTSUP = -4
DRR_ITEM_JAC = 1
DRR_ITEM_COUNT = 2
DRR_ITEM_NCC = 4
DRR_PLAN_PERSISTENT = 0
DRR_PLAN_FLAT = 1
DRR_PLAN_AUTO = 2
DRR_NOALLOC_SCRATCH_BYTES = 8 << 20


class DrrError(RuntimeError):
    def __init__(self, func: str, status: int, detail: str):
        super().__init__(f"{func} failed with status {status}: {detail}")
        self.status = status


class VolumeDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("spacing", ctypes.c_double * 3), ("origin", ctypes.c_double * 3),
                ("layout", ctypes.c_int32)]


class DetectorDesc(ctypes.Structure):
    _fields_ = [("height", ctypes.c_int32), ("width", ctypes.c_int32),
                ("delta_x", ctypes.c_double), ("delta_y", ctypes.c_double),
                ("offset_u", ctypes.c_double), ("offset_v", ctypes.c_double)]


class WorkItem(ctypes.Structure):
    _fields_ = [("volume", ctypes.c_int32), ("flags", ctypes.c_int32), ("det", DetectorDesc),
                ("pose", ctypes.c_void_p), ("image", ctypes.c_void_p), ("jac", ctypes.c_void_p),
                ("counts", ctypes.c_void_p), ("target", ctypes.c_void_p), ("loss", ctypes.c_void_p),
                ("grad", ctypes.c_void_p), ("partials", ctypes.c_void_p)]


class PlanDesc(ctypes.Structure):
    _fields_ = [("max_items", ctypes.c_int32), ("n_volumes", ctypes.c_int32),
                ("volumes", ctypes.POINTER(VolumeDesc)), ("packed", ctypes.POINTER(ctypes.c_void_p)),
                ("use_graph", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("tune_cache_path", ctypes.c_char_p), ("strategy", ctypes.c_int32),
                ("tile_code", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32)]


_V = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t
_F = ctypes.c_float
_VD = ctypes.POINTER(VolumeDesc)
_DD = ctypes.POINTER(DetectorDesc)

# name -> (restype, argtypes)
SIGNATURES = {
    "drr_volume_packed_bytes": (_SZ, [_VD]),
    "drr_volume_pack": (_I32, [_V, _V, _VD, _V]),
    "drr_render": (_I32, [_V, _VD, _DD, _V, _I32, _V, _V, _V]),
    "drr_render_count": (_I32, [_V, _VD, _DD, _V, _I32, _V, _V, _V]),
    "drr_render_detector_jacobian": (_I32, [_V, _VD, _DD, _V, _I32, _V, _V, _V]),
    "drr_backward_workspace_bytes": (_SZ, [_DD, _I32]),
    "drr_render_backward": (_I32, [_DD, _I32, _V, _V, _V, _V, _SZ, _V]),
    "drr_render_backward_retrace": (_I32, [_V, _VD, _DD, _V, _I32, _V, _V, _V, _SZ, _V]),
    "drr_ncc_workspace_bytes": (_SZ, [_I32, _I64]),
    "drr_ncc_forward": (_I32, [_V, _V, _I64, _I32, _I64, _V, _V, _V, _SZ, _V]),
    "drr_ncc_backward": (_I32, [_V, _V, _I64, _V, _V, _I32, _I64, _V, _V]),
    "drr_ncc_grad_workspace_bytes": (_SZ, [_DD, _I32]),
    "drr_render_ncc_grad": (_I32, [_V, _VD, _DD, _V, _I32, _V, _I64, _V, _V, _V, _V, _SZ, _V]),
    "drr_render_ncc_grad_noalloc": (_I32, [_V, _VD, _DD, _V, _I32, _V, _I64, _V, _V, _V, _V]),
    "drr_ncc_loss_workspace_bytes": (_SZ, [_DD, _I32]),
    "drr_render_ncc_loss": (_I32, [_V, _VD, _DD, _V, _I32, _V, _I64, _V, _V, _V, _SZ, _V]),
    "drr_l2_workspace_bytes": (_SZ, [_DD, _I32]),
    "drr_render_l2": (_I32, [_V, _VD, _DD, _V, _I32, _V, _I64, _V, _V, _V, _V, _SZ, _V]),
    "drr_pose_momentum_step": (_I32, [_V, _V, _V, _V, _F, _I32, _V]),
    "drr_plan_create": (_I32, [ctypes.POINTER(PlanDesc), ctypes.POINTER(WorkItem), _I32, _V,
                               ctypes.POINTER(_V)]),
    "drr_plan_execute": (_I32, [_V, ctypes.POINTER(WorkItem), _I32, _V]),
    "drr_plan_config": (_I32, [_V, ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                               ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "drr_plan_destroy": (None, [_V]),
    "drr_plan_item_workspace_bytes": (_SZ, [_DD]),
    "drr_set_launch_occupancy": (_I32, [_I32]),
    "drr_status_string": (ctypes.c_char_p, [_I32]),
    "drr_last_error": (ctypes.c_char_p, []),
    "drr_version": (_I32, []),
}

_lib = None


def load():
    """Load libdrr.so (built in-tree by paper_2208_12737_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2208_12737_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(func: str, status: int):
    if status != DRR_OK:
        detail = load().drr_last_error().decode(errors="replace")
        raise DrrError(func, status, detail)


def call(func: str, *args):
    """Call a status-returning entry point and raise DrrError on failure."""
    st = getattr(load(), func)(*args)
    check(func, st)
    return st


DRR_LAYOUT_INPUT = 0
DRR_LAYOUT_PER_AXIS = 1


def volume_desc(shape, spacing, origin, layout=DRR_LAYOUT_INPUT) -> VolumeDesc:
    d = VolumeDesc()
    d.layout = int(layout)
    d.nx, d.ny, d.nz = (int(v) for v in shape)
    for c in range(3):
        d.spacing[c] = float(spacing[c])
        d.origin[c] = float(origin[c])
    return d


def detector_desc(height, width, delta_x, delta_y, offset_u=0.0, offset_v=0.0) -> DetectorDesc:
    d = DetectorDesc()
    d.height, d.width = int(height), int(width)
    d.delta_x, d.delta_y = float(delta_x), float(delta_y)
    d.offset_u, d.offset_v = float(offset_u), float(offset_v)
    return d
