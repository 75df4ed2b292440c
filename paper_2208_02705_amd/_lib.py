"""ctypes binding of libr360.so (the C ABI in include/r360.h).

Argument marshalling only: every step of the path runs in the library's
HIP kernels. Loading fails loudly when the library has not been built; there
is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libr360.so")

R360_OK, R360_EINVAL, R360_ENOMEM, R360_EHIP, R360_EUNSUPPORTED, R360_EWORKSPACE = 0, -1, -2, -3, -4, -5
FP32, BF16, FP16, FP64_GRADCHECK = 0, 1, 2, 3
PRECISIONS = {"fp32": FP32, "bf16": BF16, "fp16": FP16, "fp64": FP64_GRADCHECK}
NSTAGES = 9
STAGES = ["sample", "route", "mlp_forward", "composite", "loss", "composite_backward", "mlp_backward",
          "global_field", "occupancy"]


class GridDesc(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("lo", C.c_float * 3), ("voxel", C.c_float), ("threshold", C.c_float)]


class MlpDesc(C.Structure):
    _fields_ = [("n_fields", C.c_int32), ("hidden", C.c_int32), ("L_xyz", C.c_int32), ("L_dir", C.c_int32),
                ("center", C.c_float * 3), ("half_extent", C.c_float)]


class RenderOpts(C.Structure):
    _fields_ = [("near_", C.c_float), ("far_", C.c_float), ("max_samples", C.c_int32), ("precision", C.c_int32),
                ("samples_per_voxel", C.c_int32), ("term_eps", C.c_float), ("term_after", C.c_int32)]


class GlobalDesc(C.Structure):
    _fields_ = [("width", C.c_int32), ("color_width", C.c_int32), ("n_samples", C.c_int32), ("near_", C.c_float),
                ("far_", C.c_float), ("center", C.c_float * 3), ("half_extent", C.c_float),
                ("grid_n", C.c_int32 * 3), ("grid_lo", C.c_float * 3), ("voxel", C.c_float)]


class OccDesc(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("lo", C.c_float * 3), ("voxel", C.c_float), ("near_", C.c_float),
                ("far_", C.c_float), ("l_hit", C.c_float), ("l_miss", C.c_float), ("l_min", C.c_float),
                ("l_max", C.c_float), ("min_opacity", C.c_float)]


class R360Error(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"r360 status {status}: {msg}")
        self.status = status


vp, i32, i64, f32, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_size_t
F12 = C.POINTER(C.c_float)

SIGNATURES = {
    "r360_field_params": (i64, [i32, i32, i32]),
    "r360_scene_create": (i32, [C.POINTER(GridDesc), vp, vp, C.POINTER(MlpDesc), vp, vp, C.POINTER(vp)]),
    "r360_scene_set_weights": (i32, [vp, vp, vp]),
    "r360_scene_set_grid": (i32, [vp, vp, vp, vp]),
    "r360_scene_destroy": (None, [vp]),
    "r360_field_frames_workspace_bytes": (sz, [i32]),
    "r360_field_frames": (i32, [C.POINTER(GridDesc), vp, i32, vp, vp, vp, sz, vp]),
    "r360_scene_set_frames": (i32, [vp, vp, vp, vp]),
    "r360_equirect_create": (i32, [i32, i32, C.POINTER(vp)]),
    "r360_equirect_destroy": (None, [vp]),
    "r360_equirect_tables": (i32, [vp, vp, vp, vp, vp]),
    "r360_equirect_rays": (i32, [vp, F12, vp, i64, vp, vp, vp]),
    "r360_ods_rays": (i32, [vp, F12, f32, vp, i64, vp, vp, vp]),
    "r360_render_ods": (i32, [vp, vp, F12, f32, C.POINTER(RenderOpts), vp, vp, vp, vp, sz, vp]),
    "r360_pinhole_rays": (i32, [i32, i32, f32, f32, F12, vp, vp, vp]),
    "r360_lr_schedule": (C.c_double, [i64, i64, C.c_double, C.c_double]),
    "r360_occ_desc_init": (i32, [C.POINTER(OccDesc), i32, f32, f32, f32, f32, C.c_double, C.c_double, f32, f32,
                                 f32]),
    "r360_workspace_bytes": (sz, [vp, i64, i32]),
    "r360_sample_rays": (i32, [vp, vp, vp, i64, C.POINTER(RenderOpts), C.POINTER(i64), vp, vp, vp, vp, vp, vp, vp, sz, vp]),
    "r360_render_rays": (i32, [vp, vp, vp, i64, C.POINTER(RenderOpts), vp, vp, vp, vp, sz, vp]),
    "r360_render_rays_noalloc": (i32, [vp, vp, vp, i64, C.POINTER(RenderOpts), vp, vp, vp, vp]),
    "r360_render_equirect": (i32, [vp, vp, F12, C.POINTER(RenderOpts), vp, vp, vp, vp, sz, vp]),
    "r360_render_pinhole": (i32, [vp, i32, i32, f32, f32, F12, C.POINTER(RenderOpts), vp, vp, vp, vp, sz, vp]),
    "r360_backward": (i32, [vp, vp, vp, i64, C.POINTER(RenderOpts), vp, vp, vp, sz, vp]),
    "r360_train_step": (i32, [vp, vp, vp, i64, vp, C.POINTER(RenderOpts), vp, vp, vp, vp, sz, vp]),
    "r360_adam_step": (i32, [vp, vp, vp, vp, i64, i64, f32, f32, f32, f32, vp]),
    "r360_gradcheck_forward": (i32, [vp, vp, vp, vp, i64, C.POINTER(RenderOpts), vp, vp, sz, vp]),
    "r360_gradcheck_backward": (i32, [vp, vp, vp, vp, i64, C.POINTER(RenderOpts), vp, vp, vp, sz, vp]),
    "r360_global_params": (i64, [i32, i32]),
    "r360_global_workspace_bytes": (sz, [C.POINTER(GlobalDesc), i64]),
    "r360_global_field_step": (i32, [C.POINTER(GlobalDesc), vp, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, sz, vp]),
    "r360_depth_uncertainty": (i32, [vp, vp, vp, i64, i32, vp, vp, vp, vp]),
    "r360_occupancy_workspace_bytes": (sz, [C.POINTER(OccDesc)]),
    "r360_occupancy_update": (i32, [C.POINTER(OccDesc), vp, vp, vp, vp, i64, vp, vp, vp, vp, sz, vp]),
    "r360_global_field_measure": (i32, [C.POINTER(GlobalDesc), vp, vp, vp, i64, vp, vp, vp, vp, sz, vp]),
    "r360_global_points_workspace_bytes": (sz, [C.POINTER(GlobalDesc), i64]),
    "r360_global_field_points": (i32, [C.POINTER(GlobalDesc), vp, vp, vp, i64, vp, vp, vp, sz, vp]),
    "r360_distill_step": (i32, [vp, vp, vp, vp, i64, vp, vp, C.POINTER(RenderOpts), vp, vp, vp, sz, vp]),
    "r360_assign_workspace_bytes": (sz, [vp]),
    "r360_assign_fields": (i32, [vp, vp, f32, i32, vp, C.POINTER(i64), vp, sz, vp]),
    "r360_assign_uniform_workspace_bytes": (sz, [vp]),
    "r360_assign_uniform": (i32, [vp, vp, f32, vp, vp, C.POINTER(i32), vp, sz, vp]),
    "r360_profile_enable": (i32, [i32]),
    "r360_profile_read": (i32, [vp, vp]),
    "r360_status_string": (C.c_char_p, [i32]),
    "r360_last_error": (C.c_char_p, []),
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it first (python -m paper_2208_02705_amd.build)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int):
    if status != R360_OK:
        L = lib()
        raise R360Error(status, f"{L.r360_status_string(status).decode()}: {L.r360_last_error().decode()}")


def c2w_arg(c2w) -> "C.Array":
    vals = [float(x) for x in c2w]
    if len(vals) != 12:
        raise ValueError("c2w must hold 12 floats (row-major 3x4)")
    return (C.c_float * 12)(*vals)
