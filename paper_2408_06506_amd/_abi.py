"""ctypes mirror of include/tacsl.h (argument marshalling only).

The library is loaded after ``torch`` so that both share one HIP runtime in
the process.  A missing or unloadable library raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtacsl.so")

P = ctypes.c_void_p
I32 = ctypes.c_int32
I64 = ctypes.c_int64

OK = 0
STATUS_NAMES = {
    0: "TACSL_OK", -1: "TACSL_ERR_NULL_ARG", -2: "TACSL_ERR_SHAPE", -3: "TACSL_ERR_RANGE",
    -4: "TACSL_ERR_HIP", -5: "TACSL_ERR_ALLOC", -6: "TACSL_ERR_UNSUPPORTED", -7: "TACSL_ERR_STATE",
}
DEV_NONFINITE_POSE = 0x1
DEV_ZERO_QUAT = 0x2
DEV_BAD_CONTACT = 0x4
DEV_DEPTH_CAPPED = 0x8

EXPORTS = [
    "tacsl_abi_version", "tacsl_status_string", "tacsl_validate_scene", "tacsl_build_worklist",
    "tacsl_plan_create", "tacsl_plan_set_tuning", "tacsl_plan_get_info", "tacsl_plan_offsets",
    "tacsl_force_field", "tacsl_force_field_backward", "tacsl_graph_create", "tacsl_graph_launch",
    "tacsl_graph_destroy", "tacsl_plan_timer_start", "tacsl_plan_timer_read", "tacsl_plan_destroy",
    "tacsl_contact_impulse", "tacsl_plan_set_observation", "tacsl_force_field_observe",
    "tacsl_plan_set_camera", "tacsl_depth_image", "tacsl_plan_set_normal_law", "tacsl_force_field_noalloc",
    "tacsl_pose_step", "tacsl_graph_create_path",
]
MAX_OBS_BINS = 256


class SceneDesc(ctypes.Structure):
    _fields_ = [("n_env", I32), ("n_inst", I32), ("n_tmpl", I32), ("n_sdf", I32),
                ("inst_env", P), ("inst_tmpl", P), ("env_sdf", P), ("tmpl_offset", P),
                ("tmpl_xyz", P), ("sdf_dims", P), ("sdf_origin", P), ("sdf_spacing", P),
                ("sdf_offset", P), ("sdf_data", P)]


class Tuning(ctypes.Structure):
    _fields_ = [("block", I32), ("tile_taxels", I32), ("schedule", I32), ("grid", I32), ("order", I32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class PosePath(ctypes.Structure):
    _fields_ = [("pose0", P), ("twist", P), ("dt", ctypes.c_double), ("poses", P)]


class State(ctypes.Structure):
    _fields_ = [("pad_pose", P), ("obj_pose", P), ("pad_twist", P), ("obj_twist", P),
                ("params", P), ("obj_pose_delta", P)]


class Outputs(ctypes.Structure):
    _fields_ = [("depth", P), ("normal", P), ("fn", P), ("ft", P), ("wrench", P), ("status", P)]


class Grads(ctypes.Structure):
    _fields_ = [("w_fn", P), ("w_ft", P), ("g_obj_pose", P), ("g_obj_twist", P),
                ("g_params", P), ("status", P)]


class Camera(ctypes.Structure):
    _fields_ = [("rows", I32), ("cols", I32), ("ortho", I32), ("x0", ctypes.c_float), ("y0", ctypes.c_float),
                ("dx", ctypes.c_float), ("dy", ctypes.c_float), ("cam_dist", ctypes.c_float), ("gel", ctypes.c_float)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_taxels", I64), ("n_tiles", I64), ("n_env", I32), ("n_inst", I32),
                ("cu_count", I32), ("xcd_count", I32), ("prepared_bytes", I64),
                ("workspace_bytes", I64), ("tuning", Tuning)]


class TacslError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__(f"{what}: {STATUS_NAMES.get(code, code)}")


_lib = None


def load():
    """Load libtacsl.so (after torch, so both use the same HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (HIP runtime first)
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libtacsl.so not built ({LIB_PATH}); run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    for name in EXPORTS:
        getattr(lib, name)  # raises AttributeError if a symbol is missing
    lib.tacsl_abi_version.restype = ctypes.c_int
    lib.tacsl_status_string.argtypes = [ctypes.c_int]
    lib.tacsl_status_string.restype = ctypes.c_char_p
    lib.tacsl_validate_scene.argtypes = [P]
    lib.tacsl_build_worklist.argtypes = [P, P, I32, I64, P, P, P, P, P]
    lib.tacsl_plan_create.argtypes = [P, P, P]
    lib.tacsl_plan_set_tuning.argtypes = [P, P]
    lib.tacsl_plan_get_info.argtypes = [P, P]
    lib.tacsl_plan_offsets.argtypes = [P, P]
    lib.tacsl_force_field.argtypes = [P, P, P, P]
    lib.tacsl_force_field_noalloc.argtypes = [P, P, P, P]
    lib.tacsl_force_field_backward.argtypes = [P, P, P, P]
    lib.tacsl_graph_create.argtypes = [I32, P, I32, P, P, P]
    lib.tacsl_graph_create_path.argtypes = [I32, P, I32, P, P, P, P]
    lib.tacsl_pose_step.argtypes = [I32, P, P, ctypes.c_double, P, P]
    lib.tacsl_graph_launch.argtypes = [P, P]
    lib.tacsl_graph_destroy.argtypes = [P]
    lib.tacsl_plan_timer_start.argtypes = [P, I32]
    lib.tacsl_plan_timer_read.argtypes = [P, I32, P, P]
    lib.tacsl_plan_destroy.argtypes = [P]
    lib.tacsl_plan_set_observation.argtypes = [P, I32, P, P, ctypes.c_float]
    lib.tacsl_force_field_observe.argtypes = [P, P, P, P, P]
    lib.tacsl_plan_set_camera.argtypes = [P, P]
    lib.tacsl_plan_set_normal_law.argtypes = [P, ctypes.c_float]
    lib.tacsl_depth_image.argtypes = [P, P, P, P, P]
    lib.tacsl_contact_impulse.argtypes = [I64, P, P, P, P, I32, P, ctypes.c_float, P, P, P, P]
    for name in EXPORTS:
        if name not in ("tacsl_status_string",):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def check(rc, what):
    if rc != OK:
        raise TacslError(rc, what)
