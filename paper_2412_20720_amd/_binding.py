"""ctypes binding of libg4d.so: the C ABI of include/g4d.h, same names, argument marshalling only.

Loading fails loudly (RuntimeError) when the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libg4d.so")

G4D_OK, G4D_EINVAL, G4D_ENOMEM, G4D_ECAPACITY, G4D_EHIP, G4D_ESTATE = 0, -1, -2, -3, -4, -5
G4D_RECORD_FLOATS = 12
STATUS_NAMES = {0: "G4D_OK", -1: "G4D_EINVAL", -2: "G4D_ENOMEM", -3: "G4D_ECAPACITY",
                -4: "G4D_EHIP", -5: "G4D_ESTATE"}

EXPORTED = ["g4d_default_settings", "g4d_create", "g4d_destroy", "g4d_last_error",
            "g4d_preprocess", "g4d_render_forward", "g4d_render_backward", "g4d_sync_status",
            "g4d_get_stats", "g4d_eval_counters", "g4d_autotune", "g4d_profile",
            "g4d_stage_name", "g4d_render_step", "g4d_render_channels_forward",
            "g4d_render_channels_backward", "g4d_render_sky_forward", "g4d_render_sky_backward",
            "g4d_decode_compact", "g4d_render_compact_forward", "g4d_profile_mask",
            "g4d_get_pairs", "g4d_render_step_noalloc"]
G4D_STEP_GRAPH = 1
G4D_NOALLOC_SCRATCH_BYTES = 64 << 20
G4D_NUM_STAGES = 8
G4D_MAX_CHANNELS = 36


class g4d_gaussians(C.Structure):
    _fields_ = [("n", C.c_int32), ("sh_degree", C.c_int32), ("t_degree", C.c_int32),
                ("mean4", C.c_void_p), ("scale4", C.c_void_p), ("rot_l", C.c_void_p),
                ("rot_r", C.c_void_p), ("opacity", C.c_void_p), ("sh", C.c_void_p),
                ("mask", C.c_void_p), ("mask_threshold", C.c_float)]


class g4d_grads(C.Structure):
    _fields_ = [("mean4", C.c_void_p), ("scale4", C.c_void_p), ("rot_l", C.c_void_p),
                ("rot_r", C.c_void_p), ("opacity", C.c_void_p), ("sh", C.c_void_p),
                ("mask", C.c_void_p), ("densify", C.c_void_p)]


class g4d_view(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("world_to_cam", C.c_float * 12),
                ("t", C.c_float), ("background", C.c_float * 3)]


class g4d_settings(C.Structure):
    _fields_ = [("near_z", C.c_float), ("marginal_min", C.c_float), ("cutoff_sigma", C.c_float),
                ("blur", C.c_float), ("jacobian_margin", C.c_float), ("alpha_min", C.c_float),
                ("alpha_max", C.c_float), ("T_min", C.c_float), ("color_offset", C.c_float),
                ("color_min", C.c_float), ("time_period", C.c_float), ("tile_size", C.c_int32),
                ("lds_batch", C.c_int32), ("px_per_lane", C.c_int32),
                ("bwd_px_per_lane", C.c_int32)]


class g4d_channels(C.Structure):
    _fields_ = [("n_features", C.c_int32), ("features", C.c_void_p), ("gate", C.c_void_p),
                ("depth", C.c_int32), ("flow", C.c_int32), ("flow_dt", C.c_float)]


class g4d_sky(C.Structure):
    _fields_ = [("cube", C.c_void_p), ("resolution", C.c_int32)]


class g4d_compact(C.Structure):
    _fields_ = [("n", C.c_int32), ("sh_degree", C.c_int32), ("t_degree", C.c_int32),
                ("mean4_h", C.c_void_p), ("scale_idx", C.c_void_p), ("rot_l_idx", C.c_void_p),
                ("rot_r_idx", C.c_void_p), ("opacity_q", C.c_void_p), ("dc_idx", C.c_void_p),
                ("rest_idx", C.c_void_p), ("opacity_lo", C.c_float), ("opacity_hi", C.c_float),
                ("scale_cb", C.c_void_p), ("rot_cb", C.c_void_p), ("dc_cb", C.c_void_p),
                ("rest_cb", C.c_void_p)]


class g4d_stats(C.Structure):
    _fields_ = [("n_slots", C.c_int64), ("n_visible", C.c_int64), ("n_pairs", C.c_int64),
                ("n_tiles", C.c_int64), ("n_pixels", C.c_int64), ("pair_capacity", C.c_int64),
                ("n_clamped_batches", C.c_int64)]


_lib: Optional[C.CDLL] = None


def lib() -> C.CDLL:
    """Load libg4d.so once; raise if it is missing (build it with __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first "
                           "(the HIP library is required, there is no CPU path)")
    L = C.CDLL(LIB_PATH)
    vp, i32 = C.c_void_p, C.c_int32
    L.g4d_default_settings.argtypes = [C.POINTER(g4d_settings)]
    L.g4d_create.argtypes = [C.POINTER(vp), C.c_int]
    L.g4d_destroy.argtypes = [vp]
    L.g4d_last_error.argtypes = [vp]
    L.g4d_last_error.restype = C.c_char_p
    L.g4d_preprocess.argtypes = [vp, C.POINTER(g4d_gaussians), C.POINTER(g4d_view), i32,
                                 C.POINTER(g4d_settings), vp, vp, vp]
    L.g4d_render_forward.argtypes = [vp, C.POINTER(g4d_gaussians), C.POINTER(g4d_view), i32,
                                     C.POINTER(g4d_settings), vp, vp, vp]
    L.g4d_render_backward.argtypes = [vp, C.POINTER(g4d_gaussians), C.POINTER(g4d_view), i32,
                                      C.POINTER(g4d_settings), vp, C.POINTER(g4d_grads), vp]
    L.g4d_sync_status.argtypes = [vp, vp]
    L.g4d_get_stats.argtypes = [vp, C.POINTER(g4d_stats), vp]
    L.g4d_get_pairs.argtypes = [vp, vp, vp, vp, vp]
    L.g4d_eval_counters.argtypes = [vp, C.c_int, vp, vp]
    L.g4d_render_step.argtypes = [vp, C.POINTER(g4d_gaussians), C.POINTER(g4d_view), i32,
                                  C.POINTER(g4d_settings), vp, vp, vp, C.POINTER(g4d_grads), i32,
                                  vp]
    L.g4d_render_step_noalloc.argtypes = [vp, C.POINTER(g4d_gaussians), C.POINTER(g4d_view), i32,
                                          C.POINTER(g4d_settings), vp, vp, vp,
                                          C.POINTER(g4d_grads), vp]
    L.g4d_autotune.argtypes = [vp, C.POINTER(g4d_gaussians), C.POINTER(g4d_view), i32,
                               C.POINTER(g4d_settings), vp, vp, vp, C.POINTER(g4d_grads), i32,
                               C.POINTER(C.c_double), vp]
    L.g4d_render_channels_forward.argtypes = [vp, C.POINTER(g4d_gaussians), C.POINTER(g4d_view),
                                              i32, C.POINTER(g4d_settings),
                                              C.POINTER(g4d_channels), vp, vp, vp, vp]
    L.g4d_render_channels_backward.argtypes = [vp, C.POINTER(g4d_gaussians), C.POINTER(g4d_view),
                                               i32, C.POINTER(g4d_settings),
                                               C.POINTER(g4d_channels), vp, vp,
                                               C.POINTER(g4d_grads), vp, vp, vp]
    L.g4d_render_sky_forward.argtypes = [vp, C.POINTER(g4d_gaussians), C.POINTER(g4d_view), i32,
                                         C.POINTER(g4d_settings), C.POINTER(g4d_sky), vp, vp, vp]
    L.g4d_render_sky_backward.argtypes = [vp, C.POINTER(g4d_gaussians), C.POINTER(g4d_view), i32,
                                          C.POINTER(g4d_settings), C.POINTER(g4d_sky), vp,
                                          C.POINTER(g4d_grads), vp, vp]
    L.g4d_decode_compact.argtypes = [vp, C.POINTER(g4d_compact), vp, vp, vp, vp, vp, vp, vp]
    L.g4d_render_compact_forward.argtypes = [vp, C.POINTER(g4d_compact), C.POINTER(g4d_view), i32,
                                             C.POINTER(g4d_settings), vp, vp, vp]
    L.g4d_profile.argtypes = [vp, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int]
    L.g4d_profile_mask.argtypes = [vp, C.c_uint32]
    L.g4d_stage_name.argtypes = [C.c_int]
    L.g4d_stage_name.restype = C.c_char_p
    for name in EXPORTED:
        if name not in ("g4d_last_error", "g4d_stage_name"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


class G4DError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def check(status: int, ctx=None) -> None:
    if status != G4D_OK:
        msg = lib().g4d_last_error(ctx).decode() if ctx else ""
        raise G4DError(status, msg)


def default_settings(**overrides) -> g4d_settings:
    s = g4d_settings()
    check(lib().g4d_default_settings(C.byref(s)))
    for k, v in overrides.items():
        if not hasattr(s, k):
            raise KeyError(k)
        setattr(s, k, v)
    return s


def make_views(views) -> C.Array:
    """Array of g4d_view from a list of dicts (see paper_2412_20720_amd.scenes)."""
    arr = (g4d_view * len(views))()
    for i, v in enumerate(views):
        w2c = [float(x) for x in __import__("numpy").asarray(v["world_to_cam"], "float32").ravel()]
        bg = [float(x) for x in __import__("numpy").asarray(v.get("background", (0, 0, 0)), "float32").ravel()]
        arr[i] = g4d_view(int(v["width"]), int(v["height"]), float(v["fx"]), float(v["fy"]),
                          float(v["cx"]), float(v["cy"]), (C.c_float * 12)(*w2c), float(v["t"]),
                          (C.c_float * 3)(*bg))
    return arr
