"""ctypes binding of libtide.so (the C ABI in include/tide.h).

Argument marshalling only: every step of the hot path runs in the HIP
library.  Importing this module on a machine without the built library
raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtide.so")

TIDE_OK = 0
TIDE_EINVAL = -1
TIDE_ECAPACITY = -2
TIDE_EHIP = -3
TIDE_EIO = -4
TIDE_ESTATE = -5
TIDE_F32 = 0
TIDE_F64 = 1
TIDE_D = 59
TIDE_MAX_CAMS = 8
TIDE_PREPROCESS_NOALLOC_SCRATCH = 262144
TIDE_PREPROCESS_NOALLOC_MAX_PIDX = 134086656


class TideError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"tide error {code}: {msg}")
        self.code = code


class tide_camera(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("t", C.c_double * 3), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("width", C.c_int32), ("height", C.c_int32),
                ("z_near", C.c_double), ("z_far", C.c_double)]


class tide_pool(C.Structure):
    _fields_ = [("params", C.c_void_p), ("exp_avg", C.c_void_p), ("exp_avg_sq", C.c_void_p),
                ("step", C.c_void_p), ("slot_block", C.c_void_p), ("slot_rows", C.c_void_p),
                ("order", C.c_void_p), ("n_slots", C.c_int32), ("block_rows", C.c_int32),
                ("n_order", C.c_int32), ("dtype", C.c_int32)]


class tide_proj(C.Structure):
    _fields_ = [("rec", C.c_void_p), ("depth", C.c_void_p), ("rect", C.c_void_p),
                ("tiles_touched", C.c_void_p), ("active", C.c_void_p), ("act_idx", C.c_void_p),
                ("n_active", C.c_void_p), ("n_pidx", C.c_int64), ("n_cams", C.c_int32), ("dtype", C.c_int32)]


class tide_bins(C.Structure):
    _fields_ = [("vis_rec", C.c_void_p), ("inst_off", C.c_void_p), ("inst_e", C.c_void_p),
                ("inst_rec", C.c_void_p), ("ranges", C.c_void_p), ("tile_order", C.c_void_p),
                ("tile_visits", C.c_void_p), ("n_vis", C.c_int64), ("n_inst", C.c_int64),
                ("n_cams", C.c_int32), ("tiles_x", C.c_int32), ("tiles_y", C.c_int32), ("n_pidx", C.c_int64),
                ("ws_required", C.c_size_t)]


class tide_frame(C.Structure):
    _fields_ = [("image", C.c_void_p), ("t_final", C.c_void_p), ("last", C.c_void_p), ("visits", C.c_void_p),
                ("width", C.c_int32), ("height", C.c_int32)]


class tide_adam_cfg(C.Structure):
    _fields_ = [("lr", C.c_float * TIDE_D), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("kappa", C.c_float)]


class tide_store_cfg(C.Structure):
    _fields_ = [("dir", C.c_char_p), ("n_rows", C.c_int64), ("block_rows", C.c_int32), ("capacity", C.c_int32),
                ("host_cache_blocks", C.c_int64), ("io_threads", C.c_int32), ("flags", C.c_int32),
                ("lambda_", C.c_double), ("gamma", C.c_double), ("kappa", C.c_double)]


class tide_tier_stats(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("blocks_in", C.c_int64), ("blocks_out", C.c_int64),
                ("readmissions", C.c_int64), ("h2d_bytes", C.c_int64), ("d2h_bytes", C.c_int64),
                ("ssd_read_bytes", C.c_int64), ("ssd_write_bytes", C.c_int64), ("host_hits", C.c_int64),
                ("host_misses", C.c_int64), ("sync_fetches", C.c_int64), ("stall_seconds", C.c_double),
                ("resident", C.c_int64), ("prefetch_issued", C.c_int64), ("prefetch_used", C.c_int64),
                ("skipped", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


TIDE_MLP_MAX_LAYERS = 8


class tide_mlp(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("dims", C.c_int32 * (TIDE_MLP_MAX_LAYERS + 1)), ("params", C.c_void_p),
                ("params_bf16", C.c_void_p), ("grad", C.c_void_p), ("exp_avg", C.c_void_p),
                ("exp_avg_sq", C.c_void_p), ("step", C.c_int64)]


TIDE_TIER_HOST_POOL = 1
TIDE_TIER_ODIRECT = 2
TIDE_TIER_NO_TIDE = 4
TIDE_TIER_NO_OVERLAP = 8
TIDE_TIER_COLD_RESTART = 16
TIDE_TIER_BOUNDED = 32

_P = C.POINTER
_vp = C.c_void_p
_pi32 = C.POINTER(C.c_int32)

# name -> (restype, argtypes); every symbol include/tide.h declares
SIGNATURES = {
    "tide_last_error": (C.c_char_p, []),
    "tide_abi_version": (C.c_int32, []),
    "tide_preprocess_ws_bytes": (C.c_size_t, [C.c_int64]),
    "tide_preprocess": (C.c_int32, [_P(tide_pool), _P(tide_camera), C.c_int32, _P(tide_proj), _vp, C.c_size_t, _vp]),
    "tide_preprocess_noalloc": (C.c_int32, [_P(tide_pool), _P(tide_camera), C.c_int32, _P(tide_proj), _vp]),
    "tide_bin_sort_ws_bytes": (C.c_size_t, [C.c_int32, C.c_int64, C.c_int32, C.c_int32, C.c_int64]),
    "tide_bin_sort": (C.c_int32, [_P(tide_proj), C.c_int32, C.c_int32, _vp, C.c_size_t, _P(tide_bins), _vp]),
    "tide_render_fwd": (C.c_int32, [_P(tide_proj), _P(tide_bins), _P(C.c_float), _P(tide_frame), _vp]),
    "tide_loss_ws_bytes": (C.c_size_t, [C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "tide_loss": (C.c_int32, [_vp, _vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _vp, _vp, _vp, C.c_size_t, _vp]),
    "tide_render_bwd_ws_bytes": (C.c_size_t, [_P(tide_bins), C.c_int32]),
    "tide_render_bwd": (C.c_int32, [_P(tide_pool), _P(tide_camera), C.c_int32, _P(tide_proj), _P(tide_bins),
                                    _P(tide_frame), _P(C.c_float), _vp, _vp, C.c_int64, _vp, C.c_size_t, _vp]),
    "tide_adam_ws_bytes": (C.c_size_t, [C.c_int64]),
    "tide_adam_sparse": (C.c_int32, [_P(tide_pool), _P(tide_proj), _vp, C.c_int64, _P(tide_adam_cfg), _vp, _vp,
                                     C.c_int64, _vp, C.c_size_t, _vp]),
    "tide_render_bwd_adam": (C.c_int32, [_P(tide_pool), _P(tide_camera), C.c_int32, _P(tide_proj), _P(tide_bins),
                                         _P(tide_frame), _P(C.c_float), _vp, _P(tide_adam_cfg), _vp, _vp, C.c_int64,
                                         _vp, C.c_size_t, _vp]),
    "tide_timer_arm": (C.c_int32, [C.c_char_p, _vp, _vp]),
    "tide_residency_create": (C.c_int32, [_P(tide_store_cfg), _P(tide_pool), _vp, _vp, _P(_vp)]),
    "tide_residency_destroy": (C.c_int32, [_vp]),
    "tide_store_put_block": (C.c_int32, [_vp, C.c_int64, _vp]),
    "tide_store_finalize": (C.c_int32, [_vp]),
    "tide_store_open": (C.c_int32, [_vp]),
    "tide_cull_blocks": (C.c_int32, [_vp, _P(tide_camera), C.c_int32, _pi32, _pi32, C.c_int64]),
    "tide_ensure_resident": (C.c_int32, [_vp, _pi32, C.c_int32, _vp, _P(C.c_double)]),
    "tide_stream_delta": (C.c_int32, [_vp, _pi32, _pi32, C.c_int32, _vp, _pi32, _pi32, _pi32, _pi32, C.c_int64]),
    "tide_residency_end_iteration": (C.c_int32, [_vp, _vp]),
    "tide_residency_sync_bounds": (C.c_int32, [_vp]),
    "tide_prefetch_hint": (C.c_int32, [_vp, _pi32, C.c_int32, C.c_int32]),
    "tide_checkpoint": (C.c_int32, [_vp]),
    "tide_block_record_bytes": (C.c_size_t, [C.c_int32]),
    "tide_read_block": (C.c_int32, [_vp, C.c_int64, _vp]),
    "tide_tier_get_stats": (C.c_int32, [_vp, _P(tide_tier_stats)]),
    "tide_tier_spheres": (C.c_int32, [_vp, _P(C.c_float), C.c_int64]),
    "tide_tier_resident": (C.c_int32, [_vp, _P(C.c_int32), C.c_int64, _P(C.c_int32)]),
    "tide_timer_clear": (C.c_int32, []),
    "tide_mlp_param_count": (C.c_int64, [_pi32, C.c_int32]),
    "tide_mlp_ws_bytes": (C.c_size_t, [_P(tide_mlp), C.c_int32]),
    "tide_mlp_sync_bf16": (C.c_int32, [_P(tide_mlp), _vp]),
    "tide_mlp_fwd": (C.c_int32, [_P(tide_mlp), _vp, C.c_int32, _vp, _vp, C.c_size_t, _vp]),
    "tide_mlp_bwd": (C.c_int32, [_P(tide_mlp), _vp, _vp, _vp, _vp, C.c_int32, _vp, _vp, C.c_size_t, _vp]),
    "tide_mlp_adam": (C.c_int32, [_P(tide_mlp), C.c_float, C.c_float, C.c_float, C.c_float, _vp]),
    "tide_mlp_predict_bits": (C.c_int32, [_vp, C.c_int32, C.c_int32, C.c_float, _vp, _vp]),
    "tide_pose_features": (C.c_int32, [_P(tide_camera), C.c_int32, C.c_double, _P(C.c_float)]),
    "tide_cull_bits": (C.c_int32, [_P(C.c_float), C.c_int64, _P(tide_camera), C.c_int32, _P(C.c_uint32), C.c_int64]),
    "tide_morton_order": (C.c_int32, [_P(C.c_float), C.c_int64, C.c_int64, _P(C.c_int64)]),
    "tide_view_order": (C.c_int32, [_P(tide_camera), C.c_int64, C.c_int32, C.c_double, _P(C.c_int32)]),
    "tide_layout_build": (C.c_int32, [_vp, C.c_char_p, C.c_char_p, C.c_int64]),
    "tide_store_compact": (C.c_int32, [_vp]),
    "tide_block_sphere": (C.c_int32, [_P(C.c_float), C.c_int64, C.c_int64, C.c_double, _P(C.c_float)]),
}

_lib = None


def load():
    """Load libtide.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2605_20150_amd.build`")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(code: int):
    if code != TIDE_OK:
        raise TideError(code, load().tide_last_error().decode(errors="replace"))
    return code


def make_camera(cam) -> tide_camera:
    """synth.Camera (or any object with the same fields) -> tide_camera."""
    c = tide_camera()
    R = [float(x) for x in __import__("numpy").asarray(cam.R, dtype="float64").reshape(9)]
    t = [float(x) for x in __import__("numpy").asarray(cam.t, dtype="float64").reshape(3)]
    c.R = (C.c_double * 9)(*R)
    c.t = (C.c_double * 3)(*t)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    c.z_near, c.z_far = float(cam.z_near), float(cam.z_far)
    return c


def camera_array(cams):
    arr = (tide_camera * len(cams))()
    for i, cam in enumerate(cams):
        arr[i] = make_camera(cam)
    return arr
