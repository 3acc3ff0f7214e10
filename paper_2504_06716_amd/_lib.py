"""ctypes binding of libgsta (include/gsta.h): the same entry points, with
plain integers for device pointers and streams.  Argument marshalling only;
every step runs in the HIP library, which must be built (see build.py)."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# GSTA_LIB selects another build of the same library (same ABI).
LIB_PATH = os.environ.get("GSTA_LIB") or os.path.join(_HERE, "libgsta.so")

GSTA_OK, GSTA_ERR_INVALID, GSTA_ERR_CAPACITY, GSTA_ERR_HIP, GSTA_ERR_OOM, GSTA_ERR_NONFINITE = range(6)
STATUS_NAMES = {0: "OK", 1: "INVALID", 2: "CAPACITY", 3: "HIP", 4: "OOM", 5: "NONFINITE"}

(STATE_REC_GEO, STATE_REC_COL, STATE_REC_RGB, STATE_RECT, STATE_DEPTH_ORDER, STATE_INST_KEYS,
 STATE_INST_IDS, STATE_RANGES, STATE_T_FINAL, STATE_LAST, STATE_N_INSTANCES, STATE_INST_GID) = range(12)
OPT_FWD_WAVES, OPT_BWD_WAVES, OPT_BWD_SEGMENT, OPT_BINNING, OPT_DEPTH_SORT, OPT_BWD_VARIANT = 0, 1, 2, 3, 4, 5
FREEZE_RULE_MINGRAD, FREEZE_RULE_RANDOM = 1, 2


class Limits(ctypes.Structure):
    _fields_ = [("max_gaussians", ctypes.c_int64), ("max_views", ctypes.c_int32),
                ("max_height", ctypes.c_int32), ("max_width", ctypes.c_int32),
                ("instance_capacity", ctypes.c_int64), ("tile_w", ctypes.c_int32),
                ("tile_h", ctypes.c_int32), ("n_slots", ctypes.c_int32)]


class Camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("world_to_cam", ctypes.c_float * 12), ("cam_pos", ctypes.c_float * 3),
                ("near_z", ctypes.c_float)]


class Params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("ld", ctypes.c_int64), ("sh_degree", ctypes.c_int32),
                ("opacity_act", ctypes.c_int32), ("block", ctypes.c_void_p), ("sh_mask", ctypes.c_void_p),
                ("sh_mask_threshold", ctypes.c_float)]


class AdamSched(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int32), ("decay_iters", ctypes.c_int32), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("pos_lr_init", ctypes.c_float),
                ("pos_lr_final", ctypes.c_float), ("pos_scale", ctypes.c_float), ("lr", ctypes.c_float * 64)]


class DensifyCfg(ctypes.Structure):
    _fields_ = [("grad_threshold", ctypes.c_float), ("rgb_threshold", ctypes.c_float),
                ("use_rgb", ctypes.c_int32), ("split_log_scale", ctypes.c_float),
                ("prune_logit", ctypes.c_float), ("child_log_scale_shift", ctypes.c_float),
                ("noise_seed", ctypes.c_uint64), ("noise_draw", ctypes.c_int64)]


class Columns(ctypes.Structure):
    _fields_ = [("base", ctypes.c_void_p), ("rows", ctypes.c_int64), ("ld", ctypes.c_int64),
                ("elem_bytes", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("fwd_waves", ctypes.c_int32), ("bwd_waves", ctypes.c_int32), ("bwd_segment", ctypes.c_int32),
                ("candidates", ctypes.c_int32), ("fwd_ms", ctypes.c_float), ("step_ms", ctypes.c_float),
                ("bwd_variant", ctypes.c_int32)]


class GstaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"gsta error {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None

EXPORTS = ["gsta_create", "gsta_reserve", "gsta_destroy", "gsta_last_error", "gsta_check",
           "gsta_get_state", "gsta_render_forward", "gsta_render_forward_l1", "gsta_render_backward", "gsta_adam_masked",
           "gsta_update_freeze_mask", "gsta_partition_frozen", "gsta_l1_loss", "gsta_set_profiling", "gsta_read_profile", "gsta_set_option", "gsta_adam_masked_sched",
           "gsta_densify_prune", "gsta_opacity_reset", "gsta_traj_push", "gsta_mlp_feature_stats",
           "gsta_mlp_features", "gsta_mlp_forward", "gsta_mlp_bce", "gsta_mlp_backward", "gsta_mlp_adam",
           "gsta_mlp_sync_bf16", "gsta_mlp_propose", "gsta_l1_loss_noalloc", "gsta_update_freeze_mask_rule", "gsta_dssim_loss", "gsta_opacity_to_absolute", "gsta_adam_rows", "gsta_sh_mask_reg",
           "gsta_graph_begin", "gsta_graph_end", "gsta_graph_launch", "gsta_graph_destroy", "gsta_autotune"]

MLP_PARAMS, MLP_BF16 = 6337, 6144
L1_NOALLOC_MAX_COUNT = 1 << 30
PROFILE_COUNTERS = 1 << 30

PHASES = ["preprocess", "depth_sort", "binning", "tile_sort", "composite", "composite_bwd",
          "preprocess_bwd", "adam", "freeze", "loss", "densify"]


def load(path: str = LIB_PATH):
    """Load libgsta.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libgsta.so not found at {path}: build it with "
                           "`python -m paper_2504_06716_amd.build` (hipcc, gfx950)")
    L = ctypes.CDLL(path)
    P, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    PP = ctypes.POINTER(Params)
    L.gsta_create.argtypes = [ctypes.POINTER(Limits), ctypes.POINTER(P)]
    L.gsta_reserve.argtypes = [P, ctypes.POINTER(Limits)]
    L.gsta_destroy.argtypes = [P]
    L.gsta_destroy.restype = None
    L.gsta_last_error.argtypes = [P]
    L.gsta_last_error.restype = ctypes.c_char_p
    L.gsta_check.argtypes = [P, P, ctypes.POINTER(i64)]
    L.gsta_get_state.argtypes = [P, i32, i32, P, i64, P]
    L.gsta_render_forward.argtypes = [P, PP, ctypes.POINTER(Camera), i32, ctypes.POINTER(f32), P, i32, P]
    L.gsta_render_forward_l1.argtypes = [P, PP, ctypes.POINTER(Camera), i32, ctypes.POINTER(f32), P, P, P, P, i32, P]
    L.gsta_render_backward.argtypes = [P, PP, ctypes.POINTER(Camera), i32, ctypes.POINTER(f32), i32, P, P,
                                       PP, P, P, f32, P, P]
    L.gsta_densify_prune.argtypes = [P, PP, PP, PP, P, P, P, P, ctypes.POINTER(DensifyCfg), PP, PP, PP, P, P, P, P]
    L.gsta_opacity_reset.argtypes = [P, PP, PP, PP, P, f32, P]
    L.gsta_opacity_to_absolute.argtypes = [P, PP, PP, PP, P]
    L.gsta_graph_begin.argtypes = [P, P]
    L.gsta_graph_end.argtypes = [P, P, ctypes.POINTER(P)]
    L.gsta_graph_launch.argtypes = [P, P]
    L.gsta_graph_destroy.argtypes = [P]
    L.gsta_graph_destroy.restype = None
    L.gsta_autotune.argtypes = [P, PP, ctypes.POINTER(Camera), i32, ctypes.POINTER(f32), P, P, PP, P, i32,
                                ctypes.POINTER(Tuning), P]
    L.gsta_traj_push.argtypes = [P, P, i64, P, i32, P]
    L.gsta_mlp_feature_stats.argtypes = [P, P, i64, i32, P, P]
    L.gsta_mlp_features.argtypes = [P, P, i64, i32, P, P, P, P]
    L.gsta_mlp_forward.argtypes = [P, P, P, P, i64, P, P, P, P]
    L.gsta_mlp_bce.argtypes = [P, P, P, i64, P, P, P]
    L.gsta_mlp_backward.argtypes = [P, P, P, P, P, P, P, i64, P, P]
    L.gsta_mlp_adam.argtypes = [P, P, P, P, P, f32, f32, f32, f32, i32, P, P]
    L.gsta_mlp_sync_bf16.argtypes = [P, P, P, P]
    L.gsta_mlp_propose.argtypes = [P, P, P, P, i64, f32, f32, f32, P, P]
    L.gsta_adam_masked.argtypes = [P, PP, PP, PP, PP, ctypes.POINTER(f32), f32, f32, f32, i32, P, P]
    L.gsta_update_freeze_mask.argtypes = [P, P, P, i64, f32, f32, i32, P, P, P, P]
    L.gsta_partition_frozen.argtypes = [P, i64, P, ctypes.POINTER(Columns), i32, P, i64, P, P]
    L.gsta_l1_loss.argtypes = [P, P, P, i64, P, P, P]
    L.gsta_l1_loss_noalloc.argtypes = [P, P, i64, P, P, P]
    L.gsta_dssim_loss.argtypes = [P, P, P, i32, i32, i32, f32, P, P, P]
    L.gsta_adam_rows.argtypes = [P, P, P, P, P, i64, i64, i32, ctypes.POINTER(f32), f32, f32, f32, i32, P, P]
    L.gsta_sh_mask_reg.argtypes = [P, P, i64, i64, f32, f32, P, P, P, P]
    L.gsta_update_freeze_mask_rule.argtypes = [P, i32, P, i64, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64,
                                               i32, P, P, P]
    L.gsta_set_profiling.argtypes = [P, i32]
    L.gsta_set_option.argtypes = [P, i32, i64]
    L.gsta_adam_masked_sched.argtypes = [P, PP, PP, PP, PP, P, P, P]
    L.gsta_read_profile.argtypes = [P, P, P, P]
    for name in EXPORTS:
        if name not in ("gsta_destroy", "gsta_last_error", "gsta_graph_destroy"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def check(ctx, status: int):
    if status != GSTA_OK:
        msg = load().gsta_last_error(ctx)
        raise GstaError(status, msg.decode() if msg else "")
