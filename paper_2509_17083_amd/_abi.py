"""ctypes mirror of include/hyrf.h and loader of libhyrf.so.

Argument marshalling only: every computation happens in the library's HIP
kernels.  Importing this module without the built library raises.
"""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libhyrf.so")

HYRF_OK, HYRF_ERR_INVALID_ARGUMENT, HYRF_ERR_UNSUPPORTED, HYRF_ERR_CAPACITY, HYRF_ERR_LAUNCH = range(5)
HYRF_F32, HYRF_F16, HYRF_BF16, HYRF_U8 = 0, 1, 2, 3
HYRF_RENDER, HYRF_TRAIN = 0, 1
HYRF_QUERY_NOALLOC_MAX_GAUSSIANS = 1 << 22
TILE = 16
MAX_VIEWS = 8

P = C.c_void_p


class hyrf_gaussians(C.Structure):
    _fields_ = [("n", C.c_int32), ("pos", P), ("scale_e", P), ("rot_e", P), ("opac_e", P), ("col_e", P),
                ("pos_dtype", C.c_int32)]


class hyrf_fields(C.Structure):
    _fields_ = [("levels", C.c_int32), ("features", C.c_int32), ("log2_T_geo", C.c_int32),
                ("log2_T_rad", C.c_int32), ("base_res", C.c_float), ("growth", C.c_float),
                ("table_dtype", C.c_int32), ("table_geo", P), ("table_rad", P),
                ("hidden", C.c_int32), ("n_hidden", C.c_int32), ("mlp_dtype", C.c_int32),
                ("mlp_geo", P), ("mlp_col", P), ("aabb_center", C.c_float * 3),
                ("aabb_inv_half", C.c_float * 3), ("bg_radius", C.c_float), ("tau_T", C.c_float),
                ("qparams_geo", P), ("qparams_rad", P), ("single_field", C.c_int32),
                ("scatter_merge", C.c_int32)]


class hyrf_camera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32),
                ("z_near", C.c_float), ("cull_tol", C.c_float)]


class hyrf_query_out(C.Structure):
    _fields_ = [("vis_count", P), ("vis_idx", P), ("opacity", P), ("scale", P), ("quat", P),
                ("rgb", P), ("feat_geo", P), ("feat_rad", P), ("dbg_index", P), ("feat_jac", P)]


class hyrf_splats(C.Structure):
    _fields_ = [("n_max", C.c_int32), ("count", P), ("rec", P), ("rect", P), ("depth", P), ("total", P)]


class hyrf_grads(C.Structure):
    _fields_ = [("pos", P), ("scale_e", P), ("rot_e", P), ("opac_e", P), ("col_e", P),
                ("table_geo", P), ("table_rad", P), ("mlp_geo", P), ("mlp_col", P),
                ("dens_accum", P), ("dens_count", P)]


class hyrf_adam_group(C.Structure):
    _fields_ = [("param", P), ("grad", P), ("m", P), ("v", P), ("param_half", P), ("n", C.c_int64),
                ("lr", C.c_float)]


HYRF_PRUNE, HYRF_CLONE, HYRF_SPLIT, HYRF_JUDGED = 1, 2, 4, 8
ADAM_MAX_GROUPS = 16


class hyrf_fwd_state(C.Structure):
    _fields_ = [("query", C.POINTER(hyrf_query_out)), ("splats", C.POINTER(hyrf_splats)),
                ("vals", P), ("tile_ranges", P), ("T_final", P), ("last", P), ("bg_rgb", P), ("bg_feat", P)]


EXPORTS = {
    "hyrf_query_fields": (C.c_int, [C.POINTER(hyrf_fields), C.POINTER(hyrf_gaussians), C.POINTER(hyrf_camera),
                                    C.c_int32, C.POINTER(hyrf_query_out), P, C.c_size_t, P]),
    "hyrf_query_fields_noalloc": (C.c_int, [C.POINTER(hyrf_fields), C.POINTER(hyrf_gaussians),
                                            C.POINTER(hyrf_camera), C.c_int32, C.POINTER(hyrf_query_out), P]),
    "hyrf_query_noalloc_scratch_bytes": (C.c_size_t, []),
    "hyrf_project": (C.c_int, [C.POINTER(hyrf_gaussians), C.POINTER(hyrf_query_out), C.POINTER(hyrf_camera),
                               C.c_int32, C.POINTER(hyrf_splats), P]),
    "hyrf_bin_sort": (C.c_int, [C.POINTER(hyrf_splats), C.POINTER(hyrf_camera), C.c_int32, C.c_int64,
                                C.c_int64, P, P, P, P, C.c_size_t, P]),
    "hyrf_composite": (C.c_int, [C.POINTER(hyrf_splats), P, P, C.POINTER(hyrf_camera), C.c_int32,
                                 C.POINTER(hyrf_fields), C.c_int32, P, P, P, P, P, P, C.c_size_t, P]),
    "hyrf_background": (C.c_int, [C.POINTER(hyrf_fields), C.POINTER(hyrf_camera), C.c_int32, P, P, P]),
    "hyrf_blend_background": (C.c_int, [P, P, P, C.c_int32, C.c_int32, C.c_int32, P]),
    "hyrf_render_backward": (C.c_int, [C.POINTER(hyrf_fields), C.POINTER(hyrf_gaussians), C.POINTER(hyrf_camera),
                                       C.c_int32, C.POINTER(hyrf_fwd_state), P, C.POINTER(hyrf_grads), P,
                                       C.c_size_t, P]),
    "hyrf_render_backward_stage": (C.c_int, [C.c_int32, C.POINTER(hyrf_fields), C.POINTER(hyrf_gaussians),
                                             C.POINTER(hyrf_camera), C.c_int32, C.POINTER(hyrf_fwd_state), P,
                                             C.POINTER(hyrf_grads), P, C.c_size_t, P]),
    "hyrf_l1_loss": (C.c_int, [P, P, C.c_int64, P, P, P, C.c_size_t, P]),
    "hyrf_l1_dssim_loss": (C.c_int, [P, P, C.c_int32, C.c_int32, C.c_int32, C.c_float, P, P, P, C.c_size_t, P]),
    "hyrf_l1_dssim_workspace_bytes": (C.c_size_t, [C.c_int32, C.c_int32, C.c_int32]),
    "hyrf_query_workspace_bytes": (C.c_size_t, [C.c_int32]),
    "hyrf_bin_sort_workspace_bytes": (C.c_size_t, [C.c_int32, C.c_int32, C.c_int64, C.c_int32, C.c_int32]),
    "hyrf_composite_workspace_bytes": (C.c_size_t, [C.c_int32, C.c_int32, C.c_int32]),
    "hyrf_backward_workspace_bytes": (C.c_size_t, [C.POINTER(hyrf_fields), C.c_int32, C.c_int32, C.c_int32,
                                                   C.c_int32]),
    "hyrf_l1_workspace_bytes": (C.c_size_t, [C.c_int64]),
    "hyrf_adam_step": (C.c_int, [C.POINTER(hyrf_adam_group), C.c_int32, C.c_int32, C.c_float, C.c_float,
                                 C.c_float, C.c_int32, P]),
    "hyrf_densify_masks": (C.c_int, [C.POINTER(hyrf_query_out), C.c_int32, C.c_int32, P, P, C.c_float, C.c_float,
                                     C.c_float, P, P]),
    "hyrf_reset_opacity": (C.c_int, [P, C.c_int32, C.c_float, P]),
    "hyrf_quantize_table": (C.c_int, [P, C.c_int32, C.c_int32, P, P, P, C.c_size_t, P]),
    "hyrf_quantize_workspace_bytes": (C.c_size_t, [C.c_int32, C.c_int32]),
    "hyrf_spatial_order": (C.c_int, [C.POINTER(hyrf_fields), P, C.c_int32, P, P, C.c_size_t, P]),
    "hyrf_spatial_order_workspace_bytes": (C.c_size_t, [C.c_int32]),
    "hyrf_last_error": (C.c_char_p, []),
    "hyrf_version": (C.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libhyrf.so (after torch, so that both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  -- torch's HIP runtime must be the one the library binds to
    if not os.path.exists(path):
        raise RuntimeError(f"libhyrf.so not built ({path}); run __graft_entry__.build() or "
                           f"python -m paper_2509_17083_amd.build")
    lib = C.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class HyrfError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn} failed with status {status}: {msg}")
        self.status = status


def check(fn: str, status: int):
    if status != HYRF_OK:
        raise HyrfError(fn, status, load().hyrf_last_error().decode())
