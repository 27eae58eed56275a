"""HyRF differentiable render step for AMD MI355X (gfx950).

The computation lives in lib/libhyrf.so (hand-written HIP kernels behind the
C ABI of include/hyrf.h); this package only marshals torch device buffers
into those calls.
"""
from . import _abi
from .render import (BF16, F16, F32, U8, RENDER, TRAIN, DeviceScene, ForwardState, HyRFRender, Workspace, bin_sort,
                     adam_step, c_cameras, composite, densify_masks, l1_dssim_loss, l1_loss, project, query_fields, query_fields_noalloc, render, render_backward,
                     render_differentiable, reset_opacity)

__all__ = ["DeviceScene", "ForwardState", "Workspace", "render", "query_fields", "query_fields_noalloc", "project", "bin_sort",
           "composite", "l1_dssim_loss", "l1_loss", "c_cameras", "render_backward", "render_differentiable", "HyRFRender", "adam_step", "densify_masks", "reset_opacity",
           "RENDER", "TRAIN", "F32", "F16", "BF16", "U8"]
