"""Python binding of the HyRF render step: device buffers (torch tensors,
used only for device memory and streams) and the calls of the C ABI in
their order.  Every step of the computation runs in libhyrf.so.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import _abi as A

F32, F16, BF16, U8 = A.HYRF_F32, A.HYRF_F16, A.HYRF_BF16, A.HYRF_U8
RENDER, TRAIN = A.HYRF_RENDER, A.HYRF_TRAIN


def _p(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class DeviceScene:
    """Explicit Gaussians + both fields resident on the GPU (planar float32)."""
    pos: torch.Tensor          # (3, n)
    scale_e: torch.Tensor      # (3, n)
    rot_e: Optional[torch.Tensor]  # (4, n) or None
    opac_e: torch.Tensor       # (n,)
    col_e: torch.Tensor        # (3, n)
    table_geo: torch.Tensor    # (L, T_geo, 2)
    table_rad: torch.Tensor    # (L, T_rad, 2)
    mlp_geo: torch.Tensor      # flat float32
    mlp_col: torch.Tensor
    levels: int
    log2_T_geo: int
    log2_T_rad: int
    hidden: int
    n_hidden: int
    base_res: float = 16.0
    growth: float = 1.5
    aabb_center: Sequence[float] = (0.0, 0.0, 0.0)
    aabb_inv_half: Sequence[float] = (1.0, 1.0, 1.0)
    bg_radius: float = 100.0
    tau_T: float = 0.2
    table_dtype: int = F32
    mlp_dtype: int = F32
    qparams_geo: Optional[torch.Tensor] = None   # (L, 2) (min, step) for U8 tables
    qparams_rad: Optional[torch.Tensor] = None
    pos_dtype: int = F32     # F16: positions stored in half precision (render-only)
    single_field: int = 0    # one field (the radiance table) feeds both decoders
    scatter_merge: int = 0   # background table scatter: 0 automatic, 1 merge shared corners, 2 never

    @property
    def n(self) -> int:
        return int(self.pos.shape[1])

    @staticmethod
    def from_host(s, device: str = "cuda") -> "DeviceScene":
        """From an object with numpy fields pos (3,n), scale_e, rot_e, opac_e,
        col_e, table_geo, table_rad, mlp_geo / mlp_col (lists of [out][in])
        and a cfg with levels, log2_T_rad, log2_T_geo, hidden, n_hidden,
        base_res, growth."""
        def t(a):
            return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
        cfg = s.cfg
        return DeviceScene(
            pos=t(s.pos), scale_e=t(s.scale_e), rot_e=None if s.rot_e is None else t(s.rot_e),
            opac_e=t(s.opac_e), col_e=t(s.col_e), table_geo=t(s.table_geo), table_rad=t(s.table_rad),
            mlp_geo=t(np.concatenate([w.reshape(-1) for w in s.mlp_geo])),
            mlp_col=t(np.concatenate([w.reshape(-1) for w in s.mlp_col])),
            levels=cfg.levels, log2_T_geo=cfg.log2_T_geo, log2_T_rad=cfg.log2_T_rad,
            hidden=cfg.hidden, n_hidden=cfg.n_hidden, base_res=cfg.base_res, growth=cfg.growth,
            aabb_center=tuple(float(x) for x in s.aabb_center),
            aabb_inv_half=tuple(float(x) for x in s.aabb_inv_half),
            bg_radius=float(s.bg_radius), tau_T=float(s.tau_T))

    def with_precision(self, table_dtype: int = F16, mlp_dtype: int = BF16) -> "DeviceScene":
        """The same scene with float16 tables and/or bfloat16 decoder operands
        (weights stay float32 in memory; the kernels round them on load)."""
        import dataclasses
        tt = torch.float16 if table_dtype == F16 else torch.float32
        return dataclasses.replace(self, table_geo=self.table_geo.to(tt).contiguous(),
                                   table_rad=self.table_rad.to(tt).contiguous(),
                                   table_dtype=table_dtype, mlp_dtype=mlp_dtype)

    def quantized(self, mlp_dtype: Optional[int] = None) -> "DeviceScene":
        """The same scene with both tables stored as 8-bit min-max codes
        (quantised on the GPU by hyrf_quantize_table); a render-only format."""
        import dataclasses
        assert self.table_dtype == F32, "quantise from float32 tables"
        lib = A.load()

        def q(t, log2_T):
            codes = torch.empty(t.shape, dtype=torch.uint8, device=t.device)
            qp = torch.empty(self.levels, 2, dtype=torch.float32, device=t.device)
            nb = max(lib.hyrf_quantize_workspace_bytes(self.levels, log2_T), 256)
            w = torch.empty(nb, dtype=torch.uint8, device=t.device)
            A.check("hyrf_quantize_table", lib.hyrf_quantize_table(_p(t), self.levels, log2_T, _p(codes), _p(qp),
                                                                   _p(w), w.numel(), _stream()))
            return codes, qp
        cg, qg = q(self.table_geo, self.log2_T_geo)
        cr, qr = q(self.table_rad, self.log2_T_rad)
        return dataclasses.replace(self, table_geo=cg, table_rad=cr, table_dtype=U8, qparams_geo=qg, qparams_rad=qr,
                                   mlp_dtype=self.mlp_dtype if mlp_dtype is None else mlp_dtype)

    def with_half_positions(self) -> "DeviceScene":
        """The same scene with its positions stored in float16 (rounded to
        nearest even): the compressed model's position format, a
        render-only format decoded where the kernels read positions."""
        import dataclasses
        assert self.pos_dtype == F32
        return dataclasses.replace(self, pos=self.pos.to(torch.float16).contiguous(), pos_dtype=F16)

    def as_single_field(self) -> "DeviceScene":
        """The single-field (non-decoupled) model: the radiance table alone
        feeds both decoders."""
        import dataclasses
        return dataclasses.replace(self, table_geo=self.table_rad, log2_T_geo=self.log2_T_rad,
                                   qparams_geo=self.qparams_rad, single_field=1)

    def spatial_order(self) -> torch.Tensor:
        """Morton-order permutation of the Gaussians (computed on the GPU)."""
        assert self.pos_dtype == F32, "spatial_order takes float32 positions"
        lib = A.load()
        n = self.n
        perm = torch.empty(max(n, 1), dtype=torch.int32, device=self.pos.device)
        w = torch.empty(max(lib.hyrf_spatial_order_workspace_bytes(n), 256), dtype=torch.uint8, device=self.pos.device)
        f = self.c_fields()
        A.check("hyrf_spatial_order", lib.hyrf_spatial_order(C.byref(f), _p(self.pos), n, _p(perm), _p(w), w.numel(),
                                                             _stream()))
        return perm[:n].long()

    def reordered(self, perm: torch.Tensor) -> "DeviceScene":
        """The same scene with its Gaussians stored in the order `perm`."""
        import dataclasses

        def take(t):
            return None if t is None else t[..., perm].contiguous()
        return dataclasses.replace(self, pos=take(self.pos), scale_e=take(self.scale_e), rot_e=take(self.rot_e),
                                   opac_e=take(self.opac_e), col_e=take(self.col_e))

    def c_fields(self) -> A.hyrf_fields:
        f = A.hyrf_fields()
        f.levels, f.features = self.levels, 2
        f.log2_T_geo, f.log2_T_rad = self.log2_T_geo, self.log2_T_rad
        f.base_res, f.growth = self.base_res, self.growth
        f.table_dtype = self.table_dtype
        f.table_geo, f.table_rad = self.table_geo.data_ptr(), self.table_rad.data_ptr()
        f.hidden, f.n_hidden, f.mlp_dtype = self.hidden, self.n_hidden, self.mlp_dtype
        f.mlp_geo, f.mlp_col = self.mlp_geo.data_ptr(), self.mlp_col.data_ptr()
        f.aabb_center[:] = list(self.aabb_center)
        f.aabb_inv_half[:] = list(self.aabb_inv_half)
        f.bg_radius, f.tau_T = self.bg_radius, self.tau_T
        if self.table_dtype == U8:
            f.qparams_geo, f.qparams_rad = self.qparams_geo.data_ptr(), self.qparams_rad.data_ptr()
        f.single_field = int(self.single_field)
        f.scatter_merge = int(self.scatter_merge)
        return f

    def c_gauss(self) -> A.hyrf_gaussians:
        g = A.hyrf_gaussians()
        g.n = self.n
        g.pos, g.scale_e, g.opac_e, g.col_e = (self.pos.data_ptr(), self.scale_e.data_ptr(),
                                               self.opac_e.data_ptr(), self.col_e.data_ptr())
        g.rot_e = None if self.rot_e is None else self.rot_e.data_ptr()
        g.pos_dtype = int(self.pos_dtype)
        return g


def c_cameras(cams) -> "C.Array":
    arr = (A.hyrf_camera * len(cams))()
    for k, c in enumerate(cams):
        arr[k].R[:] = [float(x) for x in np.asarray(c.R, np.float32).reshape(-1)]
        arr[k].t[:] = [float(x) for x in np.asarray(c.t, np.float32).reshape(-1)]
        arr[k].fx, arr[k].fy, arr[k].cx, arr[k].cy = c.fx, c.fy, c.cx, c.cy
        arr[k].width, arr[k].height = c.width, c.height
        arr[k].z_near, arr[k].cull_tol = c.z_near, c.cull_tol
    return arr


class Workspace:
    """Grow-only device scratch buffers, one per named use."""

    def __init__(self):
        self.bufs: Dict[str, torch.Tensor] = {}
        # the last train-mode forward had more tile entries per pixel than
        # BG_LATE_ENTRIES_PER_PIXEL (see `render`)
        self.bg_late = False

    def side_stream(self) -> torch.cuda.Stream:
        """A second stream (default priority) for work that overlaps the
        caller's stream."""
        st = getattr(self, "_side", None)
        if st is None:
            st = self._side = torch.cuda.Stream()
        return st

    def get(self, name: str, nbytes: int) -> torch.Tensor:
        b = self.bufs.get(name)
        if b is None or b.numel() < nbytes:
            b = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device="cuda")
            self.bufs[name] = b
        return b


@dataclass
class ForwardState:
    mode: int
    V: int
    W: int
    H: int
    n_entries: int
    query: Dict[str, torch.Tensor]
    splats: Dict[str, torch.Tensor]
    vals: torch.Tensor
    keys: Optional[torch.Tensor]
    ranges: torch.Tensor
    image: torch.Tensor     # (V, 3, H, W)
    T: torch.Tensor         # (V, H, W)
    last: Optional[torch.Tensor]
    bg: Optional[torch.Tensor]
    bg_feat: Optional[torch.Tensor] = None   # (V*H*W, 2L) background-point features (TRAIN)
    c: Dict[str, object] = field(default_factory=dict)   # ctypes structs kept alive


def _query_outputs(scene: DeviceScene, V: int, mode: int, debug_index: bool):
    n, L = scene.n, scene.levels
    dev = scene.pos.device
    q = dict(vis_count=torch.empty(1, dtype=torch.int32, device=dev),
             vis_idx=torch.empty(max(n, 1), dtype=torch.int32, device=dev),
             opacity=torch.empty(max(n, 1), device=dev), scale=torch.empty(3, max(n, 1), device=dev),
             quat=torch.empty(4, max(n, 1), device=dev), rgb=torch.empty(V, 3, max(n, 1), device=dev))
    if mode == TRAIN:
        q["feat_geo"] = torch.empty(max(n, 1), 2 * L, device=dev)
        q["feat_rad"] = torch.empty(max(n, 1), 2 * L, device=dev)
        q["feat_jac"] = torch.empty(max(n, 1), L, 12, device=dev)   # d(features)/dx for the backward
    if debug_index:
        q["dbg_index"] = torch.empty(max(n, 1), 2, L, 8, dtype=torch.int32, device=dev)
    out = A.hyrf_query_out(*[q[k].data_ptr() if k in q else None for k in
                             ("vis_count", "vis_idx", "opacity", "scale", "quat", "rgb", "feat_geo",
                              "feat_rad", "dbg_index", "feat_jac")])
    return q, out


def query_fields(scene: DeviceScene, cams, mode: int = RENDER, debug_index: bool = False,
                 ws: Optional[Workspace] = None):
    lib = A.load()
    ws = ws or Workspace()
    q, out = _query_outputs(scene, len(cams), mode, debug_index)
    f, g, cc = scene.c_fields(), scene.c_gauss(), c_cameras(cams)
    nb = lib.hyrf_query_workspace_bytes(scene.n)
    w = ws.get("query", nb)
    A.check("hyrf_query_fields", lib.hyrf_query_fields(C.byref(f), C.byref(g), cc, len(cams), C.byref(out),
                                                       _p(w), w.numel(), _stream()))
    return q, out


def query_fields_noalloc(scene: DeviceScene, cams, mode: int = RENDER, debug_index: bool = False,
                         outputs=None):
    """hyrf_query_fields_noalloc: the same query with the library's own
    scratch instead of a workspace.  `outputs` = (q, out) from an earlier call
    to reuse its buffers (then this call allocates nothing at all)."""
    lib = A.load()
    q, out = outputs if outputs is not None else _query_outputs(scene, len(cams), mode, debug_index)
    f, g, cc = scene.c_fields(), scene.c_gauss(), c_cameras(cams)
    A.check("hyrf_query_fields_noalloc", lib.hyrf_query_fields_noalloc(C.byref(f), C.byref(g), cc, len(cams),
                                                                       C.byref(out), _stream()))
    return q, out


def project(scene: DeviceScene, cams, q, qout):
    lib = A.load()
    n, V = scene.n, len(cams)
    dev = scene.pos.device
    sp = dict(rec=torch.empty(V, max(n, 1), 12, device=dev),
              rect=torch.empty(V, max(n, 1), 4, dtype=torch.int32, device=dev),
              depth=torch.empty(V, max(n, 1), device=dev),
              total=torch.empty(1, dtype=torch.int64, device=dev))
    cs = A.hyrf_splats(max(n, 1), q["vis_count"].data_ptr(), sp["rec"].data_ptr(), sp["rect"].data_ptr(),
                       sp["depth"].data_ptr(), sp["total"].data_ptr())
    g, cc = scene.c_gauss(), c_cameras(cams)
    A.check("hyrf_project", lib.hyrf_project(C.byref(g), C.byref(qout), cc, V, C.byref(cs), _stream()))
    return sp, cs


def bin_sort(cams, splats_c, n_max: int, n_entries: int, want_keys: bool = False,
             ws: Optional[Workspace] = None, capacity: Optional[int] = None):
    lib = A.load()
    ws = ws or Workspace()
    V, W, H = len(cams), cams[0].width, cams[0].height
    tiles = ((W + 15) // 16) * ((H + 15) // 16)
    cap = n_entries if capacity is None else capacity
    vals = torch.empty(max(cap, 1), dtype=torch.int32, device="cuda")
    keys = torch.empty(max(cap, 1), dtype=torch.int32, device="cuda") if want_keys else None
    ranges = torch.empty(V * tiles, 2, dtype=torch.int32, device="cuda")
    nb = lib.hyrf_bin_sort_workspace_bytes(V, n_max, cap, W, H)
    w = ws.get("bin", nb)
    cc = c_cameras(cams)
    A.check("hyrf_bin_sort", lib.hyrf_bin_sort(C.byref(splats_c), cc, V, n_entries, cap, _p(keys), _p(vals),
                                               _p(ranges), _p(w), w.numel(), _stream()))
    return keys, vals, ranges


def composite(scene: Optional[DeviceScene], cams, splats_c, vals, ranges, mode: int,
              ws: Optional[Workspace] = None, keep_bg_feat: bool = True):
    lib = A.load()
    ws = ws or Workspace()
    V, W, H = len(cams), cams[0].width, cams[0].height
    img = torch.empty(V, 3, H, W, device="cuda")
    T = torch.empty(V, H, W, device="cuda")
    last = torch.empty(V, H, W, dtype=torch.int32, device="cuda") if mode == TRAIN else None
    bg = torch.empty(V, 3, H, W, device="cuda") if (mode == TRAIN and scene is not None) else None
    # background-point features kept for the backward (TRAIN mode)
    bg_feat = (torch.empty(V * H * W, 2 * scene.levels, device="cuda")
               if (mode == TRAIN and scene is not None and keep_bg_feat) else None)
    nb = lib.hyrf_composite_workspace_bytes(V, W, H)
    w = ws.get("composite", nb)
    cc = c_cameras(cams)
    f = scene.c_fields() if scene is not None else None
    A.check("hyrf_composite", lib.hyrf_composite(C.byref(splats_c), _p(vals), _p(ranges), cc, V,
                                                 C.byref(f) if f is not None else None, mode, _p(img), _p(T),
                                                 _p(last), _p(bg), _p(bg_feat), _p(w), w.numel(), _stream()))
    return img, T, last, bg, bg_feat


def _mark(events, name, stream=None):
    if events is not None:
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        events.setdefault(name, []).append(e)


# Tile entries per pixel above which blending outlasts the background query
# of every pixel (blending ~20 ps per entry, the background ~0.3 ns per pixel
# on one MI355X), so that the train-mode background is started after binning.
BG_LATE_ENTRIES_PER_PIXEL = 15


def render(scene: DeviceScene, cams, mode: int = RENDER, debug_index: bool = False, want_keys: bool = False,
           ws: Optional[Workspace] = None, events: Optional[dict] = None, overlap: bool = True) -> ForwardState:
    """The forward render step: query -> project -> bin/sort -> composite
    (+ background).  One host read (the tile-entry count).  `events`, if
    given, collects torch.cuda.Event pairs around each ABI call.  In TRAIN
    mode with `overlap`, the background of every pixel (which needs only the
    cameras and the fields) runs on a second stream and is blended in at the
    end; the result is bit-identical.  It starts once the field query is
    done (both are gather-bound), beside projection, binning and blending;
    when blending is the longer stage (more than BG_LATE_ENTRIES_PER_PIXEL
    tile entries per pixel in the previous train-mode forward with the same
    workspace: the count of this one is known only after projection), after
    binning, so that it shares the CUs with blending's VALU work rather than
    with the sort's memory streams."""
    lib = A.load()
    ws = ws or Workspace()
    V, W, H = len(cams), cams[0].width, cams[0].height
    split_bg = mode == TRAIN and overlap
    late_bg = split_bg and ws.bg_late

    def launch_bg():
        main = torch.cuda.current_stream()
        side = ws.side_stream()
        e_start = torch.cuda.Event()
        e_start.record(main)
        side.wait_event(e_start)
        f_bg, cc_bg = scene.c_fields(), c_cameras(cams)
        _mark(events, "bg0", side)
        A.check("hyrf_background", lib.hyrf_background(C.byref(f_bg), cc_bg, V, _p(bg), _p(bg_feat),
                                                       C.c_void_p(side.cuda_stream)))
        _mark(events, "bg1", side)
        e_bg = torch.cuda.Event()
        e_bg.record(side)
        return e_bg

    _mark(events, "query0")
    q, qout = query_fields(scene, cams, mode, debug_index, ws)
    _mark(events, "query1")
    if split_bg:
        bg = torch.empty(V, 3, H, W, device="cuda")
        bg_feat = torch.empty(V * H * W, 2 * scene.levels, device="cuda")
        if not late_bg:
            e_bg = launch_bg()
    sp, spc = project(scene, cams, q, qout)
    _mark(events, "project1")
    n_entries = int(sp["total"].item())
    if split_bg:
        ws.bg_late = n_entries > BG_LATE_ENTRIES_PER_PIXEL * V * W * H
    _mark(events, "bin0")
    keys, vals, ranges = bin_sort(cams, spc, max(scene.n, 1), n_entries, want_keys, ws)
    _mark(events, "bin1")
    if split_bg:
        if late_bg:
            e_bg = launch_bg()
        img, T, last, _, _ = composite(None, cams, spc, vals, ranges, mode, ws)
        torch.cuda.current_stream().wait_event(e_bg)
        A.check("hyrf_blend_background", lib.hyrf_blend_background(_p(bg), _p(T), _p(img), V, W, H, _stream()))
    else:
        img, T, last, bg, bg_feat = composite(scene, cams, spc, vals, ranges, mode, ws)
    _mark(events, "composite1")
    return ForwardState(mode=mode, V=V, W=W, H=H, n_entries=n_entries, query=q, splats=sp, vals=vals,
                        keys=keys, ranges=ranges, image=img, T=T, last=last, bg=bg, bg_feat=bg_feat,
                        c=dict(qout=qout, splats=spc))


def l1_loss(img: torch.Tensor, target: torch.Tensor, grad: bool = True, ws: Optional[Workspace] = None):
    lib = A.load()
    ws = ws or Workspace()
    n = img.numel()
    loss = torch.empty(1, device="cuda")
    g = torch.empty_like(img) if grad else None
    w = ws.get("l1", lib.hyrf_l1_workspace_bytes(n))
    A.check("hyrf_l1_loss", lib.hyrf_l1_loss(_p(img), _p(target), n, _p(loss), _p(g), _p(w), w.numel(),
                                             _stream()))
    return loss, g


def l1_dssim_loss(img: torch.Tensor, target: torch.Tensor, lam: float = 0.2, grad: bool = True,
                  ws: Optional[Workspace] = None):
    """(1 - lam) L1 + lam (1 - SSIM) of (..., H, W) float32 images and its
    gradient, fused in one kernel.  Returns (float32[3] = (loss, L1, SSIM),
    dloss/dimg or None)."""
    lib = A.load()
    ws = ws or Workspace()
    H, W = img.shape[-2], img.shape[-1]
    planes = img.numel() // (H * W)
    assert img.is_contiguous() and target.is_contiguous() and target.shape == img.shape
    loss = torch.empty(3, device="cuda")
    g = torch.empty_like(img) if grad else None
    w = ws.get("l1_dssim", lib.hyrf_l1_dssim_workspace_bytes(planes, H, W))
    A.check("hyrf_l1_dssim_loss", lib.hyrf_l1_dssim_loss(_p(img), _p(target), planes, H, W, float(lam), _p(loss),
                                                         _p(g), _p(w), w.numel(), _stream()))
    return loss, g


def render_backward(scene: DeviceScene, cams, st: ForwardState, dL_drgb: torch.Tensor,
                    grads: Optional[Dict[str, torch.Tensor]] = None, ws: Optional[Workspace] = None,
                    events: Optional[dict] = None, overlap: bool = True):
    """Adjoint of a TRAIN-mode `render`: accumulates (+=) gradients of every
    explicit parameter, both tables and both decoders into `grads` (zeroed
    here when not given).  dL_drgb: (V, 3, H, W) float32.  overlap: run the
    Gaussian and background branches of the adjoint on two streams."""
    lib = A.load()
    ws = ws or Workspace()
    if st.mode != TRAIN:
        raise ValueError("render_backward needs a TRAIN-mode forward state")
    dL = dL_drgb.contiguous().float()
    if grads is None:
        z = torch.zeros_like
        grads = dict(pos=z(scene.pos), scale_e=z(scene.scale_e),
                     rot_e=None if scene.rot_e is None else z(scene.rot_e), opac_e=z(scene.opac_e),
                     col_e=z(scene.col_e), table_geo=torch.zeros(scene.table_geo.shape, device="cuda"),
                     table_rad=torch.zeros(scene.table_rad.shape, device="cuda"), mlp_geo=z(scene.mlp_geo),
                     mlp_col=z(scene.mlp_col))
    cg = A.hyrf_grads(*[_p(grads.get(k)) if grads.get(k) is not None else None for k in
                        ("pos", "scale_e", "rot_e", "opac_e", "col_e", "table_geo", "table_rad", "mlp_geo",
                         "mlp_col", "dens_accum", "dens_count")])
    qout, spc = st.c["qout"], st.c["splats"]
    fs = A.hyrf_fwd_state(C.pointer(qout), C.pointer(spc), st.vals.data_ptr(), st.ranges.data_ptr(),
                          st.T.data_ptr(), st.last.data_ptr(), st.bg.data_ptr(),
                          None if st.bg_feat is None else st.bg_feat.data_ptr())
    f, g, cc = scene.c_fields(), scene.c_gauss(), c_cameras(cams)
    nb = lib.hyrf_backward_workspace_bytes(C.byref(f), len(cams), max(scene.n, 1), cams[0].width, cams[0].height)
    w = ws.get("backward", nb)
    def stage(k, stream):
        A.check("hyrf_render_backward_stage",
                lib.hyrf_render_backward_stage(k, C.byref(f), C.byref(g), cc, len(cams), C.byref(fs), _p(dL),
                                               C.byref(cg), _p(w), w.numel(), C.c_void_p(stream.cuda_stream)))

    if not overlap:
        if events is None:
            A.check("hyrf_render_backward",
                    lib.hyrf_render_backward(C.byref(f), C.byref(g), cc, len(cams), C.byref(fs), _p(dL),
                                             C.byref(cg), _p(w), w.numel(), _stream()))
            return grads
        main = torch.cuda.current_stream()
        for k in range(7):
            _mark(events, f"bwd_stage{k}")
            stage(k, main)
        _mark(events, "bwd_stage7")
        return grads
    # two streams: after the weight permutation (0), the background branch
    # (stages 4, 5) runs on a side stream while the Gaussian branch (1, 2, 3)
    # runs on the caller's stream; they join before the weight gradients (6)
    main = torch.cuda.current_stream()
    side = ws.side_stream()
    _mark(events, "bwd_stage0")
    stage(0, main)
    e0 = torch.cuda.Event()
    e0.record(main)
    side.wait_event(e0)
    _mark(events, "bwd_stage4", side)
    stage(4, side)
    _mark(events, "bwd_stage5", side)
    stage(5, side)
    _mark(events, "bwd_bg_end", side)
    e1 = torch.cuda.Event()
    e1.record(side)
    _mark(events, "bwd_stage1")
    stage(1, main)
    _mark(events, "bwd_stage2")
    stage(2, main)
    _mark(events, "bwd_stage3")
    stage(3, main)
    _mark(events, "bwd_gauss_end")
    main.wait_event(e1)
    _mark(events, "bwd_stage6")
    stage(6, main)
    _mark(events, "bwd_stage7")
    return grads


def adam_step(groups: Sequence[dict], step: int, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-15,
              zero_grad: bool = True):
    """One fused Adam step over up to 16 tensors.  Each group is a dict with
    float32 CUDA tensors param, grad, m, v (same numel, contiguous), a float
    lr and optionally a float16 tensor param_half (written from the updated
    param)."""
    lib = A.load()
    arr = (A.hyrf_adam_group * len(groups))()
    for k, g in enumerate(groups):
        n = g["param"].numel()
        for key in ("grad", "m", "v"):
            assert g[key].numel() == n and g[key].is_contiguous() and g[key].dtype == torch.float32
        ph = g.get("param_half")
        arr[k] = A.hyrf_adam_group(g["param"].data_ptr(), g["grad"].data_ptr(), g["m"].data_ptr(),
                                   g["v"].data_ptr(), None if ph is None else ph.data_ptr(), n, float(g["lr"]))
    A.check("hyrf_adam_step", lib.hyrf_adam_step(arr, len(groups), int(step), float(beta1), float(beta2),
                                                 float(eps), int(bool(zero_grad)), _stream()))


def densify_masks(st: "ForwardState", n: int, dens_accum: torch.Tensor, dens_count: torch.Tensor,
                  grad_threshold: float = 2e-4, dense_extent: float = 0.01, min_opacity: float = 0.005):
    """uint8 flags per Gaussian (HYRF_PRUNE / CLONE / SPLIT / JUDGED) from a
    forward state's query output and the accumulated statistics."""
    lib = A.load()
    flags = torch.empty(n, dtype=torch.uint8, device="cuda")
    qout = st.c["qout"]
    A.check("hyrf_densify_masks", lib.hyrf_densify_masks(C.byref(qout), n, n, _p(dens_accum), _p(dens_count),
                                                         float(grad_threshold), float(dense_extent),
                                                         float(min_opacity), _p(flags), _stream()))
    return flags


def reset_opacity(opac_e: torch.Tensor, value: float = 0.01):
    lib = A.load()
    A.check("hyrf_reset_opacity", lib.hyrf_reset_opacity(_p(opac_e), opac_e.numel(), float(value), _stream()))


class HyRFRender(torch.autograd.Function):
    """Differentiable render step: forward = `render(..., TRAIN)`, backward =
    `render_backward`.  Inputs are the scene's tensors; the scene object
    carries the configuration.  Returns the (V, 3, H, W) image."""

    @staticmethod
    def forward(ctx, scene, cams, pos, scale_e, rot_e, opac_e, col_e, table_geo, table_rad, mlp_geo, mlp_col):
        st = render(scene, cams, TRAIN)
        ctx.scene, ctx.cams, ctx.st = scene, cams, st
        ctx.has_rot = rot_e is not None
        return st.image

    @staticmethod
    def backward(ctx, g_img):
        gr = render_backward(ctx.scene, ctx.cams, ctx.st, g_img)
        return (None, None, gr["pos"], gr["scale_e"], gr["rot_e"] if ctx.has_rot else None, gr["opac_e"],
                gr["col_e"], gr["table_geo"], gr["table_rad"], gr["mlp_geo"], gr["mlp_col"])


def render_differentiable(scene: DeviceScene, cams) -> torch.Tensor:
    return HyRFRender.apply(scene, cams, scene.pos, scene.scale_e, scene.rot_e, scene.opac_e, scene.col_e,
                            scene.table_geo, scene.table_rad, scene.mlp_geo, scene.mlp_col)
