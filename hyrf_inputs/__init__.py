"""Seeded synthetic inputs for the HyRF render step.

This module only draws random numbers and lays out arrays. It holds none of
the method's arithmetic (no contraction, hashing, MLP, projection or
compositing), so that both the FP64 CPU oracle and the HIP path can be fed
from it without sharing any of the computation they are compared on.

Scenes follow the paper's representation (Sec. 3.2, "Hybrid Radiance
Fields"): explicit compact Gaussians (position, diffuse colour, scale,
opacity; plus an optional explicit rotation residual), two multi-resolution
hash tables (geometry, radiance) and two bias-free ReLU MLP decoders.
The hyper-parameters of the implementation section (16 levels, 2 features
per entry, geometry table half the radiance size, 2 hidden layers of 64)
set the full-size configurations; the table and MLP values are random
initialisations, since trained weights and the paper's datasets are not
available.

Draw order per scene (one PCG64 stream per scene): positions, scale logits
(3 per Gaussian), rotation residual (4), opacity logit, colour logit (3),
geometry table (level-major), radiance table, geometry MLP layers in order,
colour MLP layers in order.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

PE_OCTAVES = 4          # view-direction encoding: 4 octaves of sin/cos -> 24 inputs
GEO_OUT = 8             # geometry decoder outputs: opacity 1, scale 3, rotation 4
COL_OUT = 3             # colour decoder outputs


@dataclasses.dataclass
class SceneConfig:
    name: str
    n_gauss: int
    levels: int
    log2_T_rad: int           # radiance table size T; the geometry table is T/2
    width: int
    height: int
    focal: float
    eye_dist: float
    hidden: int = 64
    n_hidden: int = 2
    base_res: float = 16.0
    growth: float = 1.5
    scale_mu: float = -3.5
    scale_sd: float = 0.3
    shell_frac: float = 0.0   # fraction of positions on the unit-sphere shell
    shell_jitter: float = 0.01
    table_init: float = 1e-4  # tables drawn U(-table_init, table_init)
    n_views: int = 1
    seed: int = 1000

    @property
    def log2_T_geo(self) -> int:
        return self.log2_T_rad - 1

    @property
    def n_in_geo(self) -> int:
        return 2 * self.levels

    @property
    def n_in_col(self) -> int:
        return 2 * self.levels + 6 * PE_OCTAVES


# Workloads.  "tiny": 1k Gaussians, 64x64; "c100k": 100k Gaussians, 800x800;
# "c1m": 1M Gaussians at 1920x1080 (the full-size training / rendering case);
# "c3m_8v": 3M Gaussians, 8 views of 1280x720 in one launch.
CONFIGS = {
    "tiny": SceneConfig("tiny", 1000, 8, 14, 64, 64, 70.0, 3.0, hidden=32, n_hidden=1, seed=1000),
    "c100k": SceneConfig("c100k", 100_000, 16, 19, 800, 800, 875.0, 3.0, seed=1001),
    "c1m": SceneConfig("c1m", 1_000_000, 16, 21, 1920, 1080, 1500.0, 3.5,
                       scale_mu=-4.5, scale_sd=0.5, shell_frac=0.3, seed=1002),
    "c3m_8v": SceneConfig("c3m_8v", 3_000_000, 16, 21, 1280, 720, 1000.0, 3.5,
                          scale_mu=-4.5, scale_sd=0.5, shell_frac=0.3, n_views=8, seed=1004),
}


def with_overrides(cfg: SceneConfig, **kw) -> SceneConfig:
    return dataclasses.replace(cfg, **kw)


@dataclasses.dataclass
class Camera:
    """Pinhole camera, world->camera rotation R (row-major 3x3) and translation t,
    OpenCV axes (x right, y down, z forward).  All values float32."""
    R: np.ndarray        # (3,3) float32
    t: np.ndarray        # (3,) float32
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    z_near: float = 0.2
    cull_tol: float = 0.3


@dataclasses.dataclass
class Scene:
    cfg: SceneConfig
    pos: np.ndarray        # (3, N) float32, planar
    scale_e: np.ndarray    # (3, N) float32, scale logits
    rot_e: Optional[np.ndarray]  # (4, N) float32 (w, x, y, z) or None
    opac_e: np.ndarray     # (N,) float32, opacity logits
    col_e: np.ndarray      # (3, N) float32, colour logits
    table_geo: np.ndarray  # (L, T/2, 2) float32
    table_rad: np.ndarray  # (L, T, 2) float32
    mlp_geo: List[np.ndarray]   # row-major [out][in] float32, layer order
    mlp_col: List[np.ndarray]
    aabb_center: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(3, np.float32))
    aabb_inv_half: np.ndarray = dataclasses.field(default_factory=lambda: np.ones(3, np.float32))
    bg_radius: float = 100.0
    tau_T: float = 0.2

    @property
    def n(self) -> int:
        return self.pos.shape[1]


def look_at(eye, target, focal, width, height, cx=None, cy=None) -> Camera:
    """Camera at `eye` looking at `target`, world up +z, OpenCV axes."""
    eye = np.asarray(eye, np.float64)
    fwd = np.asarray(target, np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    up = np.array([0.0, 0.0, 1.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd]).astype(np.float32)
    t = (-(R.astype(np.float64) @ eye)).astype(np.float32)
    return Camera(R=R, t=t, fx=float(focal), fy=float(focal),
                  cx=float(width / 2 if cx is None else cx),
                  cy=float(height / 2 if cy is None else cy),
                  width=int(width), height=int(height))


def _mlp_layers(rng, n_in, hidden, n_hidden, n_out):
    dims = [n_in] + [hidden] * n_hidden + [n_out]
    out = []
    for a, b in zip(dims[:-1], dims[1:]):
        bound = 1.0 / math.sqrt(a)
        out.append(rng.uniform(-bound, bound, size=(b, a)).astype(np.float32))
    return out


def make_scene(cfg: SceneConfig, seed: Optional[int] = None, with_rot: bool = True,
               table_init: Optional[float] = None) -> Scene:
    rng = np.random.Generator(np.random.PCG64(cfg.seed if seed is None else seed))
    n = cfg.n_gauss
    n_shell = int(round(cfg.shell_frac * n))
    pos = rng.uniform(-1.0, 1.0, size=(n, 3))
    if n_shell:
        d = rng.normal(size=(n_shell, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        d += rng.normal(0.0, cfg.shell_jitter, size=(n_shell, 3))
        sel = rng.permutation(n)[:n_shell]
        pos[sel] = d
    scale_e = rng.normal(cfg.scale_mu, cfg.scale_sd, size=(n, 3))
    rot = rng.normal(size=(n, 4))
    rot /= np.linalg.norm(rot, axis=1, keepdims=True)
    opac = rng.normal(0.0, 1.0, size=n)
    col = rng.uniform(0.0, 1.0, size=(n, 3))
    ti = cfg.table_init if table_init is None else table_init
    T_rad = 1 << cfg.log2_T_rad
    T_geo = 1 << cfg.log2_T_geo
    table_geo = rng.uniform(-ti, ti, size=(cfg.levels, T_geo, 2)).astype(np.float32)
    table_rad = rng.uniform(-ti, ti, size=(cfg.levels, T_rad, 2)).astype(np.float32)
    mlp_geo = _mlp_layers(rng, cfg.n_in_geo, cfg.hidden, cfg.n_hidden, GEO_OUT)
    mlp_col = _mlp_layers(rng, cfg.n_in_col, cfg.hidden, cfg.n_hidden, COL_OUT)
    return Scene(cfg=cfg,
                 pos=np.ascontiguousarray(pos.T.astype(np.float32)),
                 scale_e=np.ascontiguousarray(scale_e.T.astype(np.float32)),
                 rot_e=np.ascontiguousarray(rot.T.astype(np.float32)) if with_rot else None,
                 opac_e=opac.astype(np.float32),
                 col_e=np.ascontiguousarray(col.T.astype(np.float32)),
                 table_geo=table_geo, table_rad=table_rad,
                 mlp_geo=mlp_geo, mlp_col=mlp_col)


def make_cameras(cfg: SceneConfig, seed: int = 3004) -> List[Camera]:
    """One camera at (0, -d, 0) for single-view configs; for several views,
    azimuths drawn U[0, 2pi) on the orbit of radius d at elevation 0."""
    if cfg.n_views == 1:
        return [look_at((0.0, -cfg.eye_dist, 0.0), (0, 0, 0), cfg.focal, cfg.width, cfg.height)]
    rng = np.random.Generator(np.random.PCG64(seed))
    az = rng.uniform(0.0, 2 * math.pi, size=cfg.n_views)
    return [look_at((cfg.eye_dist * math.sin(a), -cfg.eye_dist * math.cos(a), 0.0), (0, 0, 0),
                    cfg.focal, cfg.width, cfg.height) for a in az]


def crop_camera(cam: Camera, x0: int, y0: int, w: int, h: int) -> Camera:
    """The same camera restricted to the pixel window [x0, x0+w) x [y0, y0+h),
    realised by shifting the principal point."""
    return dataclasses.replace(cam, cx=cam.cx - x0, cy=cam.cy - y0, width=w, height=h)


def make_target_image(shape, seed: int = 2001) -> np.ndarray:
    """A fixed random image in [0, 1] (used as an L1 target where no rendered
    target is wanted)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(0.0, 1.0, size=shape).astype(np.float32)


def make_splat_records(n_views: int, n: int, width: int, height: int, seed: int = 77,
                       tile: int = 16, dup_depth_frac: float = 0.2):
    """Synthetic per-splat binning inputs for the tile binning / sort step:
    depth (float32, > 0, with a fraction of exact duplicates so ties occur)
    and inclusive-exclusive tile rectangles [x0, x1) x [y0, y1) in tile units
    (some empty, some clipped at the image border)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    tw = (width + tile - 1) // tile
    th = (height + tile - 1) // tile
    m = n_views * n
    depth = rng.uniform(0.2, 6.0, size=m).astype(np.float32)
    nd = int(dup_depth_frac * m)
    if nd:
        src = rng.integers(0, m, size=nd)
        dst = rng.integers(0, m, size=nd)
        depth[dst] = depth[src]
    cx = rng.integers(-2, tw + 2, size=m)
    cy = rng.integers(-2, th + 2, size=m)
    rx = rng.geometric(0.45, size=m) - 1
    ry = rng.geometric(0.45, size=m) - 1
    x0 = np.clip(cx - rx, 0, tw)
    x1 = np.clip(cx + rx + 1, 0, tw)
    y0 = np.clip(cy - ry, 0, th)
    y1 = np.clip(cy + ry + 1, 0, th)
    empty = rng.uniform(size=m) < 0.05
    x1 = np.where(empty, x0, x1)
    rect = np.stack([x0, y0, x1, y1], axis=1).astype(np.int32)   # (m, 4)
    return depth.reshape(n_views, n), rect.reshape(n_views, n, 4), tw, th


def make_image_pair(shape, seed: int = 2101):
    """A pair of images in [0, 1] shaped like a rendering and its reference
    (..., H, W): a smooth random field (a few random plane waves) with pixel
    noise and a flat patch, and the same field slightly shifted in tone with
    fresh noise.  Exercises textured, smooth and perfectly flat windows."""
    rng = np.random.Generator(np.random.PCG64(seed))
    H, W = shape[-2], shape[-1]
    planes = int(np.prod(shape[:-2])) if len(shape) > 2 else 1
    yy, xx = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    a = np.empty((planes, H, W))
    b = np.empty((planes, H, W))
    for p in range(planes):
        f = np.full((H, W), 0.5)
        for _ in range(4):
            kx, ky = rng.uniform(-0.2, 0.2, size=2)
            f += rng.uniform(0.05, 0.15) * np.sin(kx * xx + ky * yy + rng.uniform(0, 2 * np.pi))
        a[p] = f + rng.normal(0.0, 0.03, size=(H, W))
        b[p] = 0.9 * f + 0.05 + rng.normal(0.0, 0.03, size=(H, W))
        h0, w0 = rng.integers(0, max(1, H // 2)), rng.integers(0, max(1, W // 2))
        a[p, h0:h0 + H // 4, w0:w0 + W // 4] = 0.25
        b[p, h0:h0 + H // 4, w0:w0 + W // 4] = 0.3
    return (np.clip(a, 0, 1).reshape(shape).astype(np.float32),
            np.clip(b, 0, 1).reshape(shape).astype(np.float32))
