"""Shared helpers of the GPU parity tests: seeded scenes, the oracle run on
the same inputs, and the knife-edge policy for image comparisons."""
from __future__ import annotations

import numpy as np
import torch

import hyrf_inputs as hi
from oracle import hyrf_oracle as O

# relative distance to a threshold below which a pixel is a knife-edge: the
# float32 alpha carries ~1e-6 relative error, the float32 transmittance after
# many near-opaque splats up to ~1e-4
KNIFE_ALPHA = 1e-4
KNIFE_T = 1e-3


def make(cfg_name: str, seed=None, table_init=None, with_rot=True, **over):
    cfg = hi.with_overrides(hi.CONFIGS[cfg_name], **over) if over else hi.CONFIGS[cfg_name]
    scene = hi.make_scene(cfg, seed=seed, with_rot=with_rot, table_init=table_init)
    cams = hi.make_cameras(cfg)
    return cfg, scene, cams


def device_scene(scene):
    import paper_2509_17083_amd as P
    return P.DeviceScene.from_host(scene)


def oracle_view(scene, cam, mode, pixels=None, stats=True):
    params, fields = O.from_scene(scene)
    with torch.no_grad():
        return O.render_view(params, fields, cam, mode, pixels=pixels, return_stats=stats)


def knife_mask(r, mode, tau=0.2):
    st = r["stats"]
    m = (st["edge_alpha"] < KNIFE_ALPHA) | (st["edge_T"] < KNIFE_T)
    if mode == O.RENDER:
        m = m | (torch.abs(r["T"] / tau - 1.0) < KNIFE_T)
    return m


def compare_image(gpu_rgb_planar, r, mode, H, W, atol=1e-5, max_knife_frac=0.05):
    """gpu_rgb_planar: (3, H, W) numpy; r: oracle result over all pixels."""
    ref = r["rgb"].numpy().T.reshape(3, H, W)
    knife = knife_mask(r, mode).numpy().reshape(H, W)
    diff = np.abs(gpu_rgb_planar.astype(np.float64) - ref).max(axis=0)
    bad = (diff > atol) & ~knife
    return dict(max_err=float(diff[~knife].max()) if (~knife).any() else 0.0,
                n_bad=int(bad.sum()), knife_frac=float(knife.mean()), ok=(not bad.any()) and knife.mean() <= max_knife_frac)
