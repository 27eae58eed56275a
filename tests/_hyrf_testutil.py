"""Shared helpers of the GPU parity tests: seeded scenes, the oracle run on
the same inputs, and the knife-edge policy for image comparisons."""
from __future__ import annotations

import numpy as np
import torch

import hyrf_inputs as hi
from oracle import hyrf_oracle as O

# Relative distance from a threshold within which float32 may take a decision
# the other way (the knife-edge of the FP32 image tolerance): alpha >= 1/255
# and the early-stop / background tests on the transmittance.  The image
# comparison explains every pixel that differs by one such flipped decision
# (oracle/parity.py); the gradient tests weight these pixels 0.
KNIFE_ALPHA = 1e-4
KNIFE_T = 1e-4
MAX_FLIP_FRAC = 0.01


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


def knife_mask(r, mode, tau=0.2, delta_alpha=KNIFE_ALPHA, delta_T=KNIFE_T):
    """Pixels with a decision within the knife-edge distance of its threshold."""
    st = r["stats"]
    m = (st["edge_alpha"] < delta_alpha) | (st["edge_T"] < delta_T)
    if mode == O.RENDER:
        m = m | (torch.abs(r["T"] / tau - 1.0) < delta_T)
    return m


def compare_image(gpu_rgb_planar, r, mode, H, W, atol=1e-5, gpu_T=None, **kw):
    """gpu_rgb_planar: (3, H, W) numpy; r: oracle result over all pixels.
    Every pixel is compared: equal to the oracle within atol, or to the
    oracle with one near-threshold decision flipped (oracle/parity.py)."""
    from oracle import parity
    kw.setdefault("delta_alpha", KNIFE_ALPHA)
    kw.setdefault("delta_T", KNIFE_T)
    kw.setdefault("max_flip_frac", MAX_FLIP_FRAC)
    res = parity.compare_image(gpu_rgb_planar, r, H, W, gpu_T=gpu_T, atol=atol, **kw)
    if "stats" in r:
        res["knife_frac"] = float(knife_mask(r, mode).double().mean())
    return res
