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


class DirectionalCase:
    """A loss L = sum(w * C) over seeded pixels of one view (knife-edge
    pixels weighted 0) with the FP64 oracle's gradient and central
    differences along directions supported on a seeded 1% of every parameter
    tensor.  The oracle evaluates L on the Gaussians that have a (pixel,
    splat) pair among the sampled pixels, which is the same loss (checked at
    construction) at a fraction of the cost."""
    names = ["pos", "scale_e", "rot_e", "opac_e", "col_e", "table_geo", "table_rad", "mlp_geo", "mlp_col"]

    def __init__(self, cfg_name, n_pixels, seed, table_init=1.0, **over):
        self.cfg, self.scene, self.cams = make(cfg_name, table_init=table_init, **over)
        cam = self.cam = self.cams[0]
        H, W = cam.height, cam.width
        rng = np.random.default_rng(seed)
        flat = rng.choice(H * W, n_pixels, replace=False)
        self.pix = torch.from_numpy(np.stack([flat % W, flat // W], 1)).long()
        self.params, self.fields = O.from_scene(self.scene)
        with torch.no_grad():
            r = O.render_view(self.params, self.fields, cam, O.TRAIN, pixels=self.pix, return_stats=True)
            _, si = O._pairs_for_pixels(r["px"], r["py"], r["proj"]["u"], r["proj"]["v"], r["rx"], r["ry"])
        self.touched = torch.unique(r["vis_idx"][si])
        knife = knife_mask(r, O.TRAIN)
        self.w = torch.from_numpy(rng.normal(size=(n_pixels, 3))) * (~knife).double()[:, None]
        print("pixels", n_pixels, "knife", int(knife.sum()), "Gaussians with pairs", self.touched.numel(), flush=True)
        self.sizes_geo = [int(x.numel()) for x in self.fields.mlp_geo]
        self.sizes_col = [int(x.numel()) for x in self.fields.mlp_col]
        p, f = self.params, self.fields
        self.shapes = dict(pos=p.pos.shape, scale_e=p.scale_e.shape, rot_e=p.rot_e.shape, opac_e=p.opac_e.shape,
                           col_e=p.col_e.shape, table_geo=f.table_geo.shape, table_rad=f.table_rad.shape,
                           mlp_geo=(sum(self.sizes_geo),), mlp_col=(sum(self.sizes_col),))
        L_full = float(torch.sum(r["rgb"] * self.w))
        L_sub = self.loss(None, 0.0)
        assert abs(L_sub - L_full) <= 1e-12 * max(1.0, abs(L_full)), (L_sub, L_full)
        # the oracle's exact gradient on the same Gaussians (autograd)
        ps, fs = O.from_scene(self.scene, requires_grad=True)
        t = self.touched
        sub = O.Params(pos=ps.pos[t], scale_e=ps.scale_e[t], rot_e=ps.rot_e[t], opac_e=ps.opac_e[t], col_e=ps.col_e[t])
        Lo = torch.sum(O.render_view(sub, fs, cam, O.TRAIN, pixels=self.pix)["rgb"] * self.w)
        leaves = [ps.pos, ps.scale_e, ps.rot_e, ps.opac_e, ps.col_e, fs.table_geo, fs.table_rad] + fs.mlp_geo + fs.mlp_col
        gs = torch.autograd.grad(Lo, leaves)
        self.grad = dict(zip(self.names[:7], gs[:7]))
        self.grad["mlp_geo"] = torch.cat([x.reshape(-1) for x in gs[7:7 + len(self.sizes_geo)]])
        self.grad["mlp_col"] = torch.cat([x.reshape(-1) for x in gs[7 + len(self.sizes_geo):]])

    def direction(self, seed):
        rs = np.random.default_rng(seed)
        v = {}
        for k in self.names:
            m = rs.uniform(size=self.shapes[k]) < 0.01
            v[k] = torch.from_numpy(rs.normal(size=self.shapes[k]) * m * (0.05 if k.startswith("table") else 1.0))
        return v

    def loss(self, v, h):
        """L at the parameters shifted by h * v (v None: unshifted)."""
        p, f, t = self.params, self.fields, self.touched

        def sh(x, k):
            return x if v is None else x + h * v[k].reshape(x.shape)
        with torch.no_grad():
            ps = O.Params(pos=sh(p.pos, "pos")[t], scale_e=sh(p.scale_e, "scale_e")[t], rot_e=sh(p.rot_e, "rot_e")[t],
                          opac_e=sh(p.opac_e, "opac_e")[t], col_e=sh(p.col_e, "col_e")[t])
            mg = [None] * len(f.mlp_geo) if v is None else torch.split(v["mlp_geo"], self.sizes_geo)
            mc = [None] * len(f.mlp_col) if v is None else torch.split(v["mlp_col"], self.sizes_col)
            fs = O.Fields(table_geo=sh(f.table_geo, "table_geo"), table_rad=sh(f.table_rad, "table_rad"),
                          mlp_geo=[x if d is None else x + h * d.reshape(x.shape) for x, d in zip(f.mlp_geo, mg)],
                          mlp_col=[x if d is None else x + h * d.reshape(x.shape) for x, d in zip(f.mlp_col, mc)],
                          resolutions=f.resolutions, aabb_center=f.aabb_center, aabb_inv_half=f.aabb_inv_half,
                          bg_radius=f.bg_radius, tau_T=f.tau_T)
            rr = O.render_view(ps, fs, self.cam, O.TRAIN, pixels=self.pix)
            return float(torch.sum(rr["rgb"] * self.w))

    def dot(self, g, v):
        return sum(float(torch.sum(g[k].reshape(v[k].shape) * v[k])) for k in self.names)

    def check_fd(self, v, steps=(1e-7, 1e-8, 1e-9)):
        """Central differences along v against the oracle gradient.  Returns
        (fd, g_oracle . v, scale = sum |g_oracle * v|, usable).  The loss is
        only piecewise smooth: a grid-cell face of a moved Gaussian (a kink
        of the trilinear interpolation) or a predicate (a jump) within the
        step spoils the difference, so the step shrinks (1e-7, 1e-8, 1e-9)
        until the difference agrees to 1e-6; a direction that agrees at no
        step is reported and not usable."""
        an = self.dot(self.grad, v)
        scale = sum(float(torch.sum(torch.abs(self.grad[k] * v[k]))) for k in self.names)
        fds = []
        for h in steps:
            fd = (self.loss(v, h) - self.loss(v, -h)) / (2 * h)
            if abs(fd - an) <= 1e-6 * max(abs(fd), scale):
                return fd, an, scale, True
            fds.append(fd)
        print("direction with a kink or jump at every step: fd", fds, "oracle", an, flush=True)
        return fds[-1], an, scale, False
