"""Batched views: several cameras in one launch (shared field query, per-view
colour, projection, binning, blending and background; the backward sums over
views).  Each view is compared with the FP64 oracle's render of that view,
and the gradient of a loss summed over views with the oracle's."""
import numpy as np
import pytest
import torch

import hyrf_inputs as hi
from oracle import hyrf_oracle as O
from _hyrf_testutil import compare_image, device_scene, knife_mask, make, oracle_view

pytestmark = pytest.mark.gpu


def _P():
    import paper_2509_17083_amd as P
    return P


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _P()._abi.load()


def _views(cfg, n, seed=3004):
    return hi.make_cameras(hi.with_overrides(cfg, n_views=n), seed=seed)


@pytest.mark.parametrize("mode", [O.TRAIN, O.RENDER])
def test_batched_views_match_per_view_oracle(mode):
    P = _P()
    cfg, scene, _ = make("tiny", table_init=1.0)
    scene.scale_e += np.float32(1.0)
    cams = _views(cfg, 3)
    st = P.render(device_scene(scene), cams, mode)
    torch.cuda.synchronize()
    for v, cam in enumerate(cams):
        r = oracle_view(scene, cam, mode)
        res = compare_image(st.image[v].cpu().numpy(), r, mode, cam.height, cam.width)
        print("view", v, res, flush=True)
        assert res["ok"], (v, res)


def test_batched_views_gradient():
    P = _P()
    cfg, scene, _ = make("tiny", table_init=1.0)
    scene.scale_e += np.float32(1.0)
    cams = _views(cfg, 2)
    params, fields = O.from_scene(scene, requires_grad=True)
    L = 0.0
    ws = []
    for v, cam in enumerate(cams):
        r = O.render_view(params, fields, cam, O.TRAIN, return_stats=True)
        knife = knife_mask(r, O.TRAIN).reshape(cam.height, cam.width)
        w = torch.from_numpy(hi.make_target_image((3, cam.height, cam.width), seed=40 + v) - 0.5).double()
        w = w * (~knife).double()[None]
        L = L + torch.sum(r["rgb"].T.reshape(3, cam.height, cam.width) * w)
        ws.append(w.float())
    leaves = [params.pos, params.scale_e, params.rot_e, params.opac_e, params.col_e, fields.table_geo,
              fields.table_rad] + fields.mlp_geo + fields.mlp_col
    gs = torch.autograd.grad(L, leaves, allow_unused=True)
    ref = dict(pos=gs[0], scale_e=gs[1], rot_e=gs[2], opac_e=gs[3], col_e=gs[4], table_geo=gs[5], table_rad=gs[6],
               mlp_geo=torch.cat([g.reshape(-1) for g in gs[7:7 + len(fields.mlp_geo)]]),
               mlp_col=torch.cat([g.reshape(-1) for g in gs[7 + len(fields.mlp_geo):]]))
    ds = device_scene(scene)
    st = P.render(ds, cams, P.TRAIN)
    gr = P.render_backward(ds, cams, st, torch.stack(ws).cuda())
    torch.cuda.synchronize()
    for k, r in ref.items():
        g = gr[k].detach().cpu().double()
        if k in ("pos", "scale_e", "rot_e", "col_e"):
            g = g.T
        r = r.reshape(g.shape)
        e = float((g - r).norm() / r.norm())
        print(k, f"{e:.2e}", flush=True)
        assert e < 1e-3, (k, e)


def _permuted(scene, p):
    import copy
    sc2 = copy.deepcopy(scene)
    sc2.pos, sc2.scale_e = scene.pos[:, p].copy(), scene.scale_e[:, p].copy()
    sc2.rot_e = None if scene.rot_e is None else scene.rot_e[:, p].copy()
    sc2.opac_e, sc2.col_e = scene.opac_e[p].copy(), scene.col_e[:, p].copy()
    return sc2


@pytest.mark.timeout(900)
def test_batched_views_full_size_sampled_pixels():
    """The batched-view workload as the benchmark launches it: 3M Gaussians
    (Morton order), 8 views of 1280x720 in one launch.  View 0 of the train
    render and view 5 of the render-mode frame against the FP64 oracle of
    that view on 256 seeded pixels each."""
    from oracle import parity
    P = _P()
    cfg = hi.CONFIGS["c3m_8v"]
    scene = hi.make_scene(cfg)
    cams = hi.make_cameras(cfg)
    assert len(cams) == 8
    ds = device_scene(scene)
    perm = ds.spatial_order()
    ds = ds.reordered(perm)
    scene = _permuted(scene, perm.cpu().numpy())
    params, fields = O.from_scene(scene)
    rng = np.random.default_rng(29)
    for mode, v in ((O.TRAIN, 0), (O.RENDER, 5)):
        st = P.render(ds, cams, mode)
        torch.cuda.synchronize()
        print("mode", mode, "entries", st.n_entries, flush=True)
        img = st.image[v].cpu().numpy()
        T_gpu = st.T[v].cpu().numpy()
        del st
        cam = cams[v]
        px = rng.integers(0, cam.width, 256)
        py = rng.integers(0, cam.height, 256)
        with torch.no_grad():
            r = O.render_view(params, fields, cam, mode, pixels=torch.from_numpy(np.stack([px, py], 1)).long(),
                              return_stats=True)
        res = parity.compare_pixels(img[:, py, px].T, r, gpu_T=T_gpu[py, px])
        print("view", v, "sampled pixels", {k: res[k] for k in ("max_err", "n_flip", "n_bad", "T_rel_err_max")},
              flush=True)
        assert res["ok"], res
        assert float(np.abs(T_gpu[py, px] - r["T"].numpy()).max()) <= 1e-4


def test_batched_views_gradient_720p():
    """Gradient of a loss over two 1280x720 views rendered in one launch (the
    colour decoder's first layer shared over the views) on a 20k-Gaussian
    scene with the batched-view distributions: L = sum over views of
    sum(w_v * C_v) on 2048 seeded pixels per view (knife-edge pixels weighted
    0), every parameter tensor against the FP64 oracle's autograd gradient.
    Bar: per-tensor relative L2 <= 1e-3."""
    P = _P()
    cfg = hi.with_overrides(hi.CONFIGS["c3m_8v"], n_gauss=20000, n_views=2)
    scene = hi.make_scene(cfg, table_init=1.0)
    scene.scale_e += np.float32(1.5)
    cams = hi.make_cameras(cfg)
    assert len(cams) == 2
    H, W = cams[0].height, cams[0].width
    params, fields = O.from_scene(scene, requires_grad=True)
    rng = np.random.default_rng(47)
    L = 0.0
    dL = torch.zeros(2, 3, H, W, dtype=torch.float64)
    for v, cam in enumerate(cams):
        flat = rng.choice(H * W, 2048, replace=False)
        pix = torch.from_numpy(np.stack([flat % W, flat // W], 1)).long()
        r = O.render_view(params, fields, cam, O.TRAIN, pixels=pix, return_stats=True)
        knife = knife_mask(r, O.TRAIN)
        w = torch.from_numpy(rng.normal(size=(2048, 3))) * (~knife).double()[:, None]
        L = L + torch.sum(r["rgb"] * w)
        dL[v, :, pix[:, 1], pix[:, 0]] = w.T
        print("view", v, "knife pixels", int(knife.sum()), flush=True)
    leaves = [params.pos, params.scale_e, params.rot_e, params.opac_e, params.col_e, fields.table_geo,
              fields.table_rad] + fields.mlp_geo + fields.mlp_col
    gs = torch.autograd.grad(L, leaves, allow_unused=True)
    ref = dict(pos=gs[0], scale_e=gs[1], rot_e=gs[2], opac_e=gs[3], col_e=gs[4], table_geo=gs[5], table_rad=gs[6],
               mlp_geo=torch.cat([g.reshape(-1) for g in gs[7:7 + len(fields.mlp_geo)]]),
               mlp_col=torch.cat([g.reshape(-1) for g in gs[7 + len(fields.mlp_geo):]]))
    ds = device_scene(scene)
    st = P.render(ds, cams, P.TRAIN)
    gr = P.render_backward(ds, cams, st, dL.float().cuda())
    torch.cuda.synchronize()
    for k, r in ref.items():
        g = gr[k].detach().cpu().double()
        if k in ("pos", "scale_e", "rot_e", "col_e"):
            g = g.T
        r = r.reshape(g.shape)
        e = float((g - r).norm() / r.norm())
        print(k, f"{e:.2e}", flush=True)
        assert e < 1e-3, (k, e)
