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
