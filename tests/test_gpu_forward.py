"""GPU parity of the forward render step against the FP64 oracle, through
the C ABI.  Integer work (culling, hash indices, binning order) must match
bit for bit; float32 values within the stated tolerances."""
import numpy as np
import pytest
import torch

import hyrf_inputs as hi
from oracle import hyrf_oracle as O
from _hyrf_testutil import compare_image, device_scene, make, oracle_view

pytestmark = pytest.mark.gpu


def _P():
    import paper_2509_17083_amd as P
    return P


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _P()._abi.load()
    _say("device:", torch.cuda.get_device_name(0))


# ------------------------------------------------------------------ query
@pytest.mark.parametrize("cfg_name,over,table_init", [
    ("tiny", {}, 1.0),
    ("tiny", {}, None),
    ("c100k", {"n_gauss": 20000, "width": 320, "height": 240, "focal": 350.0}, 1.0),
])
def test_query_indices_and_values(cfg_name, over, table_init):
    _say("case", cfg_name, over, table_init)
    P = _P()
    cfg, scene, cams = make(cfg_name, table_init=table_init, **over)
    ds = device_scene(scene)
    q, _ = P.query_fields(ds, cams, P.TRAIN, debug_index=True)
    torch.cuda.synchronize()
    params, fields = O.from_scene(scene)
    keep = O.precull(params.pos, cams[0])
    idx = torch.nonzero(keep, as_tuple=True)[0]
    cnt = int(q["vis_count"].item())
    assert cnt == idx.numel()
    assert np.array_equal(q["vis_idx"][:cnt].cpu().numpy(), idx.numpy())
    with torch.no_grad():
        qo = O.query_gaussians(params, fields, idx, cams[0])
        x = qo["x"]
        _, ig = O.hash_encode(x, fields.table_geo, fields.resolutions, return_index=True)
        _, ir = O.hash_encode(x, fields.table_rad, fields.resolutions, return_index=True)
    dbg = q["dbg_index"][:cnt].cpu().numpy().astype(np.int64)
    assert np.array_equal(dbg[:, 0], ig.numpy()), "geometry table rows differ"
    assert np.array_equal(dbg[:, 1], ir.numpy()), "radiance table rows differ"
    # features (float32 gather vs float64)
    fg = q["feat_geo"][:cnt].cpu().double()
    fr = q["feat_rad"][:cnt].cpu().double()
    scale_f = max(1.0, float(np.abs(scene.table_rad).max()))
    assert float((fg - qo["f_geo"]).abs().max()) < 2e-6 * scale_f
    assert float((fr - qo["f_rad"]).abs().max()) < 2e-6 * scale_f
    # aggregated properties
    errs = {
        "opacity": float((q["opacity"][:cnt].cpu().double() - qo["opacity"]).abs().max()),
        "scale": float((q["scale"][:, :cnt].cpu().double().T - qo["scale"]).abs().max()),
        "quat": float((q["quat"][:, :cnt].cpu().double().T - qo["quat"]).abs().max()),
        "rgb": float((q["rgb"][0, :, :cnt].cpu().double().T - qo["rgb"]).abs().max()),
    }
    _say("query errors", errs)
    for k, e in errs.items():
        assert e < 2e-5, (k, e)


# ------------------------------------------------------------------ projection
@pytest.mark.parametrize("cfg_name,over", [
    ("tiny", {}),
    ("c100k", {"n_gauss": 20000, "width": 320, "height": 240, "focal": 350.0}),
])
def test_project_matches_oracle(cfg_name, over):
    """Depth keys bit-exact; centres within float32 rounding of u = f x / z + c
    (a few ulps of each term); conics within 1e-4 relative (they carry the
    decoders' float32 scale and rotation); rectangles hold every pixel with
    alpha >= 1/255 (brute force)."""
    P = _P()
    cfg, scene, cams = make(cfg_name, table_init=1.0, **over)
    ds = device_scene(scene)
    q, qout = P.query_fields(ds, cams, P.RENDER)
    sp, spc = P.project(ds, cams, q, qout)
    torch.cuda.synchronize()
    r = oracle_view(scene, cams[0], O.RENDER, stats=False)
    cnt = int(q["vis_count"].item())
    rec = sp["rec"][0, :cnt].cpu().double()
    pr = r["proj"]
    assert np.array_equal(sp["depth"][0, :cnt].cpu().numpy(), r["depth_key"].numpy())
    live = sp["rect"][0, :cnt].cpu().numpy()
    live = (live[:, 2] > live[:, 0]) & (live[:, 3] > live[:, 1])
    uv = torch.stack([pr["u"], pr["v"]], 1)
    # float32 u = fx * tx * (1/tz) + cx from the rounded camera-space point:
    # error below 8 ulps of the projected offset plus 8 ulps of u itself
    cxy = torch.tensor([cams[0].cx, cams[0].cy], dtype=torch.float64)
    tol = 8 * 2.0 ** -24 * ((uv - cxy).abs() + uv.abs() + cxy)
    err_uv = (rec[:, 0:2] - uv).abs()
    print("centre error max %.3e px, max error / tolerance %.3f" % (float(err_uv[live].max()),
                                                                     float((err_uv / tol)[live].max())), flush=True)
    assert bool((err_uv[live] <= tol[live]).all())
    con = pr["conic"]
    rel = ((rec[live, 2:5] - con[live]).abs() / con[live].abs().amax(1, keepdim=True)).max()
    print("conic relative error max %.3e" % float(rel), flush=True)
    assert float(rel) < 1e-4
    # rectangles hold every pixel the oracle finds with alpha >= 1/255 (brute force)
    rx, ry = O.splat_extent(pr["cov2d"], r["query"]["opacity"])
    rect = sp["rect"][0, :cnt].cpu().numpy()
    W, H = cams[0].width, cams[0].height
    for i in np.nonzero(live)[0][:200]:
        xs = np.arange(W) + 0.5
        ys = np.arange(H) + 0.5
        dx = float(pr["u"][i]) - xs[None, :]
        dy = float(pr["v"][i]) - ys[:, None]
        c = pr["conic"][i].numpy()
        a = float(r["query"]["opacity"][i]) * np.exp(-0.5 * (c[0] * dx * dx + c[2] * dy * dy) - c[1] * dx * dy)
        yy, xx = np.nonzero(a >= 1 / 255)
        if len(xx):
            assert rect[i, 0] <= xx.min() // 16 and rect[i, 2] > xx.max() // 16
            assert rect[i, 1] <= yy.min() // 16 and rect[i, 3] > yy.max() // 16
    tot = int(sp["total"].item())
    assert tot == int(((rect[:, 2] - rect[:, 0]) * (rect[:, 3] - rect[:, 1]))[live].sum())


# ------------------------------------------------------------------ binning / sort
@pytest.mark.parametrize("V,n,W,H,seed", [(1, 1, 16, 16, 3), (2, 3000, 200, 150, 5), (3, 20000, 1000, 700, 9)])
def test_bin_sort_bit_exact(V, n, W, H, seed):
    P = _P()
    from paper_2509_17083_amd import _abi as A
    depth, rect, tw, th = hi.make_splat_records(V, n, W, H, seed=seed)
    keys_o, ids_o, ranges_o = O.bin_and_sort(torch.from_numpy(depth), torch.from_numpy(rect), tw, th)
    dev = "cuda"
    d_depth = torch.from_numpy(depth).to(dev)
    d_rect = torch.from_numpy(rect).to(dev)
    count = torch.tensor([n], dtype=torch.int32, device=dev)
    total = torch.zeros(1, dtype=torch.int64, device=dev)
    spc = A.hyrf_splats(n, count.data_ptr(), None, d_rect.data_ptr(), d_depth.data_ptr(), total.data_ptr())
    cams = [hi.look_at((0, -3, 0), (0, 0, 0), 100.0, W, H)] * V
    ne = int(keys_o.numel())
    keys, vals, ranges = P.bin_sort(cams, spc, n, ne, want_keys=True)
    torch.cuda.synchronize()
    assert np.array_equal(vals[:ne].cpu().numpy().astype(np.int64), ids_o.numpy())
    assert np.array_equal(keys[:ne].cpu().numpy().astype(np.int64), keys_o.numpy())
    assert np.array_equal(ranges.cpu().numpy().astype(np.int64), ranges_o.numpy())


def test_bin_sort_large_order_by_definition():
    """4.5M splats (85% with an empty rectangle) and ~7M tile entries: both
    radix sorts run more than 1024 workgroups, so each digit's offsets are
    scanned over several chunks.  The oracle's per-entry loops are too slow
    at this size; the result is checked against the order's definition
    (entries by view, tile, depth, splat index), built here with numpy's
    lexsort, bit for bit."""
    P = _P()
    from paper_2509_17083_amd import _abi as A
    V, n, W, H = 1, 4_500_000, 1920, 1080
    depth, rect, tw, th = hi.make_splat_records(V, n, W, H, seed=21)
    empty = np.random.Generator(np.random.PCG64(22)).uniform(size=(V, n)) < 0.85
    rect[..., 2] = np.where(empty, rect[..., 0], rect[..., 2])
    r = rect.reshape(-1, 4).astype(np.int64)
    w, h = r[:, 2] - r[:, 0], r[:, 3] - r[:, 1]
    cnt = np.where((w > 0) & (h > 0), w * h, 0)
    sid = np.repeat(np.arange(V * n, dtype=np.int64), cnt)
    j = np.arange(sid.size, dtype=np.int64) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    tile = (r[sid, 1] + j // w[sid]) * tw + (r[sid, 0] + j % w[sid])
    key = (sid // n) * (tw * th) + tile
    order = np.lexsort((sid, depth.reshape(-1)[sid], key))
    keys_e, ids_e = key[order], sid[order]
    ne = int(keys_e.size)
    k = np.arange(V * tw * th)
    lo, hi_ = np.searchsorted(keys_e, k, "left"), np.searchsorted(keys_e, k, "right")
    ranges_e = np.stack([np.where(hi_ > lo, lo, 0), np.where(hi_ > lo, hi_, 0)], axis=1)
    _say("large bin/sort:", V * n, "splats,", ne, "entries")

    count = torch.tensor([n], dtype=torch.int32, device="cuda")
    d_rect = torch.from_numpy(rect).cuda()
    d_depth = torch.from_numpy(depth).cuda()
    spc = A.hyrf_splats(n, count.data_ptr(), None, d_rect.data_ptr(), d_depth.data_ptr(), None)
    cams = [hi.look_at((0, -3, 0), (0, 0, 0), 100.0, W, H)] * V
    keys, vals, ranges = P.bin_sort(cams, spc, n, ne, want_keys=True)
    torch.cuda.synchronize()
    assert np.array_equal(keys[:ne].cpu().numpy().astype(np.int64), keys_e)
    assert np.array_equal(vals[:ne].cpu().numpy().astype(np.int64), ids_e)
    assert np.array_equal(ranges.cpu().numpy().astype(np.int64), ranges_e)


def test_bin_sort_capacity_error():
    P = _P()
    from paper_2509_17083_amd import _abi as A
    depth, rect, tw, th = hi.make_splat_records(1, 100, 64, 64, seed=1)
    count = torch.tensor([100], dtype=torch.int32, device="cuda")
    d_rect = torch.from_numpy(rect).cuda()
    d_depth = torch.from_numpy(depth).cuda()
    spc = A.hyrf_splats(100, count.data_ptr(), None, d_rect.data_ptr(), d_depth.data_ptr(), None)
    cams = [hi.look_at((0, -3, 0), (0, 0, 0), 100.0, 64, 64)]
    with pytest.raises(A.HyrfError) as e:
        P.bin_sort(cams, spc, 100, 50, capacity=10)
    assert e.value.status == A.HYRF_ERR_CAPACITY


# ------------------------------------------------------------------ whole forward
@pytest.mark.parametrize("mode", [O.TRAIN, O.RENDER])
@pytest.mark.parametrize("cfg_name,over,table_init,scale_shift", [
    ("tiny", {}, None, 0.0),
    ("tiny", {}, 1.0, 1.0),
    ("c100k", {"n_gauss": 20000, "width": 250, "height": 190, "focal": 300.0, "log2_T_rad": 16}, 1.0, 1.0),
])
def test_render_matches_oracle(mode, cfg_name, over, table_init, scale_shift):
    _say("case", mode, cfg_name, over, table_init, scale_shift)
    P = _P()
    cfg, scene, cams = make(cfg_name, table_init=table_init, **over)
    scene.scale_e += np.float32(scale_shift)
    ds = device_scene(scene)
    st = P.render(ds, cams, mode)
    torch.cuda.synchronize()
    r = oracle_view(scene, cams[0], mode)
    H, W = cams[0].height, cams[0].width
    res = compare_image(st.image[0].cpu().numpy(), r, mode, H, W, gpu_T=st.T[0].cpu().numpy())
    _say("image", res, "entries", st.n_entries)
    assert res["ok"], res
    T_ref = r["T"].numpy().reshape(H, W)
    assert float(np.abs(st.T[0].cpu().numpy() - T_ref).max()) < 1e-4


def test_render_empty_scene_is_background():
    P = _P()
    cfg, scene, cams = make("tiny", table_init=1.0)
    scene.pos[1, :] = -10.0        # every Gaussian behind the camera
    ds = device_scene(scene)
    for mode in (O.TRAIN, O.RENDER):
        st = P.render(ds, cams, mode)
        torch.cuda.synchronize()
        assert int(st.query["vis_count"].item()) == 0 and st.n_entries == 0
        r = oracle_view(scene, cams[0], mode)
        res = compare_image(st.image[0].cpu().numpy(), r, mode, 64, 64)
        assert res["ok"], res


@pytest.mark.parametrize("cfg_name,over,n_views,late", [
    ("tiny", {}, 1, False),
    ("c100k", {"n_gauss": 20000, "width": 320, "height": 240, "focal": 350.0}, 3, False),
    ("c100k", {"n_gauss": 20000, "width": 320, "height": 240, "focal": 350.0}, 3, True),
])
def test_train_background_on_a_second_stream_equals_one_stream(cfg_name, over, n_views, late):
    """The train-mode forward with the background on a second stream (the
    default) against the one-stream forward: every output bit-identical,
    also with several views in one launch, with the background started
    after the field query or (`late`) after binning."""
    _say("case", cfg_name, over, n_views, late)
    P = _P()
    ws = P.Workspace()
    ws.bg_late = late
    cfg, scene, cams = make(cfg_name, table_init=1.0, **over)
    if n_views > 1:
        cams = hi.make_cameras(hi.with_overrides(cfg, n_views=n_views), seed=3004)
    scene.scale_e += np.float32(1.0)
    ds = device_scene(scene)
    a = P.render(ds, cams, P.TRAIN, overlap=True, ws=ws)
    b = P.render(ds, cams, P.TRAIN, overlap=False)
    torch.cuda.synchronize()
    assert a.n_entries == b.n_entries
    assert torch.equal(a.bg, b.bg) and torch.equal(a.bg_feat, b.bg_feat) and torch.equal(a.T, b.T)
    assert torch.equal(a.last, b.last)
    # c_fg + T c_s: one fused multiply-add in both
    assert torch.equal(a.image, b.image)


def test_forward_is_deterministic():
    P = _P()
    cfg, scene, cams = make("tiny", table_init=1.0)
    scene.scale_e += np.float32(1.0)
    ds = device_scene(scene)
    a = P.render(ds, cams, P.TRAIN)
    b = P.render(ds, cams, P.TRAIN)
    torch.cuda.synchronize()
    assert torch.equal(a.image, b.image) and torch.equal(a.T, b.T) and torch.equal(a.last, b.last)


def test_spatial_order_is_a_permutation_and_render_is_unchanged():
    P = _P()
    cfg, scene, cams = make("tiny", table_init=1.0)
    scene.scale_e += np.float32(1.0)
    ds = device_scene(scene)
    perm = ds.spatial_order()
    torch.cuda.synchronize()
    p = perm.cpu().numpy()
    assert np.array_equal(np.sort(p), np.arange(scene.n))
    # neighbours in the new order are closer in space than in the seeded order
    pos = scene.pos.T
    d_new = np.linalg.norm(pos[p[1:]] - pos[p[:-1]], axis=1).mean()
    d_old = np.linalg.norm(pos[1:] - pos[:-1], axis=1).mean()
    assert d_new < 0.5 * d_old
    # the reordered scene renders like the oracle of the reordered scene
    import copy
    sc2 = copy.deepcopy(scene)
    sc2.pos, sc2.scale_e, sc2.rot_e = scene.pos[:, p].copy(), scene.scale_e[:, p].copy(), scene.rot_e[:, p].copy()
    sc2.opac_e, sc2.col_e = scene.opac_e[p].copy(), scene.col_e[:, p].copy()
    st = P.render(ds.reordered(perm), cams, P.TRAIN)
    torch.cuda.synchronize()
    r = oracle_view(sc2, cams[0], O.TRAIN)
    res = compare_image(st.image[0].cpu().numpy(), r, O.TRAIN, 64, 64)
    assert res["ok"], res


@pytest.mark.timeout(900)
@pytest.mark.parametrize("mode", [O.TRAIN, O.RENDER])
def test_full_size_1080p_sampled_pixels(mode):
    """The benchmark's launch configuration -- 1M Gaussians stored in Morton
    order, tables 2^21 / 2^20, 1920x1080, every tile -- against the oracle
    of the same (reordered) scene evaluated on 384 seeded pixels."""
    from oracle import parity
    P = _P()
    cfg = hi.CONFIGS["c1m"]
    scene = hi.make_scene(cfg)
    cam = hi.make_cameras(cfg)[0]
    ds = device_scene(scene)
    perm = ds.spatial_order()
    ds = ds.reordered(perm)
    st = P.render(ds, [cam], mode)
    torch.cuda.synchronize()
    img = st.image[0].cpu().numpy()
    T_gpu = st.T[0].cpu().numpy()
    _say("entries", st.n_entries)
    scene = _permuted(scene, perm.cpu().numpy())
    rng = np.random.default_rng(23)
    px = rng.integers(0, cam.width, 384)
    py = rng.integers(0, cam.height, 384)
    params, fields = O.from_scene(scene)
    with torch.no_grad():
        r = O.render_view(params, fields, cam, mode, pixels=torch.from_numpy(np.stack([px, py], 1)).long(),
                          return_stats=True)
    res = parity.compare_pixels(img[:, py, px].T, r, gpu_T=T_gpu[py, px])
    _say("sampled pixels", res)
    assert res["ok"], res
    assert float(np.abs(T_gpu[py, px] - r["T"].numpy()).max()) <= 1e-4


def _permuted(scene, p):
    import copy
    sc2 = copy.deepcopy(scene)
    sc2.pos, sc2.scale_e = scene.pos[:, p].copy(), scene.scale_e[:, p].copy()
    sc2.rot_e = None if scene.rot_e is None else scene.rot_e[:, p].copy()
    sc2.opac_e, sc2.col_e = scene.opac_e[p].copy(), scene.col_e[:, p].copy()
    return sc2


def test_render_with_no_gaussians_is_the_background_and_its_gradient():
    """n = 0 (empty explicit arrays): the image is the neural background in
    both modes, and the adjoint reaches only the radiance table and the
    colour decoder, as in the oracle."""
    import copy
    P = _P()
    cfg, scene, cams = make("tiny", table_init=1.0)
    s0 = copy.deepcopy(scene)
    s0.pos, s0.scale_e, s0.rot_e = scene.pos[:, :0].copy(), scene.scale_e[:, :0].copy(), scene.rot_e[:, :0].copy()
    s0.opac_e, s0.col_e = scene.opac_e[:0].copy(), scene.col_e[:, :0].copy()
    ds = device_scene(s0)
    assert ds.n == 0
    for mode in (O.TRAIN, O.RENDER):
        st = P.render(ds, cams, mode)
        torch.cuda.synchronize()
        assert int(st.query["vis_count"].item()) == 0 and st.n_entries == 0
        r = oracle_view(s0, cams[0], mode)
        res = compare_image(st.image[0].cpu().numpy(), r, mode, 64, 64)
        assert res["ok"], res
    w = torch.from_numpy(hi.make_target_image((1, 3, 64, 64), seed=12) - 0.5)
    st = P.render(ds, cams, P.TRAIN)
    g = P.render_backward(ds, cams, st, w.float().cuda())
    torch.cuda.synchronize()
    params, fields = O.from_scene(s0, requires_grad=True)
    r = O.render_view(params, fields, cams[0], O.TRAIN)
    L = torch.sum(r["rgb"].T.reshape(3, 64, 64) * w[0].double())
    gt, *gm = torch.autograd.grad(L, [fields.table_rad] + list(fields.mlp_col))
    e_t = float((g["table_rad"].cpu().double() - gt).norm() / gt.norm())
    e_m = float((g["mlp_col"].cpu().double() - torch.cat([x.reshape(-1) for x in gm])).norm() /
                torch.cat([x.reshape(-1) for x in gm]).norm())
    print("no Gaussians: gradient relative L2 table_rad %.2e mlp_col %.2e" % (e_t, e_m), flush=True)
    assert e_t < 1e-3 and e_m < 1e-3
    assert float(g["table_geo"].abs().max()) == 0.0 and float(g["mlp_geo"].abs().max()) == 0.0
