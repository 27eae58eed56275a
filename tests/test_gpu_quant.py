"""GPU parity of the compressed-model render (Sec. 4.3: hash tables stored as
8-bit min-max codes and decoded inside the gather) against the oracle,
through the C ABI.  The codes are integers decided in float32 on both sides
and must match bit for bit; the render is compared with the FP64 oracle fed
the exactly decoded tables, to the same tolerances as the float32 render."""
import copy
import ctypes

import numpy as np
import pytest
import torch

import hyrf_inputs as hi
from oracle import compress_oracle as QO
from oracle import hyrf_oracle as O
from _hyrf_testutil import compare_image, make, oracle_view

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2509_17083_amd as P
    P._abi.load()


def _quantize_gpu(table):
    from paper_2509_17083_amd import _abi as A
    lib = A.load()
    t = torch.from_numpy(np.ascontiguousarray(table)).cuda()
    L, T = table.shape[0], table.shape[1]
    log2_T = int(T).bit_length() - 1
    codes = torch.empty(t.shape, dtype=torch.uint8, device="cuda")
    qp = torch.empty(L, 2, dtype=torch.float32, device="cuda")
    w = torch.empty(max(lib.hyrf_quantize_workspace_bytes(L, log2_T), 256), dtype=torch.uint8, device="cuda")
    vp = lambda x: ctypes.c_void_p(x.data_ptr())  # noqa: E731
    A.check("hyrf_quantize_table", lib.hyrf_quantize_table(vp(t), L, log2_T, vp(codes), vp(qp), vp(w), w.numel(),
                                                           None))
    torch.cuda.synchronize()
    return codes.cpu().numpy(), qp.cpu().numpy()


@pytest.mark.parametrize("L,log2_T,seed,scale", [(1, 1, 1, 1.0), (3, 10, 2, 1e-4), (16, 14, 3, 1.0),
                                                 (16, 21, 4, 1e-4)])
def test_quantize_bit_exact(L, log2_T, seed, scale):
    _say("case", L, log2_T, seed)
    rng = np.random.default_rng(seed)
    table = rng.uniform(-scale, scale, size=(L, 1 << log2_T, 2)).astype(np.float32)
    if L >= 3:
        table[1] = np.float32(0.5)          # a constant level (step 0)
    codes, qp = _quantize_gpu(table)
    codes_o, qp_o = QO.quantize_table(table)
    assert np.array_equal(qp, qp_o)
    assert np.array_equal(codes, codes_o)


def _quant_scene(scene):
    """The scene with both tables replaced by their exactly decoded 8-bit
    codes (what the oracle renders)."""
    sq = copy.deepcopy(scene)
    cg, qg = QO.quantize_table(scene.table_geo)
    cr, qr = QO.quantize_table(scene.table_rad)
    return sq, QO.dequantize_table(cg, qg), QO.dequantize_table(cr, qr)


def _oracle_quant(scene, cam, mode):
    sq, dg, dr = _quant_scene(scene)
    params, fields = O.from_scene(sq)
    fields.table_geo = torch.from_numpy(dg)
    fields.table_rad = torch.from_numpy(dr)
    with torch.no_grad():
        return O.render_view(params, fields, cam, mode, return_stats=True), params, fields


@pytest.mark.parametrize("mode", [O.TRAIN, O.RENDER])
@pytest.mark.parametrize("cfg_name,over,table_init,scale_shift", [
    ("tiny", {}, 1.0, 1.0),
    ("c100k", {"n_gauss": 20000, "width": 250, "height": 190, "focal": 300.0, "log2_T_rad": 16}, 1.0, 1.0),
])
def test_quantized_render_matches_oracle(mode, cfg_name, over, table_init, scale_shift):
    _say("case", mode, cfg_name, over)
    import paper_2509_17083_amd as P
    cfg, scene, cams = make(cfg_name, table_init=table_init, **over)
    scene.scale_e += np.float32(scale_shift)
    ds = P.DeviceScene.from_host(scene).quantized()
    st = P.render(ds, cams, mode)
    torch.cuda.synchronize()
    r, _, _ = _oracle_quant(scene, cams[0], mode)
    H, W = cams[0].height, cams[0].width
    res = compare_image(st.image[0].cpu().numpy(), r, mode, H, W)
    _say("image", res)
    assert res["ok"], res


def test_quantized_query_features():
    import paper_2509_17083_amd as P
    cfg, scene, cams = make("tiny", table_init=1.0)
    ds = P.DeviceScene.from_host(scene).quantized()
    q, _ = P.query_fields(ds, cams, P.TRAIN, debug_index=True)
    torch.cuda.synchronize()
    _, params, fields = _oracle_quant(scene, cams[0], O.TRAIN)
    keep = O.precull(params.pos, cams[0])
    idx = torch.nonzero(keep, as_tuple=True)[0]
    cnt = int(q["vis_count"].item())
    assert cnt == idx.numel()
    with torch.no_grad():
        qo = O.query_gaussians(params, fields, idx, cams[0])
    fg = q["feat_geo"][:cnt].cpu().double()
    fr = q["feat_rad"][:cnt].cpu().double()
    e = max(float((fg - qo["f_geo"]).abs().max()), float((fr - qo["f_rad"]).abs().max()))
    _say("feature error", e)
    assert e < 2e-6


def test_quantized_tables_have_no_backward():
    import paper_2509_17083_amd as P
    from paper_2509_17083_amd import _abi as A
    cfg, scene, cams = make("tiny", table_init=1.0)
    ds = P.DeviceScene.from_host(scene).quantized()
    st = P.render(ds, cams, P.TRAIN)
    dL = torch.ones_like(st.image)
    with pytest.raises(A.HyrfError) as e:
        P.render_backward(ds, cams, st, dL)
    assert e.value.status == A.HYRF_ERR_UNSUPPORTED


def _half_positions(scene):
    """The scene with its positions rounded to float16 (nearest even) and
    widened back: what a render from float16 positions sees."""
    sr = copy.deepcopy(scene)
    sr.pos = scene.pos.astype(np.float16).astype(np.float32)
    return sr


MID = {"n_gauss": 20000, "width": 250, "height": 190, "focal": 300.0, "log2_T_rad": 16}


@pytest.mark.parametrize("mode", [O.TRAIN, O.RENDER])
def test_half_positions_render(mode):
    """Positions stored in float16 (Sec. 4.3, compressed model), widened
    where the cull, the query and the projection read them: the render
    equals, bit for bit, the float32 render of the rounded positions, and
    matches the FP64 oracle of the rounded scene; with 8-bit tables as well
    (the whole compressed model) it matches the oracle fed both."""
    import paper_2509_17083_amd as P
    cfg, scene, cams = make("c100k", table_init=1.0, **MID)
    scene.scale_e += np.float32(1.0)
    H, W = cams[0].height, cams[0].width
    ds = P.DeviceScene.from_host(scene)
    d16 = ds.with_half_positions()
    sr = _half_positions(scene)
    dr = P.DeviceScene.from_host(sr)
    a = P.render(d16, cams, mode)
    b = P.render(dr, cams, mode)
    torch.cuda.synchronize()
    assert int(a.query["vis_count"].item()) == int(b.query["vis_count"].item())
    assert torch.equal(a.image, b.image) and torch.equal(a.T, b.T)
    res = compare_image(a.image[0].cpu().numpy(), oracle_view(sr, cams[0], mode), mode, H, W)
    _say("half positions", res)
    assert res["ok"], res
    # the whole compressed model: float16 positions and 8-bit tables
    dq = ds.quantized().with_half_positions()
    c = P.render(dq, cams, mode)
    torch.cuda.synchronize()
    r, _, _ = _oracle_quant(sr, cams[0], mode)
    res = compare_image(c.image[0].cpu().numpy(), r, mode, H, W)
    _say("half positions + 8-bit tables", res)
    assert res["ok"], res


def test_half_positions_have_no_backward():
    import paper_2509_17083_amd as P
    from paper_2509_17083_amd import _abi as A
    cfg, scene, cams = make("tiny", table_init=1.0)
    ds = P.DeviceScene.from_host(scene).with_half_positions()
    st = P.render(ds, cams, P.TRAIN)
    with pytest.raises(A.HyrfError) as e:
        P.render_backward(ds, cams, st, torch.ones_like(st.image))
    assert e.value.status == A.HYRF_ERR_UNSUPPORTED
