"""GPU parity of the training-loop steps after the backward (Sec. 3.4):
fused Adam over several tensors, the densification statistics accumulated by
the projection adjoint, the densify / prune decisions and the opacity reset,
against the oracle, through the C ABI."""
import numpy as np
import pytest
import torch

from oracle import hyrf_oracle as O
from oracle import train_oracle as TO
from _hyrf_testutil import knife_mask, make

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def f32(x):
    return float(np.float32(x))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2509_17083_amd as P
    P._abi.load()


# ---------------------------------------------------------------- Adam
def test_adam_matches_oracle_over_steps():
    """Groups of ragged sizes (one empty) with different learning rates; three
    steps with fresh seeded gradients.  float32 kernel vs float64 oracle from
    the same float32 start values."""
    import paper_2509_17083_amd as P
    rng = np.random.default_rng(5)
    sizes, lrs = [4097, 3, 0, 100_000, 16], [1e-3, 0.1, 1e-2, 1.6e-4, 5e-3]
    host = [dict(p=rng.normal(size=n).astype(np.float32), m=np.zeros(n), v=np.zeros(n)) for n in sizes]
    dev = [dict(param=torch.from_numpy(h["p"].copy()).cuda(), grad=torch.zeros(n, device="cuda"),
                m=torch.zeros(n, device="cuda"), v=torch.zeros(n, device="cuda"), lr=lr,
                param_half=torch.zeros(n, dtype=torch.float16, device="cuda"))
           for h, n, lr in zip(host, sizes, lrs)]
    ref = [dict(p=h["p"].astype(np.float64), m=h["m"], v=h["v"]) for h in host]
    # EMA of |g|: the magnitude of the terms that m sums (and may cancel)
    mscale = [np.zeros(n) for n in sizes]
    for t in range(1, 4):
        for k, n in enumerate(sizes):
            g = (rng.normal(size=n) * 10.0 ** rng.uniform(-5, 0, size=n)).astype(np.float32)
            dev[k]["grad"].copy_(torch.from_numpy(g))
            mscale[k] = 0.9 * mscale[k] + 0.1 * np.abs(g)
            # the hyper-parameters cross the C ABI as float32: the oracle takes
            # the same float32 values
            ref[k]["p"], ref[k]["m"], ref[k]["v"] = TO.adam_step(ref[k]["p"], g, ref[k]["m"], ref[k]["v"], t,
                                                                 f32(lrs[k]), f32(0.9), f32(0.999), f32(1e-15))
        P.adam_step(dev, t, 0.9, 0.999, 1e-15, zero_grad=True)
        torch.cuda.synchronize()
        for k, n in enumerate(sizes):
            if n == 0:
                continue
            p = dev[k]["param"].cpu().double().numpy()
            # the float32 parameter is rounded once per step (half an ulp,
            # <= 6e-8 |p|), the update itself carries ~1e-6 relative error
            tol = t * (6e-8 * np.abs(ref[k]["p"]) + 1e-5 * lrs[k])
            ratio = np.abs(p - ref[k]["p"]) / tol
            _say("step", t, "group", k, "max error / tolerance", float(ratio.max()))
            assert float(ratio.max()) <= 1.0
            m_err = np.abs(dev[k]["m"].cpu().double().numpy() - ref[k]["m"])
            assert np.all(m_err <= 1e-6 * t * mscale[k])
            assert np.allclose(dev[k]["v"].cpu().double().numpy(), ref[k]["v"], rtol=1e-5, atol=1e-20)
            assert not dev[k]["grad"].any()
            assert torch.equal(dev[k]["param_half"], dev[k]["param"].half())


# ---------------------------------------------------------------- densification statistics
def test_densification_stats_match_oracle_gradients():
    import paper_2509_17083_amd as P
    cfg, scene, cams = make("tiny", table_init=1.0)
    scene.scale_e += np.float32(1.0)
    cam = cams[0]
    H, W = cam.height, cam.width
    w_img = np.random.default_rng(7).normal(size=(3, H, W)).astype(np.float32)
    params, fields = O.from_scene(scene, requires_grad=True)
    r = O.render_view(params, fields, cam, O.TRAIN, return_stats=True)
    knife = knife_mask(r, O.TRAIN).reshape(H, W)
    w = torch.from_numpy(w_img).double() * (~knife).double()[None]
    L = torch.sum(r["rgb"].T.reshape(3, H, W) * w)
    du, dv = torch.autograd.grad(L, [r["proj"]["u"], r["proj"]["v"]])
    ds = P.DeviceScene.from_host(scene)
    st = P.render(ds, cams, P.TRAIN)
    n = scene.n
    grads = dict(dens_accum=torch.zeros(n, device="cuda"), dens_count=torch.zeros(n, device="cuda"))
    dL = torch.from_numpy(w.float().numpy()).cuda()[None].contiguous()
    for _ in range(2):   # accumulates over calls
        P.render_backward(ds, cams, st, dL, grads=grads)
    torch.cuda.synchronize()
    cnt = int(st.query["vis_count"].item())
    vis = st.query["vis_idx"][:cnt].cpu().numpy()
    assert np.array_equal(vis, r["vis_idx"].numpy())
    rect = st.splats["rect"][0, :cnt].cpu().numpy()
    fp = (rect[:, 2] > rect[:, 0]) & (rect[:, 3] > rect[:, 1])
    acc_o, cnt_o = TO.densification_stats(du.numpy(), dv.numpy(), W, H, fp)
    acc = grads["dens_accum"].cpu().double().numpy()[vis]
    c = grads["dens_count"].cpu().numpy()[vis]
    assert np.array_equal(c, 2 * cnt_o)
    rel = np.linalg.norm(acc - 2 * acc_o) / np.linalg.norm(2 * acc_o)
    _say("densification accum rel L2", rel, "footprints", int(fp.sum()))
    assert rel < 1e-3
    # Gaussians culled before the query gather nothing
    mask = np.ones(n, bool)
    mask[vis] = False
    assert not grads["dens_accum"].cpu().numpy()[mask].any()


# ---------------------------------------------------------------- decisions, reset
def test_densify_masks_and_reset_match_oracle():
    import paper_2509_17083_amd as P
    from paper_2509_17083_amd import _abi as A
    cfg, scene, cams = make("tiny", table_init=1.0)
    scene.opac_e -= np.float32(3.0)          # some Gaussians below the prune opacity
    ds = P.DeviceScene.from_host(scene)
    st = P.render(ds, cams, P.TRAIN)
    n = scene.n
    rng = np.random.default_rng(9)
    acc = (rng.uniform(0, 1e-3, size=n)).astype(np.float32)
    cnt = rng.integers(0, 4, size=n).astype(np.float32)
    flags = P.densify_masks(st, n, torch.from_numpy(acc).cuda(), torch.from_numpy(cnt).cuda(),
                            grad_threshold=2e-4, dense_extent=0.02, min_opacity=0.005)
    torch.cuda.synchronize()
    k = int(st.query["vis_count"].item())
    vis = st.query["vis_idx"][:k].cpu().numpy()
    op = st.query["opacity"][:k].cpu().numpy()
    smax = st.query["scale"][:, :k].cpu().numpy().max(axis=0)
    ref = np.zeros(n, np.uint8)
    ref[vis] = TO.densify_flags(acc[vis], cnt[vis], op, smax, 2e-4, 0.02, 0.005)
    f = flags.cpu().numpy()
    _say("flags", {b: int(((f & b) > 0).sum()) for b in (1, 2, 4, 8)})
    assert np.array_equal(f, ref)
    assert ((f & A.HYRF_PRUNE) > 0).any() and ((f & A.HYRF_SPLIT) > 0).any()
    oe = ds.opac_e.clone()
    P.reset_opacity(oe, 0.01)
    torch.cuda.synchronize()
    assert np.array_equal(oe.cpu().numpy(), TO.reset_opacity(scene.opac_e, 0.01))
