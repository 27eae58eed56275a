"""Pins of the FP64 oracle against what the paper and the mathematics fix
(closed forms, special cases, invariants, brute force on tiny inputs,
finite differences).  CPU only."""
import json
import math
import os

import numpy as np
import pytest
import torch

import hyrf_inputs as hi
from oracle import hyrf_oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")
F64 = torch.float64


def gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ------------------------------------------------------------ contraction
def test_contraction_closed_form_values():
    g = gold("contraction.json")
    p = torch.tensor([c["p"] for c in g["cases"]], dtype=F64)
    x = O.contract(p, [0, 0, 0], [1, 1, 1])
    want = torch.tensor([c["x"] for c in g["cases"]], dtype=F64)
    assert torch.allclose(x, want, rtol=0, atol=1e-15)


def test_contraction_range_and_continuity():
    rng = np.random.default_rng(0)
    p = torch.from_numpy(rng.normal(size=(20000, 3)) * np.exp(rng.uniform(-3, 8, size=(20000, 1))))
    x = O.contract(p, [0, 0, 0], [1, 1, 1])
    assert bool(((x > 0) & (x < 1)).all())
    # continuity across |p| = 1 on random directions
    d = torch.from_numpy(rng.normal(size=(1000, 3)))
    d = d / d.norm(dim=1, keepdim=True)
    xin = O.contract(d * (1 - 1e-12), [0, 0, 0], [1, 1, 1])
    xout = O.contract(d * (1 + 1e-12), [0, 0, 0], [1, 1, 1])
    assert float((xin - xout).abs().max()) < 1e-10
    # monotone along rays and point symmetric about the box centre
    r = torch.linspace(0.0, 50.0, 400, dtype=F64)[:, None] * d[:1]
    xr = O.contract(r, [0, 0, 0], [1, 1, 1])
    proj = ((xr - 0.5) * d[:1]).sum(1)
    assert bool((proj[1:] > proj[:-1]).all())
    assert torch.allclose(O.contract(-p[:100], [0, 0, 0], [1, 1, 1]) - 0.5, -(x[:100] - 0.5), atol=1e-15)


def test_contraction_box_normalisation():
    # p' = (p - centre) * inv_half: a point at the box corner direction maps like the unit box
    p = torch.tensor([[3.0, -1.0, 2.0]], dtype=F64)
    x1 = O.contract(p, [1.0, 1.0, 1.0], [0.5, 0.5, 0.5])
    x2 = O.contract(torch.tensor([[1.0, -1.0, 0.5]], dtype=F64), [0, 0, 0], [1, 1, 1])
    assert torch.allclose(x1, x2, atol=1e-15)


# ------------------------------------------------------------ hash encoding
def test_level_resolutions():
    g = gold("hash_index.json")
    assert O.level_resolutions(16, 16.0, 1.5) == g["resolutions_L16_base16_growth1.5"]


def test_hash_index_values():
    g = gold("hash_index.json")
    for c in g["hashed"]:
        res = 7006   # any resolution with (res+1)^3 > T selects the hash
        got = O.corner_index(torch.tensor(c["corner"]), res, c["T"])
        assert int(got) == c["index"]
    for c in g["dense"]:
        got = O.corner_index(torch.tensor(c["corner"]), c["res"], c["T"])
        assert int(got) == c["index"]


def test_hash_structure():
    T = 1 << 19
    rng = np.random.default_rng(1)
    c = torch.from_numpy(rng.integers(0, 7007, size=(5000, 3)))
    h = O.corner_index(c, 7006, T)
    assert bool(((h >= 0) & (h < T)).all())
    # the x prime is 1: h(c,0,0) = c mod T
    cx = torch.zeros_like(c)
    cx[:, 0] = c[:, 0]
    assert torch.equal(O.corner_index(cx, 7006, T), c[:, 0] % T)
    # XOR separability of the per-axis terms (T a power of two)
    parts = []
    for a in range(3):
        ca = torch.zeros_like(c)
        ca[:, a] = c[:, a]
        parts.append(O.corner_index(ca, 7006, T))
    assert torch.equal(h, parts[0] ^ parts[1] ^ parts[2])


def test_dense_level_is_bijection():
    res, T = 16, 1 << 14
    g = torch.stack(torch.meshgrid(*[torch.arange(res + 1)] * 3, indexing="ij"), -1).reshape(-1, 3)
    idx = O.corner_index(g, res, T)
    assert idx.unique().numel() == (res + 1) ** 3 and int(idx.max()) == (res + 1) ** 3 - 1
    # x fastest
    assert int(O.corner_index(torch.tensor([1, 0, 0]), res, T)) == 1
    assert int(O.corner_index(torch.tensor([0, 1, 0]), res, T)) == res + 1


def test_dense_vs_hashed_levels():
    # (N+1)^3 <= T decides dense indexing: at T=2^14, N=16 (17^3=4913) and N=24 (15625) are dense
    res = O.level_resolutions(8, 16, 1.5)
    dense = [(r + 1) ** 3 <= (1 << 14) for r in res]
    assert dense == [True, True, False, False, False, False, False, False]


def _rand_table(L, T, seed=0):
    return torch.from_numpy(np.random.default_rng(seed).uniform(-1, 1, size=(L, T, 2)))


def test_interpolation_exact_at_vertices():
    res = O.level_resolutions(4, 16, 1.5)        # 16, 24, 36, 54
    table = _rand_table(4, 1 << 12)
    # x = k/16 is a vertex of level 0 (exactly representable)
    k = torch.tensor([[3, 7, 11], [0, 5, 15], [8, 8, 8]], dtype=F64)
    x = k / 16.0
    f, idx = O.hash_encode(x, table, res, return_index=True)
    for n in range(3):
        row = O.corner_index(k[n].to(torch.int64), 16, 1 << 12)
        assert torch.allclose(f[n, 0:2], table[0, row], atol=1e-15)


def test_interpolation_partition_and_linearity():
    res = O.level_resolutions(3, 16, 1.5)
    const = torch.full((3, 1 << 12, 2), 0.37, dtype=F64)
    x = torch.from_numpy(np.random.default_rng(2).uniform(0, 1, size=(500, 3)))
    f = O.hash_encode(x, const, res)
    assert torch.allclose(f, torch.full_like(f, 0.37), atol=1e-14)   # weights sum to 1, collisions irrelevant
    # trilinear: linear along x inside one cell at level 0
    table = _rand_table(3, 1 << 12, 3)
    base = torch.tensor([[2.25 / 16, 5.5 / 16, 9.75 / 16]], dtype=F64)
    ts = torch.linspace(0.0, 0.9, 7, dtype=F64)
    pts = base.repeat(7, 1)
    pts[:, 0] = (2.0 + ts) / 16
    f0 = O.hash_encode(pts, table, res)[:, 0:2]
    second = f0[2:] - 2 * f0[1:-1] + f0[:-2]
    assert float(second.abs().max()) < 1e-13


# ------------------------------------------------------------ decoders / PE / activations
def test_mlp_brute_force():
    rng = np.random.default_rng(4)
    Ws = [torch.from_numpy(rng.normal(size=s)) for s in [(5, 4), (5, 5), (3, 5)]]
    h = torch.from_numpy(rng.normal(size=(6, 4)))
    got = O.mlp(h, Ws)
    for r in range(6):
        a = [float(v) for v in h[r]]
        for li, W in enumerate(Ws):
            b = [sum(float(W[o, i]) * a[i] for i in range(len(a))) for o in range(W.shape[0])]
            a = [max(0.0, v) for v in b] if li < len(Ws) - 1 else b
        assert np.allclose(got[r].numpy(), a, atol=1e-13)


def test_positional_encoding_closed_form():
    d = torch.tensor([[1.0, 0.0, 0.0], [0.5, -0.5, 0.0]], dtype=F64)
    pe = O.pos_enc(d)
    assert pe.shape == (2, 24)
    # octave 0 of (0.5,-0.5,0): sin(pi/2)=1, sin(-pi/2)=-1, sin 0 = 0; cos = 0, 0, 1
    assert np.allclose(pe[1, 0:6].numpy(), [1, -1, 0, 0, 0, 1], atol=1e-15)
    # octave 1: sin(pi)=0, cos(pi)=-1
    assert np.allclose(pe[1, 6:12].numpy(), [0, 0, 0, -1, -1, 1], atol=1e-15)
    # (1,0,0): sin(2^k pi) = 0 for all k; cos(pi) = -1, cos(2^k pi) = 1 for k >= 1
    assert np.allclose(pe[0, 3::6].numpy(), [-1, 1, 1, 1]) and np.allclose(pe[0, 0::6].numpy(), 0.0, atol=1e-14)


def test_aggregation_closed_form():
    geo = torch.tensor([[0.3, 0.1, -0.2, 0.0, 1.0, 2.0, 0.0, -2.0]], dtype=F64)
    col = torch.tensor([[0.5, -0.5, 2.0]], dtype=F64)
    op, sc, q, rgb = O.aggregate(geo, col, torch.tensor([0.2], dtype=F64),
                                 torch.tensor([[-3.0, -3.0, -3.0]], dtype=F64),
                                 torch.tensor([[0.0, 0.5, 1.0]], dtype=F64), None)
    sig = lambda z: 1 / (1 + math.exp(-z))
    assert abs(float(op[0]) - sig(0.5)) < 1e-15
    assert np.allclose(sc[0].numpy(), [sig(-2.9), sig(-3.2), sig(-3.0)], atol=1e-15)
    assert np.allclose(q[0].numpy(), [1 / 3, 2 / 3, 0, -2 / 3], atol=1e-15)
    assert np.allclose(rgb[0].numpy(), [sig(0.5), sig(0.0), sig(3.0)], atol=1e-15)


# ------------------------------------------------------------ culling
def test_precull_frame_band_and_near_plane():
    cam = hi.look_at((0, -3, 0), (0, 0, 0), 70.0, 64, 64)
    # camera axes: x_cam = world x, y_cam = -world z, z_cam = world y + 3
    # normalised x = 2(f x/z + 32)/64 - 1 = (70/32) x / z.  At z = 3 the band |.| <= 1.3 is |x| <= 1.3*96/70
    edge = 1.3 * 32 / 70 * 3.0
    p = torch.tensor([[edge * 0.999, 0, 0], [edge * 1.001, 0, 0], [0, 0, -edge * 0.999],
                      [0, 0, edge * 1.001], [0, -2.85, 0], [0, -2.75, 0], [0, -4, 0]], dtype=F64)
    keep = O.precull(p, cam)
    assert keep.tolist() == [True, False, True, False, False, True, False]


# ------------------------------------------------------------ projection
def test_ewa_isotropic_closed_form():
    g = gold("ewa_isotropic.json")
    cam = hi.look_at(g["eye"], (0, 0, 0), g["focal"], g["width"], g["height"])
    p = torch.zeros(1, 3, dtype=F64)
    s = torch.full((1, 3), g["scale"], dtype=F64)
    for q in ([1.0, 0, 0, 0], [0.5, 0.5, -0.5, 0.5]):
        pr = O.project(p, s, torch.tensor([q], dtype=F64), cam)
        assert abs(float(pr["cov2d"][0, 0]) - g["cov2d_diag"]) < 1e-12
        assert abs(float(pr["cov2d"][0, 1])) < 1e-12
        assert abs(float(pr["conic"][0, 0]) - g["conic_diag"]) < 1e-12
        assert abs(float(pr["u"][0]) - g["u"]) < 1e-12 and abs(float(pr["v"][0]) - g["v"]) < 1e-12
    dx = dy = 0.5
    power = -0.5 * (pr["conic"][0, 0] * dx * dx + pr["conic"][0, 2] * dy * dy) - pr["conic"][0, 1] * dx * dy
    assert abs(math.exp(float(power)) - g["gauss_at_31_31"]) < 1e-12
    rx, _ = O.splat_extent(pr["cov2d"], torch.tensor([0.5], dtype=F64))
    assert abs(float(rx[0]) - (g["k_opacity_0.5"] * math.sqrt(g["cov2d_diag"]) + 1.0)) < 1e-12


def test_ewa_jacobian_and_conic_inverse():
    rng = np.random.default_rng(5)
    cam = hi.look_at((0.3, -3, 0.4), (0, 0, 0), 300.0, 256, 192)
    p = torch.from_numpy(rng.uniform(-0.8, 0.8, size=(50, 3)))
    s = torch.from_numpy(np.exp(rng.uniform(-4, -1, size=(50, 3))))
    q = torch.from_numpy(rng.normal(size=(50, 4)))
    q = q / q.norm(dim=1, keepdim=True)
    pr = O.project(p, s, q, cam)
    a, b, c = pr["cov2d"].T
    con = pr["conic"]
    assert torch.allclose(a * con[:, 0] + b * con[:, 1], torch.ones(50, dtype=F64), atol=1e-12)
    assert torch.allclose(b * con[:, 0] + c * con[:, 1], torch.zeros(50, dtype=F64), atol=1e-12)
    # 2D covariance = numerical Jacobian of the pinhole map applied to Sigma, + 0.3 I
    R = O.quat_to_rot(q)
    Sigma = R @ torch.diag_embed(s * s) @ R.transpose(1, 2)
    h = 1e-6
    for n in range(5):
        Jn = torch.zeros(2, 3, dtype=F64)
        for k in range(3):
            e = torch.zeros(1, 3, dtype=F64)
            e[0, k] = h
            up = O.project(p[n:n + 1] + e, s[n:n + 1], q[n:n + 1], cam)
            dn = O.project(p[n:n + 1] - e, s[n:n + 1], q[n:n + 1], cam)
            Jn[0, k] = (up["u"] - dn["u"]) / (2 * h)
            Jn[1, k] = (up["v"] - dn["v"]) / (2 * h)
        cov = Jn @ Sigma[n] @ Jn.T
        assert abs(float(cov[0, 0] + 0.3 - a[n])) < 1e-6 * float(a[n])
        assert abs(float(cov[1, 1] + 0.3 - c[n])) < 1e-6 * float(c[n])
        assert abs(float(cov[0, 1] - b[n])) < 1e-6 * float(a[n] + c[n])


def test_extent_is_conservative_brute_force():
    rng = np.random.default_rng(6)
    cam = hi.look_at((0, -3, 0), (0, 0, 0), 200.0, 128, 128)
    n = 40
    p = torch.from_numpy(rng.uniform(-0.5, 0.5, size=(n, 3)))
    s = torch.from_numpy(np.exp(rng.uniform(-4, -2, size=(n, 3))))
    q = torch.from_numpy(rng.normal(size=(n, 4)))
    q = q / q.norm(dim=1, keepdim=True)
    o = torch.from_numpy(rng.uniform(0.01, 1.0, size=n))
    pr = O.project(p, s, q, cam)
    rx, ry = O.splat_extent(pr["cov2d"], o)
    ys, xs = torch.meshgrid(torch.arange(128, dtype=F64), torch.arange(128, dtype=F64), indexing="ij")
    for i in range(n):
        dx = pr["u"][i] - (xs + 0.5)
        dy = pr["v"][i] - (ys + 0.5)
        c = pr["conic"][i]
        alpha = o[i] * torch.exp(-0.5 * (c[0] * dx * dx + c[2] * dy * dy) - c[1] * dx * dy)
        hit = alpha >= 1 / 255
        inside = (dx.abs() <= rx[i]) & (dy.abs() <= ry[i])
        assert bool((~hit | inside).all())
        # and the box is not loose by more than the 1 px margin + 1 px pixel grid
        if bool(hit.any()):
            assert float(dx[hit].abs().max()) >= float(rx[i]) - 2.5


# ------------------------------------------------------------ compositing
def _brute_pixel(px, py, u, v, conic, opac, rgb, order):
    """Pure-Python front-to-back blending of one pixel (Eq. 1 with the 3DGS rules)."""
    T = 1.0
    C = [0.0, 0.0, 0.0]
    for i in order:
        dx = u[i] - (px + 0.5)
        dy = v[i] - (py + 0.5)
        power = -0.5 * (conic[i][0] * dx * dx + conic[i][2] * dy * dy) - conic[i][1] * dx * dy
        if power > 0:
            continue
        a = min(0.99, opac[i] * math.exp(power))
        if a < 1 / 255:
            continue
        tT = T * (1 - a)
        if tT < 1e-4:
            break
        for ch in range(3):
            C[ch] += rgb[i][ch] * a * T
        T = tT
    return C, T


def _tiny_scene(n=60, seed=7, table_init=1.0):
    cfg = hi.with_overrides(hi.CONFIGS["tiny"], n_gauss=n, width=24, height=20, focal=30.0)
    sc = hi.make_scene(cfg, seed=seed, table_init=table_init)
    sc.scale_e[:] -= 0.0
    cam = hi.look_at((0, -3, 0), (0, 0, 0), cfg.focal, cfg.width, cfg.height)
    return sc, cam


def test_composite_matches_pure_python_brute_force():
    sc, cam = _tiny_scene(n=80)
    sc.scale_e[:] += 2.0          # larger splats so that many overlap
    params, fields = O.from_scene(sc)
    r = O.render_view(params, fields, cam, O.TRAIN)
    q, pr = r["query"], r["proj"]
    order = sorted(range(q["p"].shape[0]), key=lambda i: (float(r["depth_key"][i]), int(r["vis_idx"][i])))
    u, v = pr["u"].tolist(), pr["v"].tolist()
    conic, opac, rgb = pr["conic"].tolist(), q["opacity"].tolist(), q["rgb"].tolist()
    maxdiff = 0.0
    for k in range(r["px"].numel()):
        C, T = _brute_pixel(int(r["px"][k]), int(r["py"][k]), u, v, conic, opac, rgb, order)
        maxdiff = max(maxdiff, max(abs(C[c] - float(r["rgb_fg"][k, c])) for c in range(3)),
                      abs(T - float(r["T"][k])))
    assert maxdiff < 1e-12


def test_composite_partition_of_unity_and_monotone_T():
    sc, cam = _tiny_scene(n=120, seed=8)
    sc.scale_e[:] += 2.5
    params, fields = O.from_scene(sc)
    r = O.render_view(params, fields, cam, O.TRAIN)
    P = r["px"].numel()
    ones = torch.ones_like(r["query"]["rgb"])
    order = torch.argsort(r["depth_key"].to(F64) * 1e7 + r["vis_idx"].to(F64))
    rank = torch.empty_like(order)
    rank[order] = torch.arange(order.numel())
    rx, ry = O.splat_extent(r["proj"]["cov2d"], r["query"]["opacity"])
    C, T = O.composite(r["px"], r["py"], r["proj"]["u"], r["proj"]["v"], r["proj"]["conic"],
                       r["query"]["opacity"], ones, rank, rx, ry)
    # sum_i alpha_i T_i + T_final = 1: all colours 1 and a background of 1 give exactly 1
    assert torch.allclose(C[:, 0] + T, torch.ones(P, dtype=F64), atol=1e-12)
    assert bool((T >= 1e-4).all()) and bool((T <= 1).all())
    assert float(T.min()) < 0.5     # the scene is dense enough to matter


def test_single_opaque_splat_hides_background():
    sc, cam = _tiny_scene(n=1, seed=9)
    params, fields = O.from_scene(sc)
    with torch.no_grad():
        params.pos[:] = 0.0
        params.pos[0, 0] = 0.5 / 30.0 * 3.0   # centre exactly at a pixel centre (u = 12.5)
        params.pos[0, 2] = -0.5 / 30.0 * 3.0  # v = 10.5
        params.opac_e[:] = 20.0               # sigmoid -> 1, alpha clamps at 0.99
    r_render = O.render_view(params, fields, cam, O.RENDER)
    r_train = O.render_view(params, fields, cam, O.TRAIN)
    k = 10 * 24 + 12
    c = r_render["query"]["rgb"][0]
    assert torch.allclose(r_render["rgb"][k], 0.99 * c, atol=1e-12)      # T=0.01 < tau: no background
    cs = O.background_colour(r_train["px"][k:k + 1], r_train["py"][k:k + 1], cam, fields)[0]
    assert torch.allclose(r_train["rgb"][k], 0.99 * c + 0.01 * cs, atol=1e-12)


def test_two_splats_depth_order_closed_form():
    # two co-centred isotropic splats: C = c1 a1 + c2 a2 (1 - a1), near one first
    cam = hi.look_at((0, -3, 0), (0, 0, 0), 30.0, 8, 8)
    u = torch.tensor([4.5, 4.5], dtype=F64)
    v = torch.tensor([4.5, 4.5], dtype=F64)
    conic = torch.tensor([[0.1, 0.0, 0.1], [0.1, 0.0, 0.1]], dtype=F64)
    op = torch.tensor([0.6, 0.7], dtype=F64)
    rgb = torch.tensor([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]], dtype=F64)
    for rank, first in ((torch.tensor([0, 1]), 0), (torch.tensor([1, 0]), 1)):
        C, T = O.composite(torch.tensor([4]), torch.tensor([4]), u, v, conic, op, rgb, rank,
                           torch.tensor([9.0, 9.0], dtype=F64), torch.tensor([9.0, 9.0], dtype=F64))
        a1, a2 = float(op[first]), float(op[1 - first])
        want = a1 * rgb[first] + a2 * (1 - a1) * rgb[1 - first]
        assert torch.allclose(C[0], want, atol=1e-14)
        assert abs(float(T[0]) - (1 - a1) * (1 - a2)) < 1e-14


def test_empty_scene_gives_background():
    sc, cam = _tiny_scene(n=10, seed=10)
    params, fields = O.from_scene(sc)
    with torch.no_grad():
        params.pos[:, 1] = -10.0      # all behind the camera -> culled
    for mode in (O.RENDER, O.TRAIN):
        r = O.render_view(params, fields, cam, mode)
        assert r["vis_idx"].numel() == 0
        cs = O.background_colour(r["px"], r["py"], cam, fields)
        assert torch.allclose(r["rgb"], cs, atol=1e-14)
        assert torch.allclose(r["T"], torch.ones_like(r["T"]))


# ------------------------------------------------------------ background ray
def test_sphere_hit_closed_form_and_invariant():
    o = torch.tensor([0.0, -3.0, 0.0], dtype=F64)
    d = torch.tensor([[0.0, 1.0, 0.0]], dtype=F64)
    ps, t = O.sphere_hit(o, d, 100.0)
    assert abs(float(t[0]) - 103.0) < 1e-12
    assert torch.allclose(ps, torch.tensor([[0.0, 100.0, 0.0]], dtype=F64), atol=1e-12)
    x = O.contract(ps, [0, 0, 0], [1, 1, 1])
    assert torch.allclose(x, torch.tensor([[0.5, 0.9975, 0.5]], dtype=F64), atol=1e-15)
    rng = np.random.default_rng(11)
    dd = torch.from_numpy(rng.normal(size=(1000, 3)))
    ps, t = O.sphere_hit(o, dd, 100.0)
    assert bool((t > 0).all())
    assert torch.allclose(ps.norm(dim=1), torch.full((1000,), 100.0, dtype=F64), atol=1e-10)


def test_pixel_ray_through_principal_point_is_forward():
    cam = hi.look_at((0.5, -3, 0.2), (0, 0, 0), 70.0, 64, 64)
    o, d = O.pixel_rays(torch.tensor([31.5 - 0.5]), torch.tensor([31.5 - 0.5]), cam)
    # pixel centre (31.5, 31.5) is half a pixel from the principal point (32,32)
    o2, d2 = O.pixel_rays(torch.tensor([32.0]) - 0.5, torch.tensor([32.0]) - 0.5, cam)
    fwd = torch.tensor([-0.5, 3.0, -0.2], dtype=F64)
    fwd = fwd / fwd.norm()
    assert torch.allclose(d2[0] / d2[0].norm(), fwd, atol=1e-6)
    assert torch.allclose(o, torch.tensor([0.5, -3.0, 0.2], dtype=F64), atol=1e-6)


# ------------------------------------------------------------ binning / sort
def test_bin_and_sort_against_lexsort():
    depth, rect, tw, th = hi.make_splat_records(2, 300, 100, 70, seed=12)
    keys, ids, ranges = O.bin_and_sort(torch.from_numpy(depth), torch.from_numpy(rect), tw, th)
    # independent: numpy lexsort over the expanded entry list
    ev, et, ed, ei = [], [], [], []
    for vw in range(2):
        for i in range(300):
            x0, y0, x1, y1 = rect[vw, i]
            for ty in range(y0, y1):
                for tx in range(x0, x1):
                    ev.append(vw); et.append(ty * tw + tx); ed.append(depth[vw, i]); ei.append(vw * 300 + i)
    order = np.lexsort((np.array(ei), np.array(ed, np.float32), np.array(et), np.array(ev)))
    assert np.array_equal(ids.numpy(), np.array(ei)[order])
    # ranges partition the list and agree with keys
    for k in range(2 * tw * th):
        a, b = ranges[k].tolist()
        assert bool((keys[a:b] == k).all())
    assert int((ranges[:, 1] - ranges[:, 0]).sum()) == len(ei)


# ------------------------------------------------------------ gradients
def test_oracle_gradient_matches_central_differences():
    sc, cam = _tiny_scene(n=25, seed=13)
    sc.scale_e[:] += 2.0
    params, fields = O.from_scene(sc, requires_grad=True)
    target = torch.from_numpy(hi.make_target_image((3, cam.height, cam.width), seed=5)).to(F64)

    def loss_fn():
        img = O.render_image(params, fields, cam, O.TRAIN)["image"]
        return torch.sum(img * target)        # smooth linear functional of the image

    L = loss_fn()
    leaves = [params.pos, params.scale_e, params.rot_e, params.opac_e, params.col_e,
              fields.table_geo, fields.table_rad] + fields.mlp_geo + fields.mlp_col
    grads = torch.autograd.grad(L, leaves)
    rng = np.random.default_rng(14)
    checked = 0
    for leaf, g in zip(leaves, grads):
        flat = leaf.detach().view(-1)
        gflat = g.reshape(-1)
        nz = torch.nonzero(gflat.abs() > 1e-8).reshape(-1)
        pick = nz[torch.from_numpy(rng.permutation(nz.numel())[:4])] if nz.numel() else []
        for j in pick:
            j = int(j)
            h = 1e-6 * max(1.0, abs(float(flat[j])))
            with torch.no_grad():
                old = float(flat[j])
                flat[j] = old + h
                lp = float(loss_fn())
                flat[j] = old - h
                lm = float(loss_fn())
                flat[j] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - float(gflat[j])) <= 1e-5 * max(1.0, abs(fd)), (leaf.shape, j, fd, float(gflat[j]))
            checked += 1
    assert checked >= 30


# ------------------------------------------------------------ rotation / camera centre
def _rodrigues(axis, theta):
    """Rotation by theta about the unit axis: I cos t + sin t [n]x + (1 - cos t) n n^T."""
    n = np.asarray(axis, np.float64)
    n = n / np.linalg.norm(n)
    K = np.array([[0.0, -n[2], n[1]], [n[2], 0.0, -n[0]], [-n[1], n[0], 0.0]])
    return np.eye(3) * math.cos(theta) + math.sin(theta) * K + (1 - math.cos(theta)) * np.outer(n, n)


def test_quat_to_rot_closed_forms():
    # q = (w, x, y, z) = (cos t/2, sin t/2 n): rotation by t about n, applied to column vectors
    th = 0.7
    Rz = O.quat_to_rot(torch.tensor([[math.cos(th / 2), 0.0, 0.0, math.sin(th / 2)]], dtype=F64))[0]
    assert torch.allclose(Rz @ torch.tensor([1.0, 0, 0], dtype=F64),
                          torch.tensor([math.cos(th), math.sin(th), 0.0], dtype=F64), atol=1e-15)
    assert torch.allclose(Rz @ torch.tensor([0, 1.0, 0], dtype=F64),
                          torch.tensor([-math.sin(th), math.cos(th), 0.0], dtype=F64), atol=1e-15)
    Rx = O.quat_to_rot(torch.tensor([[math.cos(th / 2), math.sin(th / 2), 0.0, 0.0]], dtype=F64))[0]
    assert torch.allclose(Rx @ torch.tensor([0, 1.0, 0], dtype=F64),
                          torch.tensor([0.0, math.cos(th), math.sin(th)], dtype=F64), atol=1e-15)
    Ry = O.quat_to_rot(torch.tensor([[math.cos(th / 2), 0.0, math.sin(th / 2), 0.0]], dtype=F64))[0]
    assert torch.allclose(Ry @ torch.tensor([0, 0, 1.0], dtype=F64),
                          torch.tensor([math.sin(th), 0.0, math.cos(th)], dtype=F64), atol=1e-15)
    # half turn about x
    assert torch.allclose(O.quat_to_rot(torch.tensor([[0.0, 1.0, 0.0, 0.0]], dtype=F64))[0],
                          torch.diag(torch.tensor([1.0, -1.0, -1.0], dtype=F64)), atol=0)
    # Rodrigues' formula for random axes and angles
    rng = np.random.default_rng(31)
    for _ in range(20):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        t = rng.uniform(-math.pi, math.pi)
        q = torch.tensor([[math.cos(t / 2), *(math.sin(t / 2) * n)]], dtype=F64)
        assert np.allclose(O.quat_to_rot(q)[0].numpy(), _rodrigues(n, t), atol=1e-14)


def test_quat_to_rot_is_a_homomorphism():
    # R(q1 q2) = R(q1) R(q2) with the Hamilton product (w, x, y, z)
    def hamilton(a, b):
        w1, x1, y1, z1 = a
        w2, x2, y2, z2 = b
        return [w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2]
    rng = np.random.default_rng(32)
    for _ in range(10):
        a, b = rng.normal(size=4), rng.normal(size=4)
        a /= np.linalg.norm(a)
        b /= np.linalg.norm(b)
        Ra = O.quat_to_rot(torch.from_numpy(a[None]))[0]
        Rb = O.quat_to_rot(torch.from_numpy(b[None]))[0]
        Rab = O.quat_to_rot(torch.tensor([hamilton(a, b)], dtype=F64))[0]
        assert torch.allclose(Rab, Ra @ Rb, atol=1e-14)
        assert torch.allclose(Ra @ Ra.T, torch.eye(3, dtype=F64), atol=1e-14)
        assert abs(float(torch.linalg.det(Ra)) - 1.0) < 1e-14


def test_ewa_anisotropic_rotated_closed_form():
    # scale (a, b, c) turned a quarter about world z: Sigma = diag(b^2, a^2, c^2).  From the eye
    # (0, -3, 0) the camera x axis is world x and camera y is world -z, so at the origin
    # (depth 3) the 2D covariance is (f/3)^2 diag(b^2, c^2) + 0.3 I.
    f = 70.0
    cam = hi.look_at((0, -3, 0), (0, 0, 0), f, 64, 64)
    a, b, c = 0.05, 0.12, 0.2
    q = torch.tensor([[math.cos(math.pi / 4), 0.0, 0.0, math.sin(math.pi / 4)]], dtype=F64)
    pr = O.project(torch.zeros(1, 3, dtype=F64), torch.tensor([[a, b, c]], dtype=F64), q, cam)
    k = (f / 3.0) ** 2
    assert abs(float(pr["cov2d"][0, 0]) - (k * b * b + 0.3)) < 1e-9
    assert abs(float(pr["cov2d"][0, 2]) - (k * c * c + 0.3)) < 1e-9
    assert abs(float(pr["cov2d"][0, 1])) < 1e-9
    # a quarter turn about world x instead swaps the y and z axes: diag(a^2, c^2, b^2)
    qx = torch.tensor([[math.cos(math.pi / 4), math.sin(math.pi / 4), 0.0, 0.0]], dtype=F64)
    pr = O.project(torch.zeros(1, 3, dtype=F64), torch.tensor([[a, b, c]], dtype=F64), qx, cam)
    assert abs(float(pr["cov2d"][0, 0]) - (k * a * a + 0.3)) < 1e-9
    assert abs(float(pr["cov2d"][0, 2]) - (k * b * b + 0.3)) < 1e-9


def test_camera_center_recovers_the_eye():
    rng = np.random.default_rng(33)
    for _ in range(10):
        eye = rng.uniform(-4, 4, size=3)
        eye[1] = -abs(eye[1]) - 1.0
        cam = hi.look_at(eye, rng.uniform(-0.5, 0.5, size=3), 100.0, 64, 48)
        o = O.camera_center(cam)
        assert np.allclose(o.numpy(), eye, atol=2e-6 * np.linalg.norm(eye))
        # the centre maps to the camera-space origin, and the ray origin of every pixel is it
        t = O.camera_space(o[None], cam)[0]
        assert float(t.abs().max()) < 2e-6 * np.linalg.norm(eye)
        ro, _ = O.pixel_rays(torch.tensor([3]), torch.tensor([5]), cam)
        assert torch.allclose(ro, o, atol=1e-12)


def test_view_direction_points_from_the_eye():
    # the colour decoder's direction for a Gaussian on the optical axis is the viewing direction
    cam = hi.look_at((1.0, -3.0, 0.5), (0, 0, 0), 70.0, 64, 64)
    o = O.camera_center(cam)
    d = -o / o.norm()
    assert torch.allclose(torch.from_numpy(cam.R[2].astype(np.float64)), d, atol=1e-6)


# ------------------------------------------------------------ pair search
def _all_pairs(px, py, u, v, rx, ry):
    cx = px.to(F64)[:, None] + 0.5
    cy = py.to(F64)[:, None] + 0.5
    m = (torch.abs(cx - u[None]) <= rx[None]) & (torch.abs(cy - v[None]) <= ry[None])
    a, b = torch.nonzero(m, as_tuple=True)
    return set(zip(a.tolist(), b.tolist()))


@pytest.mark.parametrize("pixels", ["all", "window", "scattered"])
def test_pair_search_equals_all_pairs(pixels):
    rng = np.random.default_rng(34)
    W, H, N = 160, 120, 700
    u = torch.from_numpy(rng.uniform(-20, W + 20, N))
    v = torch.from_numpy(rng.uniform(-20, H + 20, N))
    rx = torch.from_numpy(np.exp(rng.uniform(-1, 3.5, N)))
    ry = torch.from_numpy(np.exp(rng.uniform(-1, 3.5, N)))
    rx[:10] = -1.0                               # dropped splats (no box)
    u[10:20] = torch.floor(u[10:20]) + 0.5        # boxes ending exactly on pixel centres
    rx[10:20] = torch.round(rx[10:20])
    if pixels == "all":
        yy, xx = torch.meshgrid(torch.arange(H), torch.arange(W), indexing="ij")
        px, py = xx.reshape(-1), yy.reshape(-1)
    elif pixels == "window":
        yy, xx = torch.meshgrid(torch.arange(30, 70), torch.arange(50, 110), indexing="ij")
        px, py = xx.reshape(-1), yy.reshape(-1)
    else:
        px = torch.from_numpy(rng.integers(0, W, 500))
        py = torch.from_numpy(rng.integers(0, H, 500))
    pi, si = O._pairs_for_pixels(px, py, u, v, rx, ry, chunk=1 << 14)
    got = list(zip(pi.tolist(), si.tolist()))
    assert len(got) == len(set(got))
    assert set(got) == _all_pairs(px, py, u, v, rx, ry)


# ------------------------------------------------------------ decision variants / comparison rule
def test_blend_pixel_flips():
    al = [0.5, 1.0 / 255.0, 0.3]
    pw = [-0.1, -2.0, -0.5]
    rgb = [[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]]
    C, T = O.blend_pixel(al, pw, rgb)
    assert math.isclose(T, 0.5 * (1 - 1 / 255) * 0.7, rel_tol=1e-15)
    C2, T2 = O.blend_pixel(al, pw, rgb, flip_alpha=1)        # the 1/255 splat left out
    assert math.isclose(T2, 0.5 * 0.7, rel_tol=1e-15) and C2[1] == 0.0
    assert math.isclose(C2[2], 0.3 * 0.5, rel_tol=1e-15)
    # early stop: after 0.99 and 0.98, T = 2e-4 and the 0.5 splat brings it to 1e-4 (not below)
    C, T = O.blend_pixel([0.99, 0.98, 0.5], [-0.1] * 3, rgb)
    assert math.isclose(T, 1e-4, rel_tol=1e-12) and math.isclose(C[2], 0.5 * 2e-4, rel_tol=1e-12)
    C3, T3 = O.blend_pixel([0.99, 0.995, 0.5], [-0.1] * 3, rgb)           # 0.01 * 0.005 < 1e-4: stop
    C4, T4 = O.blend_pixel([0.99, 0.995, 0.5], [-0.1] * 3, rgb, flip_stop=1)
    assert math.isclose(T3, 0.01, rel_tol=1e-12) and math.isclose(T4, 0.01 * 0.005, rel_tol=1e-12)
    assert math.isclose(C4[1], 0.995 * 0.01, rel_tol=1e-12)


def test_comparison_rule_explains_one_flipped_decision_only():
    """A float64 'GPU' image made by the oracle itself, with one splat's
    opacity moved across alpha = 1/255 at one pixel, must be explained by one
    flipped decision; the same image with an unrelated error must not."""
    from oracle import parity
    sc, cam = _tiny_scene(n=60, seed=35)
    sc.scale_e[:] += 2.0
    params, fields = O.from_scene(sc)
    with torch.no_grad():
        r = O.render_view(params, fields, cam, O.TRAIN, return_stats=True)
    P_ = r["px"].numel()
    img = r["rgb"].detach().numpy().copy()
    # pick a pixel with a contributing pair and rebuild it with that pair's alpha test flipped
    var = O.decision_variants(r, torch.arange(P_), 1e9, 0.0)
    k = next(i for i, vv in enumerate(var) if len(vv) > 2 and any(
        max(abs(a - b) for a, b in zip(x[3], vv[0][3])) > 1e-3 for x in vv[1:]))
    flipped = next(x for x in var[k][1:] if max(abs(a - b) for a, b in zip(x[3], var[k][0][3])) > 1e-3)
    good = img.copy()
    good[k] = flipped[3]
    res = parity.compare_pixels(good, r, delta_alpha=1e9, delta_T=1e-4)
    assert res["n_bad"] == 0 and res["n_flip"] == 1 and res["flipped"] == [k]
    # the same flip is refused when its decision is not near the threshold
    res = parity.compare_pixels(good, r, delta_alpha=1e-4, delta_T=1e-4)
    assert res["n_bad"] == 1
    bad = img.copy()
    bad[k] += 3e-5
    res = parity.compare_pixels(bad, r)
    assert res["n_bad"] == 1 and not res["ok"]
    assert parity.compare_pixels(img, r)["ok"]


def test_oracle_gradient_matches_central_differences_at_the_100k_workload():
    """SURVEY-style pin of the oracle's gradient at scale: the 100k-Gaussian
    800x800 workload (L = 16, T = 2^19, 2x64 decoders), L = sum(w * C) over
    64 seeded pixels, 6 seeded directions on a 1% subset of every parameter
    tensor: central differences of the FP64 forward equal the autograd
    gradient's projection to 1e-6 (shrinking the step past grid-cell kinks)."""
    import sys, os
    sys.path.insert(0, os.path.dirname(__file__))
    from _hyrf_testutil import DirectionalCase
    case = DirectionalCase("c100k", n_pixels=64, seed=43)
    used = 0
    for it in range(6):
        fd, an, scale, ok = case.check_fd(case.direction(2000 + it))
        used += ok
    assert used >= 6, used
