"""Pins of the training-loss oracle (Sec. 3.4 Eq. 12 with the SSIM of Wang et
al. 2004) against closed forms, brute force and finite differences."""
import math

import numpy as np
import pytest
import torch

from oracle import train_oracle as TO


def _img(shape, seed):
    g = np.random.default_rng(seed)
    return torch.from_numpy(g.random(shape))


def test_window_is_a_normalised_gaussian():
    w = TO.gaussian_window()
    assert w.shape == (11, 11)
    assert abs(float(w.sum()) - 1.0) < 1e-15
    assert torch.allclose(w, w.T) and torch.allclose(w, w.flip(0))
    # neighbouring weights on an axis differ by exp((2k+1) / (2 sigma^2))
    assert abs(float(w[5, 5] / w[5, 4]) - math.exp(1.0 / (2 * 1.5 ** 2))) < 1e-12
    assert abs(float(w[5, 4] / w[5, 3]) - math.exp(3.0 / (2 * 1.5 ** 2))) < 1e-12
    # separable: rank one
    assert torch.linalg.matrix_rank(w).item() == 1


def test_ssim_of_an_image_with_itself_is_one():
    x = _img((2, 3, 17, 23), 1)
    assert torch.allclose(TO.ssim_map(x, x), torch.ones_like(x), atol=1e-12)
    loss, l1, s = TO.l1_dssim_loss(x, x)
    assert abs(float(loss)) < 1e-12 and float(l1) == 0.0 and abs(float(s) - 1) < 1e-12


def test_constant_images_closed_form_interior_and_border():
    """Constant planes a and b: with window mass m inside the frame,
    mu = m a, E[x^2] = m a^2, so var_x = m (1 - m) a^2 and cov = m (1 - m) a b.
    Interior pixels have m = 1 and SSIM = (2ab + C1) / (a^2 + b^2 + C1).
    Tolerance: E[x^2] - mu^2 cancels to ~1e-17 absolute, divided by C2."""
    a, b = 0.7, 0.3
    H, W = 15, 26
    x = torch.full((1, H, W), a, dtype=torch.float64)
    y = torch.full((1, H, W), b, dtype=torch.float64)
    S = TO.ssim_map(x, y)[0]
    C1, C2 = 1e-4, 9e-4
    assert abs(float(S[7, 12]) - (2 * a * b + C1) / (a * a + b * b + C1)) < 2e-12
    # corner pixel: the window keeps its quarter from the centre outwards
    i = np.arange(11) - 5.0
    g = np.exp(-i * i / (2 * 1.5 ** 2))
    g /= g.sum()
    m = g[5:].sum() ** 2
    lum = (2 * m * m * a * b + C1) / (m * m * (a * a + b * b) + C1)
    cs = (2 * m * (1 - m) * a * b + C2) / (m * (1 - m) * (a * a + b * b) + C2)
    assert abs(float(S[0, 0]) - lum * cs) < 2e-12
    # an edge pixel (row 0, column in the interior)
    m = g[5:].sum()
    lum = (2 * m * m * a * b + C1) / (m * m * (a * a + b * b) + C1)
    cs = (2 * m * (1 - m) * a * b + C2) / (m * (1 - m) * (a * a + b * b) + C2)
    assert abs(float(S[0, 12]) - lum * cs) < 2e-12


def test_ssim_map_matches_brute_force_window_sums():
    """Every local statistic summed pixel by pixel over the 11 x 11 window with
    w(di, dj) = exp(-(di^2 + dj^2) / 4.5) / Z, pixels outside the frame
    skipped."""
    x = _img((2, 9, 13), 2)
    y = _img((2, 9, 13), 3)
    S = TO.ssim_map(x, y).numpy()
    Z = sum(math.exp(-(di * di + dj * dj) / 4.5) for di in range(-5, 6) for dj in range(-5, 6))
    X, Y = x.numpy(), y.numpy()
    for c in range(2):
        for r in range(9):
            for q in range(13):
                mx = my = sxx = syy = sxy = 0.0
                for di in range(-5, 6):
                    for dj in range(-5, 6):
                        rr, qq = r + di, q + dj
                        if 0 <= rr < 9 and 0 <= qq < 13:
                            w = math.exp(-(di * di + dj * dj) / 4.5) / Z
                            u, v = X[c, rr, qq], Y[c, rr, qq]
                            mx += w * u
                            my += w * v
                            sxx += w * u * u
                            syy += w * v * v
                            sxy += w * u * v
                vx, vy, cv = sxx - mx * mx, syy - my * my, sxy - mx * my
                ref = ((2 * mx * my + 1e-4) * (2 * cv + 9e-4)) / ((mx * mx + my * my + 1e-4) * (vx + vy + 9e-4))
                assert abs(S[c, r, q] - ref) < 1e-12, (c, r, q)


def test_ssim_symmetric_and_bounded():
    x = _img((3, 20, 21), 4)
    y = _img((3, 20, 21), 5)
    Sxy = TO.ssim_map(x, y)
    assert torch.allclose(Sxy, TO.ssim_map(y, x), atol=1e-14)
    assert float(Sxy.abs().max()) <= 1.0


def test_loss_weights_l1_and_dssim():
    x = _img((1, 3, 16, 16), 6)
    y = _img((1, 3, 16, 16), 7)
    loss, l1, s = TO.l1_dssim_loss(x, y)
    assert abs(float(l1) - float(np.abs(x.numpy() - y.numpy()).mean())) < 1e-14
    assert abs(float(loss) - (0.8 * float(l1) + 0.2 * (1 - float(s)))) < 1e-14
    loss0, _, _ = TO.l1_dssim_loss(x, y, lam=0.0)
    assert abs(float(loss0) - float(l1)) < 1e-15


def test_loss_gradient_matches_central_differences():
    x = _img((1, 2, 12, 14), 8)
    y = _img((1, 2, 12, 14), 9)
    _, _, _, g = TO.l1_dssim_grad(x, y)
    rng = np.random.default_rng(10)
    h = 1e-6
    for _ in range(24):
        idx = tuple(int(rng.integers(0, n)) for n in x.shape)
        xp, xm = x.clone(), x.clone()
        xp[idx] += h
        xm[idx] -= h
        fd = (float(TO.l1_dssim_loss(xp, y)[0]) - float(TO.l1_dssim_loss(xm, y)[0])) / (2 * h)
        assert abs(fd - float(g[idx])) < 1e-7 * max(1.0, abs(fd)) + 1e-9, (idx, fd, float(g[idx]))


# ---------------------------------------------------------------- Adam
def test_adam_matches_torch_optim_adam():
    """The library optimiser (torch.optim.Adam, float64) reaches the same
    parameters after several steps."""
    rng = np.random.default_rng(11)
    p0 = rng.normal(size=50)
    grads = [rng.normal(size=50) * 10 ** rng.uniform(-6, 0, size=50) for _ in range(5)]
    pt = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([pt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for t, g in enumerate(grads, start=1):
        pt.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        p, m, v = TO.adam_step(p, g, m, v, t, lr=1e-2, eps=1e-8)
    assert np.allclose(p, pt.detach().numpy(), rtol=0, atol=1e-14)


def test_adam_first_step_is_a_signed_lr_step():
    """t = 1: m_hat = g and v_hat = g^2, so the update is -lr g / (|g| + eps)."""
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    p, m, v = TO.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.1, eps=1e-15)
    assert np.allclose(p, -0.1 * g / (np.abs(g) + 1e-15), rtol=1e-13, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_constant_gradient_keeps_unit_steps():
    """With a constant gradient g every bias-corrected step is exactly
    -lr sign(g) (m_hat = g, v_hat = g^2 for all t)."""
    p, m, v = np.array([1.0]), np.zeros(1), np.zeros(1)
    for t in range(1, 8):
        p, m, v = TO.adam_step(p, np.array([2.0]), m, v, t, lr=0.25, eps=0.0)
    assert abs(p[0] - (1.0 - 7 * 0.25)) < 1e-12


# ---------------------------------------------------------------- densification
def test_densification_stats_ndc_scaling():
    acc, cnt = TO.densification_stats([2.0, 1.0, 5.0], [0.0, 1.0, 5.0], 200, 100, [True, True, False])
    assert np.allclose(acc, [200.0, math.hypot(100.0, 50.0), 0.0]) and list(cnt) == [1.0, 1.0, 0.0]


def test_densify_flags_cases():
    acc = np.array([0.0, 4e-4, 4e-4, 1e-4, 6e-4], np.float32)
    cnt = np.array([0, 2, 2, 1, 3], np.float32)
    op = np.array([0.5, 0.5, 0.001, 0.5, 0.004], np.float32)
    smax = np.array([0.1, 0.005, 0.05, 0.005, 0.5], np.float32)
    f = TO.densify_flags(acc, cnt, op, smax, threshold=2e-4, dense_extent=0.01, min_opacity=0.005)
    J, P_, C_, S_ = TO.JUDGED, TO.PRUNE, TO.CLONE, TO.SPLIT
    # last: float32(6e-4) / 3 rounds to 2.0000001e-4 >= float32(2e-4), so it splits
    assert list(f) == [J, J | C_, J | S_ | P_, J, J | S_ | P_]


def test_reset_opacity_caps_at_logit():
    x = np.array([-10.0, -4.59511985, 0.0, 3.0], np.float32)
    r = TO.reset_opacity(x, 0.01)
    cap = np.float32(math.log(0.01 / 0.99))
    assert r[0] == np.float32(-10.0) and r[2] == cap and r[3] == cap
    assert abs(1 / (1 + math.exp(-float(r[3]))) - 0.01) < 1e-8
