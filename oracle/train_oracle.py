"""FP64 CPU oracle of the training-loop steps that follow HyRF's render step.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg call this module; the product path (the HIP library and its
Python binding) never imports it, and this module imports nothing from the
product.  Plain PyTorch CPU ops in float64, unfused, written from the paper
(Wang & Xu, "HyRF", Sec. 3.4 Eq. 12: the loss mixes an L1 term and an SSIM
term with weight lambda, as 3DGS does) and from the SSIM definition of Wang
et al. 2004 (Sec. III-B: Gaussian-weighted local means, variances and
covariance; the product of the luminance, contrast and structure terms).

Readings of what the paper leaves open (each also listed in the design doc):
  * the SSIM term of Eq. 12 is the structural dissimilarity 1 - SSIM (a loss
    that is minimised), with the 3DGS settings: lambda = 0.2; an 11 x 11
    Gaussian window of standard deviation 1.5; stabilisers C1 = (0.01 L)^2,
    C2 = (0.03 L)^2 with dynamic range L = 1; local statistics are taken per
    colour channel with the window centred on each pixel and the image
    extended by zeros outside its frame (the window is not renormalised at
    the border); SSIM is the mean of the per-pixel map over pixels, channels
    and views;
  * the L1 term is the mean absolute difference over the same elements.
"""
from __future__ import annotations

import torch
import torch.nn.functional as F

F64 = torch.float64

SSIM_WINDOW = 11
SSIM_SIGMA = 1.5
SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2
SSIM_LAMBDA = 0.2


def gaussian_window(size: int = SSIM_WINDOW, sigma: float = SSIM_SIGMA) -> torch.Tensor:
    """2D Gaussian weighting window w(i, j) proportional to
    exp(-((i-c)^2 + (j-c)^2) / (2 sigma^2)), c = (size-1)/2, normalised to
    unit sum (Wang et al. 2004, Sec. III-B)."""
    c = (size - 1) / 2.0
    i = torch.arange(size, dtype=F64) - c
    w = torch.exp(-(i[:, None] ** 2 + i[None, :] ** 2) / (2.0 * sigma * sigma))
    return w / w.sum()


def local_mean(img: torch.Tensor, window: torch.Tensor) -> torch.Tensor:
    """Window-weighted local mean of each plane of img (..., H, W): the window
    centred on every pixel, zeros outside the frame."""
    shp = img.shape
    x = img.reshape(-1, 1, shp[-2], shp[-1])
    k = window.shape[0]
    out = F.conv2d(x, window[None, None], padding=k // 2)
    return out.reshape(shp)


def ssim_map(img: torch.Tensor, target: torch.Tensor, window=None) -> torch.Tensor:
    """Per-pixel SSIM of two images (..., H, W) in float64: luminance term
    (2 mu_x mu_y + C1) / (mu_x^2 + mu_y^2 + C1) times contrast-structure term
    (2 sigma_xy + C2) / (sigma_x^2 + sigma_y^2 + C2)."""
    w = gaussian_window() if window is None else window
    x = img.to(F64)
    y = target.to(F64)
    mu_x = local_mean(x, w)
    mu_y = local_mean(y, w)
    var_x = local_mean(x * x, w) - mu_x * mu_x
    var_y = local_mean(y * y, w) - mu_y * mu_y
    cov = local_mean(x * y, w) - mu_x * mu_y
    lum = (2.0 * mu_x * mu_y + SSIM_C1) / (mu_x * mu_x + mu_y * mu_y + SSIM_C1)
    cs = (2.0 * cov + SSIM_C2) / (var_x + var_y + SSIM_C2)
    return lum * cs


def ssim(img: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
    """Mean SSIM over every pixel, channel and view."""
    return ssim_map(img, target).mean()


def l1_dssim_loss(img: torch.Tensor, target: torch.Tensor, lam: float = SSIM_LAMBDA):
    """Training loss of Sec. 3.4 Eq. 12: (1 - lambda) L1 + lambda (1 - SSIM).
    Returns (loss, l1, ssim) as float64 scalars (differentiable in img)."""
    x = img.to(F64)
    y = target.to(F64)
    l1 = torch.mean(torch.abs(x - y))
    s = ssim(x, y)
    return (1.0 - lam) * l1 + lam * (1.0 - s), l1, s


def l1_dssim_grad(img: torch.Tensor, target: torch.Tensor, lam: float = SSIM_LAMBDA):
    """(loss, l1, ssim, dloss/dimg) with the gradient from float64 autograd."""
    x = img.detach().to(F64).clone().requires_grad_(True)
    loss, l1, s = l1_dssim_loss(x, target, lam)
    (g,) = torch.autograd.grad(loss, x)
    return float(loss.detach()), float(l1.detach()), float(s.detach()), g
