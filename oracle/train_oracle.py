"""FP64 CPU oracle of the training-loop steps that follow HyRF's render step.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg call this module; the product path (the HIP library and its
Python binding) never imports it, and this module imports nothing from the
product.  Plain PyTorch CPU ops in float64, unfused, written from the paper
(Wang & Xu, "HyRF", Sec. 3.4 Eq. 12: the loss mixes an L1 term and an SSIM
term with weight lambda, as 3DGS does) and from the SSIM definition of Wang
et al. 2004 (Sec. III-B: Gaussian-weighted local means, variances and
covariance; the product of the luminance, contrast and structure terms).

The steps after the backward in a training iteration follow the paper's
statement that everything not specified is as in 3DGS (Sec. 4.1) and that
Gaussians are densified from accumulated gradients, their explicit opacity
periodically reset and low-opacity Gaussians pruned (Sec. 3.1, Sec. 3.4):
Adam (Kingma & Ba 2015, Algorithm 1), the 3DGS densification statistics and
decisions, the opacity reset.

Readings of what the paper leaves open:
  * the SSIM term of Eq. 12 is the structural dissimilarity 1 - SSIM (a loss
    that is minimised), with the 3DGS settings: lambda = 0.2; an 11 x 11
    Gaussian window of standard deviation 1.5; stabilisers C1 = (0.01 L)^2,
    C2 = (0.03 L)^2 with dynamic range L = 1; local statistics are taken per
    colour channel with the window centred on each pixel and the image
    extended by zeros outside its frame (the window is not renormalised at
    the border); SSIM is the mean of the per-pixel map over pixels, channels
    and views;
  * the L1 term is the mean absolute difference over the same elements;
  * densification statistics: for every view in which a Gaussian's
    footprint touches the image, the norm of the loss gradient with respect
    to its projected centre in normalised device coordinates,
    |(W/2 dL/du, H/2 dL/dv)|, is accumulated with a count (3DGS);
  * decisions per Gaussian judged: mean = accum / count (0 if count is 0);
    clone if mean >= threshold and its largest aggregated scale <= the dense
    extent, split if mean >= threshold and larger, prune if the aggregated
    opacity < min_opacity.  The mean and the comparisons are integer
    decisions taken in float32, the kernel's precision;
  * the opacity reset acts on the explicit opacity logit:
    alpha_e = min(alpha_e, logit(value)) (3DGS's rule, whose opacity is a
    single explicit logit), logit(value) rounded once to float32.
"""
from __future__ import annotations

import math

import numpy as np
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



# ---------------------------------------------------------------- Adam
def adam_step(param, grad, m, v, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-15):
    """One step of Adam, Algorithm 1 of Kingma & Ba (2015), in float64:
    m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2;
    m_hat = m / (1 - b1^t);  v_hat = v / (1 - b2^t);
    param <- param - lr m_hat / (sqrt(v_hat) + eps).
    (eps default: the value 3DGS trains with.)  Returns new (param, m, v)."""
    p = np.asarray(param, np.float64)
    g = np.asarray(grad, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return p - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


# ---------------------------------------------------------------- densification
def densification_stats(du, dv, width: int, height: int, footprint):
    """Per (view, Gaussian) gradients du, dv of the loss with respect to the
    projected centre (pixels) -> (accum, count) contributions: the norm of the
    NDC-space gradient (W/2 du, H/2 dv) where the footprint touches the image."""
    du = np.asarray(du, np.float64)
    dv = np.asarray(dv, np.float64)
    fp = np.asarray(footprint, bool)
    g = np.sqrt((0.5 * width * du) ** 2 + (0.5 * height * dv) ** 2)
    return np.where(fp, g, 0.0), fp.astype(np.float64)


PRUNE, CLONE, SPLIT, JUDGED = 1, 2, 4, 8


def densify_flags(accum, count, opacity, scale_max, threshold: float, dense_extent: float, min_opacity: float):
    """Flags of the judged Gaussians (float32 decisions)."""
    a = np.asarray(accum, np.float32)
    c = np.asarray(count, np.float32)
    with np.errstate(divide="ignore", invalid="ignore"):
        mean = np.where(c > 0, a / np.where(c > 0, c, np.float32(1)), np.float32(0)).astype(np.float32)
    f = np.full(a.shape, JUDGED, np.uint8)
    dens = mean >= np.float32(threshold)
    small = np.asarray(scale_max, np.float32) <= np.float32(dense_extent)
    f |= np.where(dens & small, CLONE, 0).astype(np.uint8)
    f |= np.where(dens & ~small, SPLIT, 0).astype(np.uint8)
    f |= np.where(np.asarray(opacity, np.float32) < np.float32(min_opacity), PRUNE, 0).astype(np.uint8)
    return f


def reset_opacity(opac_e, value: float):
    """alpha_e <- min(alpha_e, logit(value)), float32."""
    cap = np.float32(math.log(value / (1.0 - value)))
    return np.minimum(np.asarray(opac_e, np.float32), cap)
