"""FP64 CPU oracle of HyRF's differentiable render step.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg call this module; the product path (the HIP library and its
Python binding) never imports it, and this module imports nothing from the
product.  It is written from the paper (Wang & Xu, "HyRF: Hybrid Radiance
Fields for Memory-efficient and High-quality Novel View Synthesis"), with
plain PyTorch CPU ops in float64, untiled and unfused, step by step in the
paper's order:

  pre-cull (Sec. 3.3, Eqs. 8-9)  ->  AABB normalise + contraction (Sec. 3.2
  Eq. 2; App. A.1 Eqs. 13-14)  ->  two multi-resolution hash encodings
  (Sec. 3.2 Eq. 3; Instant-NGP)  ->  geometry / colour decoders with the
  view-direction encoding (Eqs. 4-6)  ->  aggregation with the explicit
  Gaussians (Eq. 7)  ->  EWA projection (3DGS rasterizer, Sec. 3.1)  ->
  depth-ordered front-to-back alpha blending (Eq. 1)  ->  background sphere
  colour and blend (Sec. 3.3 Eqs. 10-11; App. A.2)  ->  L1 loss (Sec. 3.4
  Eq. 12, L1 term).  Gradients are the exact derivative of this forward,
  taken by torch autograd in float64 (predicates and floors held fixed).

Readings of passages the paper leaves open:
  * contraction maps onto (0,1) with x = 0.25*m + 0.5 (the printed "+1"
    contradicts the stated (0,1) range);
  * the scene box normalisation is p' = (p - centre) * inv_half_extent;
  * hash encoding as Instant-NGP: N_l = floor(N_min * b^l); dense 1:1
    indexing when (N_l+1)^3 <= T, else the XOR-prime spatial hash mod T;
    grid coordinate g = x * N_l, no half-cell offset;
  * decoders are bias-free ReLU MLPs with no output activation; the geometry
    decoder reads f_geo, the colour decoder reads [f_rad ; PE(dir)];
  * PE(dir) = NeRF frequency encoding, 4 octaves of sin then cos -> 24 values;
  * aggregation: opacity, colour and per-axis scale through the sigmoid,
    rotation q = Normalize(r_n + r_e) (r_e = 0 is the paper's case);
  * 3DGS rasterizer conventions: 0.3 px^2 dilation, alpha clamped to 0.99,
    a splat contributes iff alpha >= 1/255, blending stops before the
    transmittance would fall below 1e-4, pixel centres at (x+.5, y+.5);
  * pre-cull keeps a Gaussian iff its depth exceeds z_near and its projected
    centre lies within the image frame widened by tol on each side, in the
    frame's normalised coordinates;
  * background: sphere at the world origin, radius r, positive root; colour
    c_s = sigmoid(colour decoder(Theta_rad(contract(p_s)), PE(ray dir)));
    in render mode it is added only where the final transmittance exceeds
    tau_T (the text's "lower than" is read as inverted), in train mode
    everywhere;
  * ties in depth are ordered by Gaussian index.

Integer decisions -- the pre-cull predicate, the float32 depth key, the
contraction branch and every grid cell / hash index -- are taken in float64
with a fixed operation order (each +, -, *, /, sqrt rounded once, no fused
multiply-add), the same sequence the GPU kernels use, so both sides reach
identical decisions from identical float32 inputs.

Parity of the whole pipeline against paper-printed values is unpinned: the
paper prints no worked example; the per-step pins are in the CPU tests.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence

import torch

F64 = torch.float64

# Spatial-hash primes of Instant-NGP (Mueller et al. 2022, Sec. 3, Eq. 4).
HASH_PRIMES = (1, 2654435761, 805459861)

ALPHA_MIN = 1.0 / 255.0      # 3DGS: splats below this alpha are skipped
ALPHA_MAX = 0.99             # 3DGS: alpha clamp
T_EPS = 1e-4                 # 3DGS: stop before transmittance drops below this
DILATION = 0.3               # 3DGS: low-pass dilation of the 2D covariance (px^2)
PE_OCTAVES = 4
RENDER, TRAIN = 0, 1


def _f64(a) -> torch.Tensor:
    if isinstance(a, torch.Tensor):
        return a.to(F64)
    return torch.as_tensor(a).to(F64)


# ---------------------------------------------------------------- hash grid
def level_resolutions(levels: int, base: float, growth: float) -> List[int]:
    """Instant-NGP level resolutions N_l = floor(N_min * b^l) (Sec. 4.1)."""
    out, s = [], float(base)
    for _ in range(levels):
        out.append(int(math.floor(s)))
        s = s * float(growth)
    return out


def contract(p: torch.Tensor, center, inv_half) -> torch.Tensor:
    """Normalise by the scene box and contract into (0,1)^3.

    Sec. 3.2 Eq. 2 and App. A.1 Eqs. 13-14 (MipNeRF360-style contraction,
    affine map onto (0,1) read as 0.25*m + 0.5).  p: (N,3) float64.
    The operation order is fixed (see module docstring)."""
    c = _f64(center).reshape(1, 3)
    h = _f64(inv_half).reshape(1, 3)
    q = (p - c) * h
    n2 = (q[:, 0] * q[:, 0] + q[:, 1] * q[:, 1]) + q[:, 2] * q[:, 2]
    outer = n2 > 1.0
    n = torch.sqrt(torch.where(outer, n2, torch.ones_like(n2)))
    s = (2.0 - 1.0 / n) / n
    m = torch.where(outer[:, None], q * s[:, None], q)
    return m * 0.25 + 0.5


def grid_cell(x: torch.Tensor, res: int):
    """Cell index i (int64, clamped to [0, res-1]) and local coordinate w."""
    g = x * float(res)
    i = torch.clamp(torch.floor(g.detach()), 0.0, float(res - 1))
    w = g - i
    return i.to(torch.int64), w


def corner_index(c: torch.Tensor, res: int, T: int) -> torch.Tensor:
    """Table row of integer grid vertices c (..., 3) at a level of resolution
    `res` in a table of T rows: dense 1:1 when (res+1)^3 <= T (x fastest),
    otherwise the XOR-prime spatial hash modulo T (Instant-NGP Eq. 4)."""
    if (res + 1) ** 3 <= T:
        s = res + 1
        return c[..., 0] + c[..., 1] * s + c[..., 2] * (s * s)
    h = (c[..., 0] * HASH_PRIMES[0]) ^ (c[..., 1] * HASH_PRIMES[1]) ^ (c[..., 2] * HASH_PRIMES[2])
    return (h & 0xFFFFFFFF) % T


CORNERS = torch.tensor([[(k >> 0) & 1, (k >> 1) & 1, (k >> 2) & 1] for k in range(8)], dtype=torch.int64)


def hash_encode(x: torch.Tensor, table: torch.Tensor, resolutions: Sequence[int],
                return_index: bool = False):
    """Multi-resolution hash encoding enc(x; Theta) (Sec. 3.2 Eq. 3).

    x: (N,3) float64 in [0,1]; table: (L, T, F) float64.  Returns (N, L*F)
    features, level-major / feature-minor, trilinearly interpolated from the
    8 vertices of the cell containing x at every level; optionally the
    (N, L, 8) table rows (corner k = dx + 2 dy + 4 dz)."""
    L, T, F = table.shape
    feats, idxs = [], []
    for l, res in enumerate(resolutions[:L]):
        i, w = grid_cell(x, res)
        c = i[:, None, :] + CORNERS[None, :, :]                   # (N,8,3)
        idx = corner_index(c, res, T)                              # (N,8)
        d = CORNERS.to(F64)[None]                                  # (1,8,3)
        wc = torch.prod(d * w[:, None, :] + (1.0 - d) * (1.0 - w[:, None, :]), dim=2)  # (N,8)
        vals = table[l][idx]                                       # (N,8,F)
        feats.append(torch.sum(wc[:, :, None] * vals, dim=1))      # (N,F)
        idxs.append(idx)
    f = torch.cat(feats, dim=1)
    if return_index:
        return f, torch.stack(idxs, dim=1)
    return f


# ---------------------------------------------------------------- decoders
def mlp(h: torch.Tensor, layers: Sequence[torch.Tensor]) -> torch.Tensor:
    """Bias-free ReLU MLP, raw (unactivated) output (Sec. 3.2 Eqs. 4, 6).
    layers: row-major [out][in] matrices in order."""
    for W in layers[:-1]:
        h = torch.relu(h @ W.T)
    return h @ layers[-1].T


def pos_enc(d: torch.Tensor, octaves: int = PE_OCTAVES) -> torch.Tensor:
    """NeRF frequency encoding of unit directions (Sec. 3.2 Eq. 5):
    for k = 0..octaves-1: sin(2^k pi d) (3 values) then cos(2^k pi d) (3)."""
    out = []
    for k in range(octaves):
        a = d * (math.pi * (2.0 ** k))
        out.append(torch.sin(a))
        out.append(torch.cos(a))
    return torch.cat(out, dim=1)


def camera_center(cam) -> torch.Tensor:
    R = _f64(cam.R)
    t = _f64(cam.t)
    return -(R.T @ t)


def aggregate(geo_raw, col_raw, opac_e, scale_e, col_e, rot_e):
    """Aggregation with the explicit Gaussian (Sec. 3.2 Eq. 7):
    opacity = sig(a_n + a_e), colour = sig(c_n + c_e), scale = sig(s_n + s_e),
    rotation = Normalize(r_n (+ r_e))."""
    a_n, s_n, r_n = geo_raw[:, 0], geo_raw[:, 1:4], geo_raw[:, 4:8]
    opacity = torch.sigmoid(a_n + opac_e)
    scale = torch.sigmoid(s_n + scale_e)
    r = r_n if rot_e is None else r_n + rot_e
    quat = r / torch.linalg.vector_norm(r, dim=1, keepdim=True)
    rgb = torch.sigmoid(col_raw + col_e)
    return opacity, scale, quat, rgb


# ---------------------------------------------------------------- culling
def camera_space(p: torch.Tensor, cam) -> torch.Tensor:
    """t = R p + t (Sec. 3.3 Eq. 8), fixed order ((R0 x + R1 y) + R2 z) + t."""
    R = _f64(cam.R)
    tt = _f64(cam.t)
    rows = []
    for r in range(3):
        rows.append(((R[r, 0] * p[:, 0] + R[r, 1] * p[:, 1]) + R[r, 2] * p[:, 2]) + tt[r])
    return torch.stack(rows, dim=1)


def precull(p: torch.Tensor, cam) -> torch.Tensor:
    """Visibility pre-culling (Sec. 3.3 Eq. 9): keep iff the depth exceeds
    z_near and the projected centre lies within [-(1+tol), 1+tol] of the
    image frame's normalised coordinates."""
    with torch.no_grad():
        t = camera_space(p.detach(), cam)
        fx, fy = _f64(cam.fx), _f64(cam.fy)
        cx, cy = _f64(cam.cx), _f64(cam.cy)
        W, H = float(cam.width), float(cam.height)
        lim = 1.0 + _f64(torch.tensor(cam.cull_tol, dtype=torch.float32))
        zn = _f64(torch.tensor(cam.z_near, dtype=torch.float32))
        front = t[:, 2] > zn
        tz = torch.where(front, t[:, 2], torch.ones_like(t[:, 2]))
        u = (fx * t[:, 0]) / tz + cx
        v = (fy * t[:, 1]) / tz + cy
        nx = (2.0 * u) / W - 1.0
        ny = (2.0 * v) / H - 1.0
        return front & (torch.abs(nx) <= lim) & (torch.abs(ny) <= lim)


def depth_key(p: torch.Tensor, cam) -> torch.Tensor:
    """Per-Gaussian depth used for ordering: camera z rounded to float32."""
    with torch.no_grad():
        return camera_space(p.detach(), cam)[:, 2].to(torch.float32)


# ---------------------------------------------------------------- projection
def quat_to_rot(q: torch.Tensor) -> torch.Tensor:
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], 1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], 1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 1),
    ], 1)


def project(p, scale, quat, cam):
    """EWA splatting (3DGS rasterizer, Sec. 3.1): 3D covariance
    Sigma = R_q diag(s^2) R_q^T, local affine Jacobian J of the pinhole map at
    the camera-space centre, 2D covariance J W Sigma W^T J^T + 0.3 I, conic
    = its inverse, projected centre (u, v)."""
    t = camera_space(p, cam)
    fx, fy = _f64(cam.fx), _f64(cam.fy)
    tx, ty, tz = t[:, 0], t[:, 1], t[:, 2]
    u = (fx * tx) / tz + _f64(cam.cx)
    v = (fy * ty) / tz + _f64(cam.cy)
    Rq = quat_to_rot(quat)
    S2 = scale * scale
    Sigma = Rq @ torch.diag_embed(S2) @ Rq.transpose(1, 2)
    zero = torch.zeros_like(tz)
    J = torch.stack([torch.stack([fx / tz, zero, -fx * tx / (tz * tz)], 1),
                     torch.stack([zero, fy / tz, -fy * ty / (tz * tz)], 1)], 1)   # (N,2,3)
    M = J @ _f64(cam.R)[None]
    cov = M @ Sigma @ M.transpose(1, 2)
    a = cov[:, 0, 0] + DILATION
    b = cov[:, 0, 1]
    c = cov[:, 1, 1] + DILATION
    det = a * c - b * b
    conic = torch.stack([c / det, -b / det, a / det], 1)
    return dict(u=u, v=v, conic=conic, cov2d=torch.stack([a, b, c], 1), det=det, depth=tz)


def splat_extent(cov2d: torch.Tensor, opacity: torch.Tensor):
    """Conservative half-extents (px) of the region where alpha >= 1/255:
    sqrt(2 ln(255 o)) * sqrt(cov_xx) (resp. yy), plus one pixel."""
    lo = torch.clamp(255.0 * opacity.detach(), min=1.0)
    k = torch.sqrt(2.0 * torch.log(lo))
    return k * torch.sqrt(cov2d[:, 0].detach()) + 1.0, k * torch.sqrt(cov2d[:, 2].detach()) + 1.0


# ---------------------------------------------------------------- compositing
def _pairs_for_pixels(px, py, u, v, rx, ry, chunk=1 << 22):
    """All (pixel, splat) pairs whose conservative box holds the pixel centre:
    |px + .5 - u| <= rx and |py + .5 - v| <= ry.  No tiling: candidates come
    either from each splat's own box, enumerated pixel by pixel over the
    rectangle spanned by the requested pixels, or (when fewer) from every
    (pixel, splat) combination; the predicate above then decides."""
    P, N = px.numel(), u.numel()
    empty = (torch.zeros(0, dtype=torch.int64), torch.zeros(0, dtype=torch.int64))
    if P == 0 or N == 0:
        return empty
    cxp = px.to(F64) + 0.5
    cyp = py.to(F64) + 0.5

    def exact(pi, si):
        m = (torch.abs(cxp[pi] - u[si]) <= rx[si]) & (torch.abs(cyp[pi] - v[si]) <= ry[si])
        return pi[m], si[m]

    xmin, xmax = int(px.min()), int(px.max())
    ymin, ymax = int(py.min()), int(py.max())
    # each splat's box in pixel indices, widened by one pixel against rounding
    # (the exact predicate decides), clipped to the requested rectangle
    x0 = torch.clamp(torch.floor(u - rx - 0.5) - 1, min=xmin)
    x1 = torch.clamp(torch.ceil(u + rx - 0.5) + 1, max=xmax)
    y0 = torch.clamp(torch.floor(v - ry - 0.5) - 1, min=ymin)
    y1 = torch.clamp(torch.ceil(v + ry - 0.5) + 1, max=ymax)
    nx = torch.clamp(x1 - x0 + 1, min=0).to(torch.int64)
    ny = torch.clamp(y1 - y0 + 1, min=0).to(torch.int64)
    nx = torch.where(rx >= 0, nx, torch.zeros_like(nx))
    area = nx * ny
    pi_list, si_list = [], []
    unique = torch.unique((py - ymin) * (xmax - xmin + 1) + (px - xmin)).numel() == P
    if unique and int(area.sum()) <= P * N:
        Wb = xmax - xmin + 1
        lut = torch.full(((ymax - ymin + 1) * Wb,), -1, dtype=torch.int64)
        lut[(py - ymin) * Wb + (px - xmin)] = torch.arange(P)
        csum = torch.cumsum(area, 0)
        s0 = 0
        while s0 < N:
            base = int(csum[s0 - 1]) if s0 else 0
            s1 = int(torch.searchsorted(csum, torch.tensor(base + chunk, dtype=csum.dtype), right=True))
            s1 = max(s1, s0 + 1)
            sel = torch.arange(s0, min(s1, N))
            cnt = area[sel]
            si = torch.repeat_interleave(sel, cnt)
            k = torch.arange(si.numel()) - torch.repeat_interleave(torch.cumsum(cnt, 0) - cnt, cnt)
            xx = x0[si].to(torch.int64) + k % nx[si]
            yy = y0[si].to(torch.int64) + torch.div(k, nx[si], rounding_mode="floor")
            pi = lut[(yy - ymin) * Wb + (xx - xmin)]
            keep = pi >= 0
            a, b = exact(pi[keep], si[keep])
            pi_list.append(a)
            si_list.append(b)
            s0 = min(s1, N)
    else:
        step = max(1, chunk // N)
        for p0 in range(0, P, step):
            pp = torch.arange(p0, min(P, p0 + step))
            pi = pp.repeat_interleave(N)
            si = torch.arange(N).repeat(pp.numel())
            a, b = exact(pi, si)
            pi_list.append(a)
            si_list.append(b)
    if not pi_list:
        return empty
    return torch.cat(pi_list), torch.cat(si_list)


def composite(px, py, u, v, conic, opacity, rgb, order_rank, rx, ry, return_stats=False):
    """Front-to-back point-based alpha blending (Sec. 3.1 Eq. 1) at pixel
    centres (px+.5, py+.5) over the splats ordered by `order_rank`
    (depth, then index).  Returns colour (P,3), final transmittance (P,)."""
    P = px.numel()
    pi, si = _pairs_for_pixels(px, py, u.detach(), v.detach(), rx, ry)
    key = pi * (int(order_rank.max().item()) + 1 if order_rank.numel() else 1) + order_rank[si]
    key, perm = torch.sort(key, stable=True)
    pi, si = pi[perm], si[perm]
    counts = torch.bincount(pi, minlength=P)
    K = int(counts.max().item()) if counts.numel() else 0
    starts = torch.cumsum(counts, 0) - counts
    slot = torch.arange(pi.numel()) - starts[pi]

    dx = u[si] - (px[pi].to(F64) + 0.5)
    dy = v[si] - (py[pi].to(F64) + 0.5)
    cA, cB, cC = conic[si, 0], conic[si, 1], conic[si, 2]
    power = -0.5 * (cA * dx * dx + cC * dy * dy) - cB * dx * dy
    a_raw = opacity[si] * torch.exp(power)
    alpha = torch.clamp(a_raw, max=ALPHA_MAX)
    contrib = ((alpha.detach() >= ALPHA_MIN) & (power.detach() <= 0.0))
    alpha = torch.where(contrib, alpha, torch.zeros_like(alpha))

    A = torch.zeros(P, max(K, 1), dtype=F64)
    A = A.index_put((pi, slot), alpha)
    Cc = torch.zeros(P, max(K, 1), 3, dtype=F64)
    Cc = Cc.index_put((pi, slot), rgb[si])
    one_minus = 1.0 - A
    T_incl = torch.cumprod(one_minus, dim=1)
    alive = T_incl.detach() >= T_EPS
    T_excl = torch.cat([torch.ones(P, 1, dtype=F64), T_incl[:, :-1]], dim=1)
    w = torch.where(alive, A * T_excl, torch.zeros_like(A))
    C = torch.sum(w[:, :, None] * Cc, dim=1)
    T_final = torch.prod(torch.where(alive, one_minus, torch.ones_like(one_minus)), dim=1)
    if not return_stats:
        return C, T_final
    # distance of every evaluated predicate from its threshold, for the
    # knife-edge policy of the parity tests
    with torch.no_grad():
        Ad = torch.zeros(P, max(K, 1), dtype=F64).index_put((pi, slot), a_raw.detach().clamp(max=ALPHA_MAX))
        ev = torch.zeros(P, max(K, 1), dtype=torch.bool).index_put((pi, slot), torch.ones_like(pi, dtype=torch.bool))
        prev_alive = torch.cat([torch.ones(P, 1, dtype=torch.bool), alive[:, :-1]], dim=1)
        tested = ev & prev_alive
        edge_a = torch.where(tested, torch.abs(255.0 * Ad - 1.0), torch.full_like(Ad, math.inf)).amin(dim=1)
        Tt = torch.where(tested & (A.detach() > 0), torch.abs(T_incl.detach() / T_EPS - 1.0),
                         torch.full_like(Ad, math.inf)).amin(dim=1)
        ncontrib = (alive & (A.detach() > 0)).sum(dim=1)
    return C, T_final, dict(edge_alpha=edge_a, edge_T=Tt, ncontrib=ncontrib)


# ---------------------------------------------------------------- background
def pixel_rays(px, py, cam):
    """World-space ray origin o = -R^T t and direction d = R^T K^{-1}(x+.5, y+.5, 1),
    fixed operation order (sums left to right)."""
    R = _f64(cam.R)
    tt = _f64(cam.t)
    dc0 = ((px.to(F64) + 0.5) - _f64(cam.cx)) / _f64(cam.fx)
    dc1 = ((py.to(F64) + 0.5) - _f64(cam.cy)) / _f64(cam.fy)
    dc2 = torch.ones_like(dc0)
    d = torch.stack([(R[0, j] * dc0 + R[1, j] * dc1) + R[2, j] * dc2 for j in range(3)], 1)
    o = torch.stack([-((R[0, j] * tt[0] + R[1, j] * tt[1]) + R[2, j] * tt[2]) for j in range(3)])
    return o, d


def sphere_hit(o, d, radius):
    """Positive root of |o + t d|^2 = r^2 (App. A.2, Eqs. 15-18):
    A = d.d, B = 2 o.d, C = o.o - r^2, t = (-B + sqrt(B^2 - 4AC)) / (2A)."""
    r = _f64(torch.tensor(radius, dtype=torch.float32))
    A = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    od = (o[0] * d[:, 0] + o[1] * d[:, 1]) + o[2] * d[:, 2]
    B = 2.0 * od
    oo = (o[0] * o[0] + o[1] * o[1]) + o[2] * o[2]
    C = oo - r * r
    disc = B * B - (4.0 * A) * C
    t = (torch.sqrt(disc) - B) / (2.0 * A)
    return o[None, :] + t[:, None] * d, t


def background_colour(px, py, cam, fields, return_index=False):
    """Background colour at the sphere intersection of each pixel's ray
    (Sec. 3.3): c_s = sigmoid(Phi_c([enc(contract(p_s); Theta_rad) ; PE(d/|d|)]))."""
    o, d = pixel_rays(px, py, cam)
    ps, _ = sphere_hit(o, d, fields.bg_radius)
    x = contract(ps, fields.aabb_center, fields.aabb_inv_half)
    enc = hash_encode(x, fields.table_rad, fields.resolutions, return_index=return_index)
    f_rad, idx = (enc if return_index else (enc, None))
    dn = d / torch.linalg.vector_norm(d, dim=1, keepdim=True)
    c = torch.sigmoid(mlp(torch.cat([f_rad, pos_enc(dn)], 1), fields.mlp_col))
    return (c, idx) if return_index else c


# ---------------------------------------------------------------- whole step
@dataclass
class Fields:
    table_geo: torch.Tensor
    table_rad: torch.Tensor
    mlp_geo: List[torch.Tensor]
    mlp_col: List[torch.Tensor]
    resolutions: List[int]
    aabb_center: torch.Tensor
    aabb_inv_half: torch.Tensor
    bg_radius: float = 100.0
    tau_T: float = 0.2


@dataclass
class Params:
    pos: torch.Tensor       # (N,3)
    scale_e: torch.Tensor   # (N,3)
    rot_e: Optional[torch.Tensor]  # (N,4) or None
    opac_e: torch.Tensor    # (N,)
    col_e: torch.Tensor     # (N,3)


def from_scene(scene, requires_grad: bool = False):
    """float64 copies of a hyrf_inputs.Scene (the same float32 values upcast)."""
    def t(a):
        x = torch.from_numpy(a).to(F64).clone()
        x.requires_grad_(requires_grad)
        return x
    cfg = scene.cfg
    params = Params(pos=t(scene.pos.T.copy()), scale_e=t(scene.scale_e.T.copy()),
                    rot_e=None if scene.rot_e is None else t(scene.rot_e.T.copy()),
                    opac_e=t(scene.opac_e), col_e=t(scene.col_e.T.copy()))
    fields = Fields(table_geo=t(scene.table_geo), table_rad=t(scene.table_rad),
                    mlp_geo=[t(w) for w in scene.mlp_geo], mlp_col=[t(w) for w in scene.mlp_col],
                    resolutions=level_resolutions(cfg.levels, cfg.base_res, cfg.growth),
                    aabb_center=torch.from_numpy(scene.aabb_center).to(F64),
                    aabb_inv_half=torch.from_numpy(scene.aabb_inv_half).to(F64),
                    bg_radius=scene.bg_radius, tau_T=scene.tau_T)
    return params, fields


def query_gaussians(params: Params, fields: Fields, idx: torch.Tensor, cam):
    """Field query + aggregation for the Gaussians `idx` seen from `cam`
    (Sec. 3.2 Eqs. 2-7)."""
    p = params.pos[idx]
    x = contract(p, fields.aabb_center, fields.aabb_inv_half)
    f_geo = hash_encode(x, fields.table_geo, fields.resolutions)
    f_rad = hash_encode(x, fields.table_rad, fields.resolutions)
    geo_raw = mlp(f_geo, fields.mlp_geo)
    dvec = p - camera_center(cam)[None]
    dirn = dvec / torch.linalg.vector_norm(dvec, dim=1, keepdim=True)
    col_raw = mlp(torch.cat([f_rad, pos_enc(dirn)], 1), fields.mlp_col)
    rot_e = None if params.rot_e is None else params.rot_e[idx]
    opacity, scale, quat, rgb = aggregate(geo_raw, col_raw, params.opac_e[idx], params.scale_e[idx],
                                          params.col_e[idx], rot_e)
    return dict(p=p, x=x, f_geo=f_geo, f_rad=f_rad, geo_raw=geo_raw, col_raw=col_raw,
                opacity=opacity, scale=scale, quat=quat, rgb=rgb)


def render_view(params: Params, fields: Fields, cam, mode: int = TRAIN,
                pixels: Optional[torch.Tensor] = None, return_stats: bool = False):
    """One view of the render step.  pixels: optional (P,2) int64 (x, y) list
    (default: every pixel, row-major).  Returns dict with 'rgb' (P,3),
    'T' (P,), and the per-Gaussian intermediates."""
    W, H = cam.width, cam.height
    if pixels is None:
        yy, xx = torch.meshgrid(torch.arange(H), torch.arange(W), indexing="ij")
        px, py = xx.reshape(-1), yy.reshape(-1)
    else:
        px, py = pixels[:, 0], pixels[:, 1]
    keep = precull(params.pos, cam)
    idx = torch.nonzero(keep, as_tuple=True)[0]
    q = query_gaussians(params, fields, idx, cam)
    pr = project(q["p"], q["scale"], q["quat"], cam)
    valid = pr["det"].detach() > 0
    dk = depth_key(q["p"], cam)
    # global order: float32 depth, then Gaussian index
    order = torch.argsort(idx, stable=True)
    order = order[torch.argsort(dk[order], stable=True)]
    rank = torch.empty_like(order)
    rank[order] = torch.arange(order.numel())
    rx, ry = splat_extent(pr["cov2d"], q["opacity"])
    inf_box = ~valid
    rx = torch.where(inf_box, torch.full_like(rx, -1.0), rx)
    res = composite(px, py, pr["u"], pr["v"], pr["conic"], q["opacity"], q["rgb"], rank, rx, ry,
                    return_stats=return_stats)
    C_fg, T_final = res[0], res[1]
    need = torch.ones_like(T_final, dtype=torch.bool) if mode == TRAIN else (T_final.detach() > fields.tau_T)
    out = C_fg.clone()
    if bool(need.any()):
        cs = background_colour(px[need], py[need], cam, fields)
        out = out.index_put((torch.nonzero(need, as_tuple=True)[0],), C_fg[need] + T_final[need, None] * cs)
    result = dict(rgb=out, rgb_fg=C_fg, T=T_final, vis_idx=idx, query=q, proj=pr, depth_key=dk, px=px, py=py,
                  rank=rank, rx=rx, ry=ry, mode=mode, cam=cam, fields=fields, bg_added=need)
    if return_stats:
        result["stats"] = res[2]
    return result


# ---------------------------------------------------------------- decision variants
def blend_pixel(alpha, power, rgb, flip_alpha: int = -1, flip_stop: int = -1):
    """Front-to-back blending of one pixel (Sec. 3.1 Eq. 1 with the 3DGS
    rules) over its depth-ordered pairs, in plain Python, with at most one
    decision negated: the contribution test of pair `flip_alpha`
    (alpha >= 1/255 and power <= 0) or the early-stop test at pair
    `flip_stop` (stop before T (1 - alpha) < 1e-4).  alpha: the clamped
    min(0.99, o e^power) per pair.  Returns (C_fg[3], T_final)."""
    T = 1.0
    C = [0.0, 0.0, 0.0]
    for j, (a, pw, c) in enumerate(zip(alpha, power, rgb)):
        take = (a >= ALPHA_MIN) and (pw <= 0.0)
        if j == flip_alpha:
            take = not take
        if not take:
            continue
        tT = T * (1.0 - a)
        stop = tT < T_EPS
        if j == flip_stop:
            stop = not stop
        if stop:
            break
        for ch in range(3):
            C[ch] += c[ch] * a * T
        T = tT
    return C, T


def decision_variants(r, ks, delta_alpha: float, delta_T: float):
    """For pixels `ks` (indices into r['px']) of a render_view result r: the
    oracle's colour, and the colour the same pixel takes when ONE of its
    threshold decisions that lies within a relative distance delta of its
    threshold is taken the other way -- a pair's alpha >= 1/255 test
    (|255 alpha - 1| < delta_alpha), an early-stop test
    (|T (1 - alpha) / 1e-4 - 1| < delta_T) or, in render mode, the background
    test T_final > tau_T (|T_final / tau_T - 1| < delta_T).  Colours include
    the background term of Sec. 3.3 Eq. 10.  Returns, per pixel, a list of
    (kind, pair, distance, rgb[3]) with kind 'base', 'alpha', 'stop' or 'tau'
    and distance the decision's relative distance from its threshold."""
    ks = torch.as_tensor(ks, dtype=torch.int64)
    if ks.numel() == 0:
        return []
    q, pr, cam, fields = r["query"], r["proj"], r["cam"], r["fields"]
    with torch.no_grad():
        px, py = r["px"][ks], r["py"][ks]
        u, v, conic = pr["u"].detach(), pr["v"].detach(), pr["conic"].detach()
        opac, rgb = q["opacity"].detach(), q["rgb"].detach()
        pi, si = _pairs_for_pixels(px, py, u, v, r["rx"].detach(), r["ry"].detach())
        cs = background_colour(px, py, cam, fields)
    out = []
    for m in range(ks.numel()):
        s = si[pi == m]
        s = s[torch.argsort(r["rank"][s])]
        dx = u[s] - (float(px[m]) + 0.5)
        dy = v[s] - (float(py[m]) + 0.5)
        power = -0.5 * (conic[s, 0] * dx * dx + conic[s, 2] * dy * dy) - conic[s, 1] * dx * dy
        alpha = torch.clamp(opac[s] * torch.exp(power), max=ALPHA_MAX)
        al, pw, cl = alpha.tolist(), power.tolist(), rgb[s].tolist()
        c_s = cs[m].tolist()

        def full(C, T, tau_flip=False):
            bg = True if r["mode"] == TRAIN else (T > fields.tau_T)
            if tau_flip:
                bg = not bg
            return [C[ch] + (T * c_s[ch] if bg else 0.0) for ch in range(3)]
        C0, T0 = blend_pixel(al, pw, cl)
        var = [("base", -1, 0.0, full(C0, T0))]
        T = 1.0
        for j in range(len(al)):
            take = al[j] >= ALPHA_MIN and pw[j] <= 0.0
            da = abs(255.0 * al[j] - 1.0)
            if da < delta_alpha:
                var.append(("alpha", j, da, full(*blend_pixel(al, pw, cl, flip_alpha=j))))
            if not take:
                continue
            tT = T * (1.0 - al[j])
            dt = abs(tT / T_EPS - 1.0)
            if dt < delta_T:
                var.append(("stop", j, dt, full(*blend_pixel(al, pw, cl, flip_stop=j))))
            if tT < T_EPS:
                break
            T = tT
        dtau = abs(T0 / fields.tau_T - 1.0)
        if r["mode"] == RENDER and dtau < delta_T:
            var.append(("tau", -1, dtau, full(C0, T0, tau_flip=True)))
        out.append(var)
    return out


def render_image(params, fields, cam, mode=TRAIN, return_stats=False):
    """Full image (3, H, W) plus final transmittance (H, W)."""
    r = render_view(params, fields, cam, mode, return_stats=return_stats)
    H, W = cam.height, cam.width
    r["image"] = r["rgb"].T.reshape(3, H, W)
    r["T_img"] = r["T"].reshape(H, W)
    return r


def l1_loss(img: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
    """L1 photometric term of the training loss (Sec. 3.4 Eq. 12), mean over
    all pixels and channels."""
    return torch.mean(torch.abs(img - target))


# ---------------------------------------------------------------- binning
def bin_and_sort(depth_f32: torch.Tensor, rect: torch.Tensor, tiles_x: int, tiles_y: int):
    """Tile binning with depth ordering, as the 3DGS rasterizer orders splats
    (Sec. 3.1: Gaussians ordered by depth).  depth_f32: (V, n) float32 > 0;
    rect: (V, n, 4) int [x0, y0, x1, y1) in tile units.  Every splat is listed
    once for each tile its rectangle covers; the list is ordered by
    (view, tile, depth, splat index).  Returns (tile_key int64 per entry,
    splat id = view*n + i per entry, ranges (V*tiles, 2) [first, last))."""
    V, n = depth_f32.shape
    ntile = tiles_x * tiles_y
    ent_view, ent_tile, ent_depth, ent_id = [], [], [], []
    for vw in range(V):
        for i in range(n):
            x0, y0, x1, y1 = [int(a) for a in rect[vw, i]]
            for ty in range(y0, y1):
                for tx in range(x0, x1):
                    ent_view.append(vw)
                    ent_tile.append(ty * tiles_x + tx)
                    ent_depth.append(float(depth_f32[vw, i]))
                    ent_id.append(vw * n + i)
    order = sorted(range(len(ent_id)), key=lambda k: (ent_view[k], ent_tile[k], ent_depth[k], ent_id[k]))
    keys = torch.tensor([ent_view[k] * ntile + ent_tile[k] for k in order], dtype=torch.int64)
    ids = torch.tensor([ent_id[k] for k in order], dtype=torch.int64)
    ranges = torch.zeros(V * ntile, 2, dtype=torch.int64)
    for pos, k in enumerate(keys.tolist()):
        if pos == 0 or keys[pos - 1] != k:
            ranges[k, 0] = pos
        ranges[k, 1] = pos + 1
    return keys, ids, ranges
