"""Comparison rule of the image parity checks (TEST INFRASTRUCTURE: used by
the tests and the smoke check only; the product never imports it).

A float32 render and the float64 oracle take the same threshold decisions
except where a decision's operand lies within float32 rounding of its
threshold (Sec. 3.1 Eq. 1 with the 3DGS rules: alpha >= 1/255, stop before
T (1 - alpha) < 1e-4; Sec. 3.3: background where T_final > tau_T in render
mode).  The rule: every pixel of the GPU image must equal the oracle's
colour within `atol`, or else equal within `atol` the oracle's colour with
ONE such decision taken the other way, where that decision lies within a
relative distance delta of its threshold (delta_alpha for the alpha test,
delta_T for the early-stop and background tests).  Pixels explained by a
flipped decision are counted and must stay below `max_flip_frac`; no pixel
is left out of the comparison.
"""
from __future__ import annotations

import numpy as np

from oracle import hyrf_oracle as O


def compare_pixels(gpu_rgb, r, atol=1e-5, delta_alpha=1e-4, delta_T=1e-4, max_flip_frac=0.01, gpu_T=None,
                   search=10.0):
    """gpu_rgb: (P, 3) GPU colours of the pixels r['px'], r['py'] of the
    oracle's render_view result r.  gpu_T: optional (P,) GPU final
    transmittance, for the report only.  Returns a dict with ok, max_err
    (over pixels matching the oracle), n_flip (pixels explained by one
    near-threshold decision), n_bad (pixels explained by nothing), and the
    largest relative threshold distance among the flipped decisions per kind
    ('alpha', 'stop', 'tau'); 'flipped' lists the explained pixels."""
    ref = r["rgb"].detach().numpy()
    gpu = np.asarray(gpu_rgb, dtype=np.float64)
    diff = np.abs(gpu - ref).max(axis=1)
    off = np.nonzero(diff > atol)[0]
    flipped, bad, worst = [], [], {}
    limits = {"alpha": delta_alpha, "stop": delta_T, "tau": delta_T}
    for k, var in zip(off.tolist(), O.decision_variants(r, off, search * delta_alpha, search * delta_T)):
        best = None
        for kind, j, dist, rgb in var[1:]:
            e = max(abs(gpu[k, ch] - rgb[ch]) for ch in range(3))
            if e <= atol and (best is None or dist / limits[kind] < best[1] / limits[best[0]]):
                best = (kind, dist)
        if best is not None:
            worst[best[0]] = max(worst.get(best[0], 0.0), best[1])
        if best is not None and best[1] < limits[best[0]]:
            flipped.append(int(k))
        else:
            bad.append(dict(pixel=int(k), err=float(diff[k]), nearest=best))
    ok_px = np.ones(diff.shape, bool)
    ok_px[off] = False
    out = dict(max_err=float(diff[ok_px].max()) if ok_px.any() else 0.0, n_flip=len(flipped), n_bad=len(bad),
               flip_frac=len(flipped) / float(max(diff.size, 1)), flipped_distance=worst, bad=bad[:10],
               flipped=flipped)
    if gpu_T is not None:
        T_ref = r["T"].detach().numpy()
        rel = np.abs(np.asarray(gpu_T, np.float64).reshape(-1) - T_ref) / T_ref
        out["T_rel_err_max"] = float(rel[ok_px].max()) if ok_px.any() else 0.0
    out["ok"] = out["n_bad"] == 0 and out["flip_frac"] <= max_flip_frac
    return out


def compare_image(gpu_rgb_planar, r, H, W, gpu_T=None, **kw):
    """compare_pixels for a whole (3, H, W) image; r covers the H x W pixels
    row-major; gpu_T optional (H, W)."""
    g = np.asarray(gpu_rgb_planar).reshape(3, H * W).T
    return compare_pixels(g, r, gpu_T=None if gpu_T is None else np.asarray(gpu_T).reshape(-1), **kw)
