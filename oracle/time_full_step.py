"""Wall time of the FP64 oracle's full train step (TEST INFRASTRUCTURE: the
oracle is never called by the product; this times it as a CPU baseline).

    python -m oracle.time_full_step --config tiny --threads 1
    python -m oracle.time_full_step --config c100k --threads 16

One step = field query and aggregation of every pre-cull survivor,
projection, untiled blending of every pixel with the background (train
mode), the L1 loss against the oracle's render of the seeded second scene
(seed 2001) and the exact backward (torch autograd) of every explicit
parameter, both tables and both decoders.  Prints one JSON line with the
median of `--repeats` runs.  `--chunk-rows R` evaluates the image in bands
of R pixel rows (the loss is a sum over pixels, so the gradient is the sum
of the bands' gradients); each band repeats the per-Gaussian work, so the
time is an upper bound of the one-pass step, whose dense per-pixel arrays
would not fit in memory at 100k Gaussians and 800x800.
"""
from __future__ import annotations

import argparse
import json
import os
import resource
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def time_step(config: str, threads: int, repeats: int = 3, chunk_rows: int = 0) -> dict:
    """Median wall time of the oracle's full train step (see the module
    docstring) on `threads` host threads."""
    import torch

    import hyrf_inputs as hi
    from oracle import hyrf_oracle as O

    prev = torch.get_num_threads()
    torch.set_num_threads(threads)
    cfg = hi.CONFIGS[config]
    scene = hi.make_scene(cfg)
    cam = hi.make_cameras(cfg)[0]
    tscene = hi.make_scene(cfg, seed=2001)
    tp, tf = O.from_scene(tscene)
    rows = chunk_rows if chunk_rows > 0 else cam.height

    def band(y0):
        yy, xx = torch.meshgrid(torch.arange(y0, min(cam.height, y0 + rows)), torch.arange(cam.width), indexing="ij")
        return torch.stack([xx.reshape(-1), yy.reshape(-1)], 1)
    with torch.no_grad():
        target = torch.cat([O.render_view(tp, tf, cam, O.TRAIN, pixels=band(y0))["rgb"]
                            for y0 in range(0, cam.height, rows)])
    times = []
    for _ in range(repeats):
        params, fields = O.from_scene(scene, requires_grad=True)
        leaves = [t for t in (params.pos, params.scale_e, params.rot_e, params.opac_e, params.col_e,
                              fields.table_geo, fields.table_rad) if t is not None]
        leaves += list(fields.mlp_geo) + list(fields.mlp_col)
        t0 = time.perf_counter()
        grads = None
        for y0 in range(0, cam.height, rows):
            pix = band(y0)
            r = O.render_view(params, fields, cam, O.TRAIN, pixels=pix)
            # L1 over the whole image = (sum over bands of |C - C_tgt|) / (3 H W)
            part = torch.sum(torch.abs(r["rgb"] - target[y0 * cam.width:y0 * cam.width + pix.shape[0]]))
            g = torch.autograd.grad(part / (3.0 * cam.height * cam.width), leaves)
            grads = list(g) if grads is None else [a + b for a, b in zip(grads, g)]
        times.append(time.perf_counter() - t0)
    out = {"config": cfg.name, "gaussians": cfg.n_gauss, "image": f"{cam.width}x{cam.height}",
           "threads": torch.get_num_threads(), "repeats": repeats, "chunk_rows": rows,
           "train_step_ms_median": round(1e3 * statistics.median(times), 1),
           "train_step_ms_all": [round(1e3 * t, 1) for t in times],
           "peak_rss_gb": round(resource.getrusage(resource.RUSAGE_SELF).ru_maxrss / 2 ** 20, 2)}
    torch.set_num_threads(prev)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="tiny")
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--repeats", type=int, default=3)
    ap.add_argument("--chunk-rows", type=int, default=0)
    args = ap.parse_args()
    print(json.dumps(time_step(args.config, args.threads, args.repeats, args.chunk_rows)), flush=True)


if __name__ == "__main__":
    main()
