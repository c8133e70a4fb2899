"""Ablation of the adaptive densification (Sec. III-A, Table 6) on synthetic RGB-D frames.

Five seedings of the same frame are each mapped for the same number of iterations, with pruning
(Sec. III-D) at fixed intervals:

* sparse equidistant, large gaussians: lattice stride n everywhere, radius factor alpha_l;
* sparse equidistant, small gaussians: stride n, radius factor alpha_h;
* dense equidistant, large / small gaussians: stride m everywhere, alpha_l / alpha_h;
* adaptive (the method): stride m and alpha_h inside the high-frequency mask, n and alpha_l
  outside it.

The equidistant seedings run the library's seeding with both strides and both radius factors
equal, so that the frequency mask changes nothing. Reported per variant: the final PSNR and SSIM of
the rendering against the frame (colour; the SSIM of the mapping loss's term), gaussians seeded and
kept, the map's memory (56 bytes per gaussian; 168 with the Adam moments) and device milliseconds
per mapping iteration. LPIPS, the table's third image metric, needs a trained network and is not
computed.
"""
from __future__ import annotations

import math

import numpy as np

from .prior import MAP_LR, frame_of

BYTES_PER_GAUSSIAN = 56        # 14 FP32 parameters
BYTES_WITH_ADAM = 3 * 56       # parameters and the two Adam moments

# name -> (m, n, alpha_h, alpha_l) of the seeding; m = n and alpha_h = alpha_l make it equidistant
VARIANTS = {
    "sparse_large": (8, 8, 4.0, 4.0),
    "sparse_small": (8, 8, 1.0, 1.0),
    "dense_large": (2, 2, 4.0, 4.0),
    "dense_small": (2, 2, 1.0, 1.0),
    "adaptive": (2, 8, 1.0, 4.0),
}


def run_variant(F, ctx, frame, variant: str, iters: int = 200, prune_every: int = 50, prune_opts=None,
                opacity: float = 0.9, loss_opts=None) -> dict:
    """Seed `frame` with `variant`, map it for `iters` iterations against itself, pruning after
    every `prune_every` iterations and at the end (default thresholds: opacity 0.005, scale 0.25 m);
    then render and measure."""
    import torch
    m, n, ah, al = VARIANTS[variant]
    so = F.SeedOpts(m=m, n=n, alpha_h=ah, alpha_l=al, opacity_logit=math.log(opacity / (1.0 - opacity)))
    prune_opts = prune_opts or F.PruneOpts(0.005, 0.25)
    rgb = torch.as_tensor(frame.rgb).cuda()
    depth = torch.as_tensor(frame.depth).cuda()
    H, W = frame.depth.shape
    cap = (W * H) // (m * m) + W + H + 16
    params = torch.zeros((14, cap), dtype=torch.float32, device="cuda")
    s = F.seed_gaussians(ctx, rgb, depth, frame.cam, so, capacity=cap, params=params)
    seeded = count = s["n"]
    adam = F.Adam.like(params, lr=MAP_LR)
    opts = F.RenderOpts()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    kept_after = []
    ev0.record(stream)
    for k in range(iters):
        F.map_step(ctx, params, count, adam, [frame.cam], [(rgb, depth)], opts, loss_opts)
        if (k + 1) % prune_every == 0 or k + 1 == iters:
            params, count, adam = F.prune(ctx, params, count, prune_opts, adam=adam)
            kept_after.append(count)
    ev1.record(stream)
    torch.cuda.synchronize()
    ctx.check()
    ms = ev0.elapsed_time(ev1)
    out = F.render(ctx, params, count, frame.cam, opts, aux=False)
    dr, dd = torch.empty_like(out["rgb"]), torch.empty_like(out["depth"])
    psnr, loss, ssim = (torch.zeros(1, device="cuda") for _ in range(3))
    F.loss_l1(ctx, out["rgb"], out["depth"], rgb, depth, F.LossOpts(), dr, dd, loss, psnr)
    F.ssim(ctx, out["rgb"], rgb, ssim)
    torch.cuda.synchronize()
    ctx.check()
    return dict(variant=variant, seeded=int(seeded), kept=int(count), kept_after_each_prune=kept_after,
                psnr_db=float(psnr.item()), ssim=float(ssim.item()), map_mb=count * BYTES_PER_GAUSSIAN / 1e6,
                map_with_adam_mb=count * BYTES_WITH_ADAM / 1e6, ms_per_iter=ms / iters)


def run(F, ctx, scenes, iters: int = 200, prune_every: int = 50, prune_opts=None, opacity: float = 0.9,
        variants=tuple(VARIANTS), log=None) -> dict:
    """Every variant on every scene (synthetic 640x480 frames); returns the per-scene rows and the
    mean of each measure per variant."""
    log = log or (lambda msg: None)
    rows = []
    for s in scenes:
        fr = frame_of(s)
        for v in variants:
            rows.append(dict(scene=int(s), **run_variant(F, ctx, fr, v, iters, prune_every, prune_opts, opacity)))
        log(f"scene {s} done")
    keys = ("psnr_db", "ssim", "seeded", "kept", "map_mb", "map_with_adam_mb", "ms_per_iter")
    summary = {}
    for v in variants:
        rs = [r for r in rows if r["variant"] == v]
        summary[v] = {k: float(np.mean([r[k] for r in rs])) for k in keys}
        summary[v]["psnr_db_std"] = float(np.std([r["psnr_db"] for r in rs]))
    return dict(summary=summary, rows=rows)
