"""Training and evaluation driver of the learned seeding prior.

The data come from the plain method itself: a frame is seeded by the Fourier rule (Sec. III-A,
Eq. 11 radii, one initial opacity) and mapped for a fixed number of iterations against that frame
(the colour and depth L1 terms of the mapping loss); what the gaussians converged to, per 16x16
tile, is the network's target:

* log-scale offsets: each seed's converged log-scales sorted in descending order, minus the log
  of its Eq. 11 radius (alpha d / fx with alpha by its frequency class), averaged over the
  tile's seeds (three values);
* opacity: the tile's mean converged opacity logit.

The network (fgs_prior.h) is trained on the GPU by the library's own forward, backward and Adam
kernels. Evaluation seeds held-out frames both ways and maps them, recording PSNR and device
timestamps after every iteration, and reports iterations and milliseconds until each run reaches
the plain run's final PSNR less a margin.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

MAP_LR = (1e-3, 5e-3, 1e-3, 5e-2, 2.5e-3)


@dataclass
class Frame:
    rgb: np.ndarray   # (3, H, W) float32
    depth: np.ndarray  # (H, W) float32
    cam: object


def frame_of(seed: int, width: int = 640, height: int = 480, n_rect: int = 40) -> Frame:
    import synth
    rgb, depth = synth.rgbd_frame(seed, width, height, n_rect=n_rect)
    cam = synth.camera_tum() if (width, height) == (640, 480) else synth.centred_camera(width, height, 525.0)
    return Frame(rgb, depth, cam)


@dataclass
class MapRun:
    n: int
    params: object          # (14, capacity) device tensor after mapping
    psnr: np.ndarray        # PSNR after every iteration
    ms: np.ndarray          # device time from the start of seeding to the end of every iteration
    seed_ms: float          # seeding (and prior inference) time
    pixel: np.ndarray = field(default=None)
    is_high: np.ndarray = field(default=None)
    from_prior: np.ndarray = field(default=None)


def seed_and_map(F, ctx, frame: Frame, iters: int, seed_opts, lr=MAP_LR, opts=None) -> MapRun:
    """Seed `frame` and map it for `iters` iterations against itself; PSNR and device timestamps
    are kept in device memory and read once at the end."""
    import torch
    d_rgb = torch.as_tensor(frame.rgb).cuda()
    d_depth = torch.as_tensor(frame.depth).cuda()
    H, W = frame.depth.shape
    cap = (W * H) // (seed_opts.m * seed_opts.m) + W + H + 16
    params = torch.zeros((14, cap), dtype=torch.float32, device="cuda")
    opts = opts or F.RenderOpts()
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(iters + 2)]
    ev[0].record(stream)
    s = F.seed_gaussians(ctx, d_rgb, d_depth, frame.cam, seed_opts, capacity=cap, params=params)
    ev[1].record(stream)
    n = s["n"]
    adam = F.Adam.like(params, lr=lr)
    psnr = torch.zeros(iters, device="cuda")
    targets = [(d_rgb, d_depth)]
    for k in range(iters):
        F.map_step(ctx, params, n, adam, [frame.cam], targets, opts, psnr=psnr[k:k + 1])
        ev[k + 2].record(stream)
    torch.cuda.synchronize()
    ctx.check()
    ms = np.array([ev[0].elapsed_time(ev[k + 2]) for k in range(iters)])
    run = MapRun(n, params, psnr.cpu().numpy().astype(np.float64), ms, ev[0].elapsed_time(ev[1]))
    run.pixel = s["pixel"][:n].cpu().numpy()
    run.is_high = s["is_high"][:n].cpu().numpy().astype(bool)
    if "from_prior" in s:
        run.from_prior = s["from_prior"][:n].cpu().numpy().astype(bool)
    return run


def tile_targets(run: MapRun, frame: Frame, alpha_h: float = 1.0, alpha_l: float = 4.0):
    """Per 16x16 tile: mean over the tile's seeds of (descending converged log-scales - the log of
    the seed's radius-rule radius) and of the converged opacity logit. Returns (targets [T, 4],
    seeds per tile [T])."""
    H, W = frame.depth.shape
    tx, ty = (W + 15) // 16, (H + 15) // 16
    p = run.params[:, :run.n].cpu().numpy().astype(np.float64)
    pix = run.pixel
    d = frame.depth.ravel()[pix].astype(np.float64)
    alpha = np.where(run.is_high, alpha_h, alpha_l)
    off = -np.sort(-p[3:6], axis=0) - np.log(alpha * d / float(frame.cam.fx))[None, :]
    tile = (pix // W // 16) * tx + (pix % W) // 16
    T = tx * ty
    cnt = np.bincount(tile, minlength=T).astype(np.float64)
    tgt = np.zeros((T, 4))
    for k in range(3):
        tgt[:, k] = np.bincount(tile, weights=off[k], minlength=T)
    tgt[:, 3] = np.bincount(tile, weights=p[10], minlength=T)
    tgt[cnt > 0] /= cnt[cnt > 0, None]
    return tgt, cnt


def build_dataset(F, ctx, scenes, iters: int = 200, tiles_per_scene: int = 100, seed_opts=None, rng_seed: int = 0):
    """(X [N, 260] device, Y [N, 4] device): features and targets of `tiles_per_scene` random tiles
    with at least one seed from each scene's converged map."""
    import torch
    seed_opts = seed_opts or F.SeedOpts()
    g = np.random.default_rng(rng_seed)
    xs, ys = [], []
    for s in scenes:
        fr = frame_of(s)
        run = seed_and_map(F, ctx, fr, iters, seed_opts)
        tgt, cnt = tile_targets(run, fr, seed_opts.alpha_h, seed_opts.alpha_l)
        ok = np.flatnonzero(cnt > 0)
        pick = np.sort(g.choice(ok, size=min(tiles_per_scene, ok.size), replace=False))
        ids = torch.as_tensor(pick.astype(np.int32)).cuda()
        feat, _ = F.tile_features(ctx, torch.as_tensor(fr.rgb).cuda(), torch.as_tensor(fr.depth).cuda(),
                                  seed_opts.depth_min, seed_opts.depth_max, tile_ids=ids)
        xs.append(feat)
        ys.append(torch.as_tensor(tgt[pick].astype(np.float32)).cuda())
        del run
    return torch.cat(xs), torch.cat(ys)


def init_weights(seed: int = 0, out_bias=None):
    """Packed FP32 weights: N(0, 1/fan_in) matrices, zero hidden biases, output bias `out_bias`
    (e.g. the mean target)."""
    g = np.random.default_rng(seed)
    parts = [g.normal(0, 1 / math.sqrt(260), 256 * 260), np.zeros(256), g.normal(0, 1 / math.sqrt(256), 256 * 256),
             np.zeros(256), g.normal(0, 0.1 / math.sqrt(256), 4 * 256),
             np.zeros(4) if out_bias is None else np.asarray(out_bias, np.float64)]
    return np.concatenate(parts).astype(np.float32)


def train(F, ctx, X, Y, steps: int = 2000, lr: float = 1e-3, seed: int = 0):
    """Full-batch Adam on the MSE; returns (weights device tensor, loss curve)."""
    import torch
    w = torch.as_tensor(init_weights(seed, Y.mean(0).cpu().numpy())).cuda()
    adam = F.PriorAdam.like(w, lr=lr)
    losses = torch.zeros(steps, device="cuda")
    for k in range(steps):
        F.prior_train_step(ctx, X, Y, w, adam, loss=losses[k:k + 1])
    return w, losses.cpu().numpy()


def first_reaching(psnr: np.ndarray, target: float):
    hit = np.flatnonzero(psnr >= target)
    return int(hit[0]) if hit.size else None


def _reach(run: MapRun, target: float) -> dict:
    """Iterations and device ms until `run` first reaches `target` dB (None when it never does),
    with the run's seeding (and prior inference) time, seeds and mean ms per mapping iteration."""
    i = first_reaching(run.psnr, target)
    iters = run.psnr.size
    return dict(iters=None if i is None else i + 1, ms=None if i is None else float(run.ms[i]),
                seed_ms=float(run.seed_ms), seeds=int(run.n), final_db=float(run.psnr[-1]),
                ms_per_iter=float((run.ms[-1] - run.seed_ms) / iters))


def evaluate(F, ctx, weights, scenes, iters: int = 200, margin_db: float = 0.1, plain_opts=None, prior_opts=None,
             mode: int = 3):
    """Per held-out scene: the plain run's final PSNR less margin_db is the target; iterations and
    device ms until each run reaches it (None: never within iters), their seeding times, seeds and
    ms per iteration. The plain run is repeated; the repeat's distance from the first is the
    scene's run-to-run spread."""
    plain_opts = plain_opts or F.SeedOpts()
    if prior_opts is None:
        prior_opts = F.SeedOpts(**{k: getattr(plain_opts, k) for k in ("D0", "m", "n", "tile", "alpha_h", "alpha_l",
                                                                       "opacity_logit", "depth_min", "depth_max")})
        prior_opts.use_prior, prior_opts.prior = mode, weights
    rows = []
    for s in scenes:
        fr = frame_of(s)
        a = seed_and_map(F, ctx, fr, iters, plain_opts)
        b = seed_and_map(F, ctx, fr, iters, prior_opts)
        a2 = seed_and_map(F, ctx, fr, iters, plain_opts)
        target = a.psnr[-1] - margin_db
        ra, rb, r2 = _reach(a, target), _reach(b, target), _reach(a2, target)
        rows.append(dict(scene=s, target_db=float(target), plain=ra, prior=rb, plain_repeat=r2,
                         prior_fraction=float(b.from_prior.mean()) if b.from_prior is not None else 0.0))
        del a, b, a2
    return rows


def summarize(rows) -> dict:
    """Headline of evaluate(): a scene is a win when the prior reaches the target sooner than the
    plain runs by more than their spread (|first - repeat|; where the repeat falls short of the
    target, the median spread of the other scenes, against the first run); a scene the prior never
    reaches counts as a loss."""
    wins = losses = failed = 0
    ratios = []
    spread = [abs(r["plain"]["ms"] - r["plain_repeat"]["ms"]) for r in rows
              if r["plain"]["ms"] is not None and r["plain_repeat"]["ms"] is not None]
    med_spread = float(np.median(spread)) if spread else 0.0
    for r in rows:
        a, b, a2 = r["plain"], r["prior"], r["plain_repeat"]
        if b["ms"] is None:
            failed += 1
            losses += 1
            continue
        if a["ms"] is None:
            continue
        if a2["ms"] is not None:
            best, sp = min(a["ms"], a2["ms"]), abs(a["ms"] - a2["ms"])
        else:
            best, sp = a["ms"], med_spread
        ratios.append(b["ms"] / best)
        if b["ms"] < best - sp:
            wins += 1
        else:
            losses += 1

    def mean(key, run):
        v = [r[run][key] for r in rows if r[run][key] is not None]
        return float(np.mean(v)) if v else None

    return dict(
        scenes=len(rows), wins=wins, losses=losses, prior_never_reached=failed,
        plain_never_reached=sum(r["plain"]["ms"] is None for r in rows),
        repeat_short_of_target=sum(r["plain_repeat"]["ms"] is None for r in rows),
        ms_ratio_median=float(np.median(ratios)) if ratios else None,
        ms_ratio_p10=float(np.percentile(ratios, 10)) if ratios else None,
        ms_ratio_p90=float(np.percentile(ratios, 90)) if ratios else None,
        spread_ms_median=float(np.median(spread)) if spread else None,
        plain_ms_mean=mean("ms", "plain"), prior_ms_mean=mean("ms", "prior"),
        plain_iters_mean=mean("iters", "plain"), prior_iters_mean=mean("iters", "prior"),
        plain_seed_ms_mean=mean("seed_ms", "plain"), prior_seed_ms_mean=mean("seed_ms", "prior"),
        plain_ms_per_iter_mean=mean("ms_per_iter", "plain"), prior_ms_per_iter_mean=mean("ms_per_iter", "prior"),
        plain_seeds_mean=mean("seeds", "plain"), prior_seeds_mean=mean("seeds", "prior"),
        plain_final_db=mean("final_db", "plain"), prior_final_db=mean("final_db", "prior"),
        prior_fraction=float(np.mean([r["prior_fraction"] for r in rows])) if rows else None,
    )


def logit(p: float) -> float:
    return math.log(p / (1.0 - p))


def best_plain_opacity(F, ctx, scenes, iters: int, choices=(0.1, 0.5, 0.9)):
    """The plain rule's initial opacity with the best mean final PSNR over `scenes` (the constant
    the plain method is compared at)."""
    best = None
    for o in choices:
        opts = F.SeedOpts(opacity_logit=logit(o))
        ps = [seed_and_map(F, ctx, frame_of(s), iters, opts).psnr[-1] for s in scenes]
        m = float(np.mean(ps))
        if best is None or m > best[0]:
            best = (m, o)
    return best[1]


def mean_predicted_opacity(F, ctx, weights, scenes) -> float:
    """The prior's opacity averaged over every valid tile of the frames `scenes` (the constant a
    plain rule would need to match it)."""
    import torch
    vals = []
    for s in scenes:
        fr = frame_of(s)
        feat, valid = F.tile_features(ctx, torch.as_tensor(fr.rgb).cuda(), torch.as_tensor(fr.depth).cuda())
        y = F.prior_forward(ctx, feat, weights)
        ok = valid.cpu().numpy() >= 4
        vals.append(1.0 / (1.0 + np.exp(-y[:, 3].cpu().numpy().astype(np.float64)[ok])))
    return float(np.mean(np.concatenate(vals)))


def run_experiment(F, ctx, train_scenes, test_scenes, iters: int = 200, tiles_per_scene: int = 100,
                   train_steps: int = 2000, lr: float = 1e-3, margin_db: float = 0.1, opacity=None,
                   log=None, mode: int = 3, other_modes=(), constant_control: bool = False) -> dict:
    """Build the training set from the plain method's converged maps, train the prior on the GPU,
    and compare time and iterations to the plain method's final PSNR on held-out scenes. mode: how
    the prior seeds (fgs_seed_opts.use_prior: 1 shape and opacity, 2 shape, 3 opacity); the
    summary is that mode's against the plain rule at `opacity` (swept over 0.1 / 0.5 / 0.9 when
    None). other_modes: further modes, evaluated the same way ("modes"); constant_control: also
    the plain rule at the prior's mean predicted opacity against `mode` ("constant_control"). log
    (optional) receives one progress line per phase."""
    import time
    log = log or (lambda msg: None)
    t0 = time.perf_counter()
    if opacity is None:
        opacity = best_plain_opacity(F, ctx, list(train_scenes)[:5], iters)
        log(f"plain opacity {opacity} chosen")
    base = F.SeedOpts(opacity_logit=logit(opacity))
    X, Y = build_dataset(F, ctx, train_scenes, iters, tiles_per_scene, base)
    t_data = time.perf_counter() - t0
    log(f"training set of {X.shape[0]} tiles built in {t_data:.1f} s")
    w, losses = train(F, ctx, X, Y, train_steps, lr)
    t_train = time.perf_counter() - t0 - t_data
    log(f"prior trained in {t_train:.1f} s")

    def prior_opts(m):
        return F.SeedOpts(opacity_logit=logit(opacity), use_prior=m, prior=w)

    rows = evaluate(F, ctx, w, test_scenes, iters, margin_db, plain_opts=base, prior_opts=prior_opts(mode))
    summary = dict(mode=mode, opacity=opacity, train_rows=int(X.shape[0]), train_loss_first=float(losses[0]),
                   train_loss_last=float(losses[-1]), data_s=t_data, train_s=t_train, **summarize(rows))
    out = dict(summary=summary, rows=rows, weights=w, losses=losses, modes={})
    for m in other_modes:
        r = evaluate(F, ctx, w, test_scenes, iters, margin_db, plain_opts=base, prior_opts=prior_opts(m))
        out["modes"][m] = dict(summary=summarize(r), rows=r)
        log(f"mode {m} evaluated")
    if constant_control:
        c = mean_predicted_opacity(F, ctx, w, test_scenes)
        r = evaluate(F, ctx, w, test_scenes, iters, margin_db, plain_opts=F.SeedOpts(opacity_logit=logit(c)),
                     prior_opts=prior_opts(mode))
        out["constant_control"] = dict(opacity=c, summary=summarize(r), rows=r)
        log(f"constant-opacity control ({c:.4f}) evaluated")
    return out
