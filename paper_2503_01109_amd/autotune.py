"""Tile- and grid-shape tuning for the keyframe window.

The rasterizer's work per tile is its list of (tile, gaussian) pairs, and the best tile shape
depends on the resolution and on how elongated the projected footprints are: a 32x8 or 8x32 tile
over a 256-thread workgroup trades fewer pairs per pixel row against more tiles per gaussian. The
persistent launch's grid (workgroups per compute unit) trades occupancy against the tail of the
queue. Both are picked by timing the real window step on the real scene:

1. per resolution, each tile shape is timed on a window holding only that resolution's views;
2. with the winning shapes, each grid size is timed on the whole window;
3. the chosen configuration is checked against the default one (16x16 tiles, one workgroup per
   (view, tile) item): the same per-view losses, and the same summed gradient per parameter row in
   relative L2 error (FP32 atomics accumulate in a different order every run). This is a guard
   against gross faults only; the library's parity with the method's definition, for every tile
   shape and grid kind this tuner can pick, is established by its tests against the FP64 oracle
   (which the library itself never loads).

Results are cached in a JSON file keyed by device name, resolution and gaussian count (rounded
to a power of two), so a later run picks them up without timing.
"""
from __future__ import annotations

import json
import os
import time

TILE_SHAPES = ((16, 16), (32, 8), (8, 32))
BLOCKS_PER_CU = (0, 2, 4, 8)  # 0: one workgroup per (view, tile) item
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "fgs_autotune.json")


def _key(device: str, W: int, H: int, n: int) -> str:
    b = 1
    while b < max(n, 1):
        b <<= 1
    return f"{device}|{W}x{H}|n<={b}"


def _time_window(F, ctx, cams, tiles, bpc, params, n, targets, opts, steps):
    import torch
    win = F.Window(ctx, cams, tiles, bpc)
    adam = F.Adam.like(params, lr=(0.0, 0.0, 0.0, 0.0, 0.0))  # the scene stays fixed while timing
    try:
        win.step(params, n, adam, targets, opts, graph=True)  # sizes the states, captures the graph
        win.step(params, n, adam, targets, opts, graph=True)
        ctx.check()
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            win.step(params, n, adam, targets, opts, graph=True)
        e1.record(stream)
        torch.cuda.synchronize()
        ctx.check()
        return e0.elapsed_time(e1) / steps
    finally:
        win.close()


def _window_result(F, ctx, cams, tiles, bpc, params, n, targets, opts):
    import torch
    win = F.Window(ctx, cams, tiles, bpc)
    adam = F.Adam.like(params, lr=(0.0, 0.0, 0.0, 0.0, 0.0))
    grad = torch.zeros_like(params)
    loss = torch.zeros(len(cams), device=params.device)
    try:
        win.step(params, n, adam, targets, opts, loss=loss, grad_out=grad, graph=False)
        ctx.check()
    finally:
        win.close()
    return loss, grad


# Parameter rows of the packed layout: mean 0-2, log-scale 3-5, quaternion 6-9 (geometric, whose
# gradients are sums of large terms of both signs), logit 10 and rgb 11-13 (appearance).
GEOMETRIC_ROWS = slice(0, 10)
APPEARANCE_ROWS = slice(10, 14)


def check_against_default(F, ctx, cams, tiles, bpc, params, n, targets, opts, tol=1e-5, app_l2_tol=1e-5,
                          app_max_tol=1e-4, geo_l2_tol=1e-2, geo_max_tol=5e-2):
    """Raise AssertionError unless the configuration reproduces the default one.

    The per-pixel blend does not depend on the tile shape, so the per-view losses must agree to
    tol relative. Gradients are sums over pixels in an order that the tile shape and the FP32
    atomics change: the appearance rows (opacity, colour) are well conditioned and are held to
    app_l2_tol relative L2 error and app_max_tol of the row's largest entry; the geometric rows
    cancel heavily: at 500k gaussians, two runs of one configuration differ by up to ~6e-4
    relative L2 on a row, and two tile shapes (which also regroup the per-tile sums) by up to
    2.4e-3 (measured). They are held to geo_l2_tol and geo_max_tol, bounds that any real fault (a
    missed pair, a wrong pixel offset) exceeds by orders of magnitude."""
    l0, g0 = _window_result(F, ctx, cams, None, 0, params, n, targets, opts)
    l1, g1 = _window_result(F, ctx, cams, tiles, bpc, params, n, targets, opts)
    dl = (l1 - l0).abs() / l0.abs().clamp_min(1e-30)
    if float(dl.max()) > tol:
        raise AssertionError(f"autotuned window: loss differs from the default by {float(dl.max()):.2e}")
    g0, g1 = g0.double(), g1.double()
    l2 = (g1 - g0).norm(dim=1) / g0.norm(dim=1).clamp_min(1e-300)
    worst = (g1 - g0).abs().amax(dim=1) / g0.abs().amax(dim=1).clamp_min(1e-300)
    bad = bool((l2[APPEARANCE_ROWS] > app_l2_tol).any()) or bool((worst[APPEARANCE_ROWS] > app_max_tol).any())
    bad = bad or bool((l2[GEOMETRIC_ROWS] > geo_l2_tol).any()) or bool((worst[GEOMETRIC_ROWS] > geo_max_tol).any())
    if bad:
        raise AssertionError(f"autotuned window: gradient rows differ from the default: relative L2 {l2.tolist()}, "
                             f"max error / row max {worst.tolist()}")


def tune_window(F, ctx, cams, params, n: int, targets, opts=None, steps: int = 5, cache: str | None = DEFAULT_CACHE,
                verify: bool = True, device: str | None = None) -> dict:
    """Pick a tile shape per resolution and a grid size for a window over cams.

    Returns {"tiles": [(tw, th) per view], "blocks_per_cu": b, "ms": {...timings...},
    "from_cache": bool}."""
    opts = opts or F.RenderOpts()
    if device is None:
        import torch
        device = torch.cuda.get_device_name(params.device)
    res = sorted({(int(c.width), int(c.height)) for c in cams})
    db = {}
    if cache and os.path.exists(cache):
        try:
            with open(cache) as f:
                db = json.load(f)
        except (OSError, ValueError):
            db = {}
    wkey = _key(device, 0, 0, n) + "|" + ",".join(f"{w}x{h}" for w, h in res) + f"|views={len(cams)}"
    hit = all(_key(device, w, h, n) in db for w, h in res) and wkey in db
    timings = {}
    if hit:
        shape = {r: tuple(db[_key(device, *r, n)]["tile"]) for r in res}
        bpc = int(db[wkey]["blocks_per_cu"])
    else:
        t0 = time.perf_counter()
        shape = {}
        for r in res:
            idx = [k for k, c in enumerate(cams) if (int(c.width), int(c.height)) == r]
            sub_c = [cams[k] for k in idx]
            sub_t = [targets[k] for k in idx]
            best = None
            for ts in TILE_SHAPES:
                ms = _time_window(F, ctx, sub_c, [ts] * len(sub_c), 0, params, n, sub_t, opts, steps)
                timings[f"{r[0]}x{r[1]} tile {ts[0]}x{ts[1]}"] = ms
                if best is None or ms < best[0]:
                    best = (ms, ts)
            shape[r] = best[1]
        tiles = [shape[(int(c.width), int(c.height))] for c in cams]
        best = None
        for b in BLOCKS_PER_CU:
            ms = _time_window(F, ctx, cams, tiles, b, params, n, targets, opts, steps)
            timings[f"window blocks_per_cu {b}"] = ms
            if best is None or ms < best[0]:
                best = (ms, b)
        bpc = best[1]
        timings["tuning_s"] = time.perf_counter() - t0
    tiles = [shape[(int(c.width), int(c.height))] for c in cams]
    if verify:
        check_against_default(F, ctx, cams, tiles, bpc, params, n, targets, opts)
    if not hit and cache:
        for r in res:
            db[_key(device, *r, n)] = {"tile": list(shape[r])}
        db[wkey] = {"blocks_per_cu": bpc}
        try:
            os.makedirs(os.path.dirname(cache), exist_ok=True)
            tmp = cache + f".{os.getpid()}"
            with open(tmp, "w") as f:
                json.dump(db, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        except OSError:
            pass
    return {"tiles": tiles, "blocks_per_cu": bpc, "ms": timings, "from_cache": hit}
