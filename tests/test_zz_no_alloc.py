"""GPU test of fgs_render_bwd_noalloc, the backward entry point that allocates nothing (its
gradient records live in a static per-GPU array): through the C ABI, against fgs_render_bwd on
the same forward state, on two calls in a row (the second with fewer gaussians and a smaller
image, so it reuses the array the first one left behind), at the gradient bar (1e-4 relative,
per tensor and elementwise from 1e-2 of each tensor's largest entry)."""
import numpy as np
import pytest

import synth
from gpu_helpers import assert_close_rel, dev, host, need_gpu

pytestmark = pytest.mark.gpu

GRAD_TOL, GRAD_FLOOR = 1e-4, 1e-2
ROWS = (("mean", slice(0, 3)), ("log_scale", slice(3, 6)), ("quat", slice(6, 10)), ("opacity", slice(10, 11)),
        ("rgb", slice(11, 14)))


def _both(F, ctx, p, cam, seed):
    n = p.shape[1]
    pd = dev(p)
    opts = F.RenderOpts()
    out = F.render(ctx, pd, n, cam, opts)
    P = cam.width * cam.height
    g = synth.rng(4200 + seed)
    gr, gd, ga = (dev(g.normal(size=s).astype(np.float32)) for s in ((3, P), P, P))
    ref = dev(np.zeros((14, n), np.float32))
    F.render_bwd(ctx, pd, n, cam, opts, out["state"], gr, gd, ga, ref)
    # the no-allocation entry point adds into grad as render_bwd does: start from a non-zero buffer
    base = synth.rng(4300 + seed).normal(size=(14, n)).astype(np.float32) * 1e-3
    got = dev(base)
    F.render_bwd_noalloc(ctx, pd, n, cam, opts, out["state"], gr, gd, ga, got)
    ctx.check()
    r, gg = host(ref), host(got).astype(np.float64) - base
    assert np.abs(r).max() > 0
    for name, rows in ROWS:
        assert_close_rel(gg[rows], r[rows], GRAD_TOL, None, f"d{name} ({n} gaussians)", floor=GRAD_FLOOR)


def test_noalloc_backward_matches_render_bwd_twice():
    need_gpu()
    import paper_2503_01109_amd as F
    ctx = F.Context()
    try:
        big_cam = synth.centred_camera(320, 240, 300.0)
        big = synth.frustum_scene(11, 40_000, big_cam, 1.0, 5.0)
        print(f"noalloc call 1: {big.shape[1]} gaussians, 320x240", flush=True)
        _both(F, ctx, big, big_cam, 0)
        small = synth.scene_small(3)
        print(f"noalloc call 2: {small.shape[1]} gaussians, 64x48", flush=True)
        _both(F, ctx, small, synth.camera_small(), 1)
    finally:
        ctx.close()

