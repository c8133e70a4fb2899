"""GPU parity: render_fwd / render_bwd through the C ABI against the FP64 oracle.

Tolerances: 1e-5 relative for rendered planes (gpu_helpers.assert_close_rel); gradients 1e-4
relative per element plus the binary32 rounding allowance on the absolute mass of the sum that
defines the element, and 1e-4 of the largest entry per tensor (gpu_helpers.assert_grad_close).
Pixels the oracle flags as ambiguous (a cutoff decision within 1e-5 relative of its threshold) are
excluded from the forward comparison and get a zero upstream gradient in the backward comparison.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import assert_close_rel, dev, host, need_gpu, oracle_opts, assert_grad_close

pytestmark = pytest.mark.gpu

FWD_TOL, GRAD_TOL = 1e-5, 1e-4


@pytest.fixture(scope="module")
def fgs():
    need_gpu()
    import paper_2503_01109_amd as F
    return F


@pytest.fixture(scope="module")
def ctx(fgs):
    c = fgs.Context()
    yield c
    c.close()



def params_dev(p, cap=None):
    n = p.shape[1]
    cap = cap or n
    block = np.zeros((14, cap), np.float32)
    block[:, :n] = p
    return dev(block)


def check_forward(fgs, ctx, p, cam, opts, max_amb_frac=0.0):
    pd = params_dev(p)
    out = fgs.render(ctx, pd, p.shape[1], cam, opts)
    ref = oracle.render_fwd(p.astype(np.float64), cam, oracle_opts(opts), mode=0, amb_rel=1e-5)
    ok = ~ref["amb"]
    assert ref["n_amb"] <= max_amb_frac * cam.width * cam.height, f"{ref['n_amb']} ambiguous pixels"
    assert_close_rel(host(out["rgb"]), ref["rgb"], FWD_TOL, ok, "rgb")
    assert_close_rel(host(out["depth"]), ref["depth"], FWD_TOL, ok, "depth")
    assert_close_rel(host(out["alpha"]), ref["alpha"], FWD_TOL, ok, "alpha")
    assert_close_rel(host(out["T_final"]), ref["T_final"], FWD_TOL, ok, "T_final")
    np.testing.assert_array_equal(host(out["n_contrib"])[ok], ref["n_contrib"][ok])
    return out, ref


def check_backward(fgs, ctx, p, cam, opts, out, ref, seed=0, with_alpha=True):
    P = cam.width * cam.height
    g = synth.rng(1000 + seed)
    gr = g.normal(size=(3, P)).astype(np.float32)
    gd = g.normal(size=P).astype(np.float32)
    ga = g.normal(size=P).astype(np.float32) if with_alpha else None
    amb = ref["amb"].ravel()
    gr[:, amb] = 0
    gd[amb] = 0
    if ga is not None:
        ga[amb] = 0
    n = p.shape[1]
    pd = params_dev(p)
    grad = dev(np.zeros((14, n), np.float32))
    fgs.render_bwd(ctx, pd, n, cam, opts, out["state"], dev(gr), dev(gd), None if ga is None else dev(ga), grad)
    ctx.check()
    gref, _, mass = oracle.render_bwd(p.astype(np.float64), cam, gr, gd, ga, oracle_opts(opts), mode=0, mass=True)
    gg = host(grad)
    assert_grad_close(gg, gref, mass, "backward", tol=GRAD_TOL)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_small_scene_forward_backward(fgs, ctx, seed):
    """2,000 gaussians, 64x48, fx = fy = 60: forward planes and all 14 parameter gradients."""
    p = synth.scene_small(seed)
    cam = synth.camera_small()
    opts = fgs.RenderOpts()
    out, ref = check_forward(fgs, ctx, p, cam, opts, max_amb_frac=0.01)
    check_backward(fgs, ctx, p, cam, opts, out, ref, seed)


def test_full_size_workload_sampled(fgs, ctx):
    """The 300k-gaussian 1200x680 workload (20% of the gaussians in 8 blobs), 16x16 tiles as the
    benchmark runs it: the forward planes at 4,000 sampled pixels against the oracle rendering those
    pixels one by one, and all 14 parameter gradients of an upstream gradient that is non-zero at
    the sampled pixels only, against the oracle's backward over the same pixels (elementwise from
    the rounding allowance on each sum's absolute mass)."""
    cam = synth.camera_replica()
    p = synth.scene_replica(0)
    n = p.shape[1]
    p64 = p.astype(np.float64)
    opts = fgs.RenderOpts()
    pd = params_dev(p)
    out = fgs.render(ctx, pd, n, cam, opts)
    W, H = cam.width, cam.height
    P = W * H
    g = synth.rng(77)
    pix = np.sort(g.choice(P, 4000, replace=False))
    ref = oracle.render_fwd(p64, cam, oracle_opts(opts), mode=0, pix=pix, amb_rel=1e-5)
    ok = ~ref["amb"]
    assert ref["n_amb"] <= 0.01 * pix.size, f"{ref['n_amb']} ambiguous sampled pixels"
    rgb = host(out["rgb"]).reshape(3, P)[:, pix]
    assert_close_rel(rgb, ref["rgb"], FWD_TOL, ok, "rgb")
    for k in ("depth", "alpha", "T_final"):
        assert_close_rel(host(out[k]).ravel()[pix], ref[k], FWD_TOL, ok, k)
    np.testing.assert_array_equal(host(out["n_contrib"]).ravel()[pix][ok], ref["n_contrib"][ok])
    keep = pix[ok]
    gr = np.zeros((3, P), np.float32)
    gd = np.zeros(P, np.float32)
    ga = np.zeros(P, np.float32)
    gr[:, keep] = g.normal(size=(3, keep.size))
    gd[keep] = g.normal(size=keep.size)
    ga[keep] = g.normal(size=keep.size)
    grad = dev(np.zeros((14, n), np.float32))
    fgs.render_bwd(ctx, pd, n, cam, opts, out["state"], dev(gr), dev(gd), dev(ga), grad)
    ctx.check()
    gref, _, mass = oracle.render_bwd(p64, cam, gr[:, keep], gd[keep], ga[keep], oracle_opts(opts), mode=0,
                                      pix=keep, mass=True)
    gg = host(grad)
    assert np.count_nonzero(gref[10]) > 1000  # the sample reaches many gaussians
    assert_grad_close(gg, gref, mass, "full size", tol=GRAD_TOL)


@pytest.mark.parametrize("tile", [(16, 16), (32, 8), (8, 32), (32, 16), (16, 32), (8, 8)])
def test_tile_shape_independence(fgs, ctx, tile):
    """P6: every rasterizer tile shape gives the oracle's image (ragged 70x50 frame)."""
    cam = synth.centred_camera(70, 50, 60.0)
    p = synth.frustum_scene(7, 1500, cam, 1.0, 5.0)
    opts = fgs.RenderOpts(tile_w=tile[0], tile_h=tile[1])
    out, ref = check_forward(fgs, ctx, p, cam, opts, max_amb_frac=0.01)
    check_backward(fgs, ctx, p, cam, opts, out, ref, seed=3)


def test_background_lowpass_and_pose(fgs, ctx):
    """Non-zero background, no low-pass filter, a rotated and translated camera."""
    import test_oracle_render as tor
    cam0 = synth.centred_camera(48, 40, 50.0)
    R = tor.rot_of(np.array([0.95, 0.1, -0.2, 0.15]))
    t = np.array([0.05, -0.02, 0.1])
    cam = synth.Camera(48, 40, 50.0, 52.0, 24.0, 20.0, R=R, t=t)
    p = synth.frustum_scene(11, 800, cam0, 1.0, 4.0).astype(np.float64)
    p[0:3] = R.T.astype(np.float32).astype(np.float64) @ (p[0:3] - t[:, None])
    p = p.astype(np.float32)
    opts = fgs.RenderOpts(lowpass=0.0, bg=(0.2, 0.4, 0.6), bg_depth=3.0)
    out, ref = check_forward(fgs, ctx, p, cam, opts, max_amb_frac=0.01)
    check_backward(fgs, ctx, p, cam, opts, out, ref, seed=5)


def test_termination_stack(fgs, ctx):
    """P3 on the GPU: 20 stacked alpha = 0.5 gaussians at the centre pixel blend exactly 13."""
    cam = synth.Camera(16, 16, 40.0, 40.0, 8.5, 8.5)
    n = 20
    p = np.zeros((14, n), np.float32)
    p[2] = 1.0 + 0.1 * np.arange(n)
    p[3:6] = np.log(0.05)
    p[6] = 1.0
    p[11:14] = synth.rng(0).uniform(size=(3, n))
    out = fgs.render(ctx, params_dev(p), n, cam, fgs.RenderOpts())
    assert host(out["n_contrib"])[8, 8] == 13
    assert host(out["T_final"])[8, 8] == np.float32(2.0 ** -13)


def test_many_super_tiles_and_huge_gaussians(fgs, ctx):
    """8x8 tiles on a 640x480 frame: 80x60 tiles in 20x15 = 300 super-tiles, more than one radix
    digit, so the super-tile order takes two passes. The scene mixes ordinary gaussians with a
    few that cover most of the frame (lists of every tile, many chunks per super-tile) and
    gaussians straddling the frame border. Forward at 3,000 sampled pixels and the full gradient
    against the oracle."""
    cam = synth.camera_tum()
    p = synth.frustum_scene(31, 3000, cam, 1.0, 6.0)
    p[3:6, :6] = np.log(0.8)  # six gaussians about a metre wide
    p[0, 6:20] = np.linspace(-3.0, 3.0, 14)  # a row across the frame border at x = 0 and x = W
    p[1, 6:20] = 0.0
    p[2, 6:20] = 2.0
    n = p.shape[1]
    opts = fgs.RenderOpts(tile_w=8, tile_h=8)
    pd = params_dev(p)
    out = fgs.render(ctx, pd, n, cam, opts)
    P = cam.width * cam.height
    g = synth.rng(78)
    pix = np.sort(g.choice(P, 3000, replace=False))
    ref = oracle.render_fwd(p.astype(np.float64), cam, oracle_opts(opts), mode=0, pix=pix, amb_rel=1e-5)
    ok = ~ref["amb"]
    assert ref["n_amb"] <= 0.01 * pix.size
    assert_close_rel(host(out["rgb"]).reshape(3, P)[:, pix], ref["rgb"], FWD_TOL, ok, "rgb")
    for k in ("depth", "alpha", "T_final"):
        assert_close_rel(host(out[k]).ravel()[pix], ref[k], FWD_TOL, ok, k)
    np.testing.assert_array_equal(host(out["n_contrib"]).ravel()[pix][ok], ref["n_contrib"][ok])
    keep = pix[ok]
    gr = np.zeros((3, P), np.float32)
    gd = np.zeros(P, np.float32)
    gr[:, keep] = g.normal(size=(3, keep.size))
    gd[keep] = g.normal(size=keep.size)
    grad = dev(np.zeros((14, n), np.float32))
    fgs.render_bwd(ctx, pd, n, cam, opts, out["state"], dev(gr), dev(gd), None, grad)
    ctx.check()
    gref, _, mass = oracle.render_bwd(p.astype(np.float64), cam, gr[:, keep], gd[keep], None, oracle_opts(opts),
                                      mode=0, pix=keep, mass=True)
    gg = host(grad)
    assert_grad_close(gg, gref, mass, "sampled", tol=GRAD_TOL)


def test_empty_and_culled(fgs, ctx):
    """n = 0 and an all-culled scene render the background."""
    cam = synth.camera_small()
    opts = fgs.RenderOpts(bg=(0.1, 0.2, 0.3), bg_depth=2.0)
    for n in (0, 5):
        p = np.zeros((14, max(n, 1)), np.float32)
        p[2] = -1.0  # behind the camera
        p[6] = 1.0
        out = fgs.render(ctx, params_dev(p), n, cam, opts)
        rgb = host(out["rgb"])
        for c in range(3):
            assert np.all(rgb[c] == np.float32(opts.bg[c]))
        assert np.all(host(out["depth"]) == 2.0)
        assert np.all(host(out["T_final"]) == 1.0)
        assert np.all(host(out["n_contrib"]) == 0)


def test_many_gaussians_take_the_two_level_scan(fgs, ctx):
    """4.5M gaussians, all but 2,000 behind the camera: the scan of the covered super-tiles then has
    more block sums than one apply workgroup adds up itself (a separate pass scans them first),
    and the result must equal the render of the 2,000 alone, bit for bit (their order by depth,
    then by index, does not change)."""
    small = synth.scene_small(5)
    cam = synth.camera_small()
    n = 4_500_000
    big = np.zeros((14, n), np.float32)
    big[2] = -1.0  # behind the camera
    big[6] = 1.0
    idx = np.sort(synth.rng(11).choice(n, small.shape[1], replace=False))
    big[:, idx] = small
    opts = fgs.RenderOpts()
    a = fgs.render(ctx, params_dev(small), small.shape[1], cam, opts)
    b = fgs.render(ctx, dev(big), n, cam, opts, max_pairs=1 << 20)
    for k in ("rgb", "depth", "alpha", "T_final", "n_contrib"):
        assert np.array_equal(host(a[k]), host(b[k])), k
    del b, big


@pytest.mark.parametrize("n", [8_193, 12_289, 16_384, 16_385, 40_000])
def test_super_tile_list_longer_than_lds(fgs, ctx, n):
    """A 64x48 frame is one super-tile, whose list holds every gaussian (each covers at least the
    pixel nearest its centre). A list of two chunks (up to 16,384 entries) is merged in LDS by four
    workgroups, a quarter each (8,193 and 12,289 leave the last quarters short or empty); 16,385 and
    40,000 take the path through global memory. Forward against the oracle, and the gradient in the
    12,289 and 16,385 cases."""
    cam = synth.camera_small()
    p = synth.frustum_scene(40 + n % 7, n, cam, 1.0, 5.0)
    opts = fgs.RenderOpts()
    out, ref = check_forward(fgs, ctx, p, cam, opts, max_amb_frac=0.02)
    assert ctx.stats()["visible"] == n
    if n in (12_289, 16_385):
        check_backward(fgs, ctx, p, cam, opts, out, ref, seed=3)


def test_invariant_weights_sum_to_one(fgs, ctx):
    """P4 on the GPU: alpha + T_final = 1 within FP32 rounding, at every pixel."""
    p = synth.scene_small(4)
    cam = synth.camera_small()
    out = fgs.render(ctx, params_dev(p), p.shape[1], cam, fgs.RenderOpts())
    s = host(out["alpha"]).astype(np.float64) + host(out["T_final"])
    assert np.abs(s - 1).max() < 1e-6


def test_capacity_overflow_is_reported(fgs, ctx):
    p = synth.scene_small(0)
    cam = synth.camera_small()
    opts = fgs.RenderOpts()
    pd = params_dev(p)
    n = p.shape[1]
    import torch
    nb = fgs.state_bytes(n, cam.width, cam.height, 16, opts)
    state = torch.empty(nb, dtype=torch.uint8, device="cuda")
    rgb = torch.empty((3, cam.height, cam.width), device="cuda")
    depth = torch.empty((cam.height, cam.width), device="cuda")
    fgs.render_fwd(ctx, pd, n, cam, opts, rgb, depth, state)
    with pytest.raises(fgs.FgsError) as e:
        ctx.check()
    assert e.value.status == fgs.ERR_CAPACITY
    K = oracle.count_duplicates(p.astype(np.float64), cam, 16, 16)
    need = fgs.ctx_required_pairs(e.value)
    assert K <= need <= K + K // 50 + 16  # the HIP path pads its tile boxes by 1e-5 relative + 1e-3 px
    ctx.check()  # the condition is cleared once reported
    # one pair short: the super-tile pairs still fit, the tile lists do not
    nb = fgs.state_bytes(n, cam.width, cam.height, need - 1, opts)
    state = torch.empty(nb, dtype=torch.uint8, device="cuda")
    fgs.render_fwd(ctx, pd, n, cam, opts, rgb, depth, state)
    with pytest.raises(fgs.FgsError) as e:
        ctx.check()
    assert e.value.status == fgs.ERR_CAPACITY and fgs.ctx_required_pairs(e.value) == need
    # exactly enough
    nb = fgs.state_bytes(n, cam.width, cam.height, need, opts)
    state = torch.empty(nb, dtype=torch.uint8, device="cuda")
    fgs.render_fwd(ctx, pd, n, cam, opts, rgb, depth, state)
    ctx.check()


def test_deterministic_forward(fgs, ctx):
    p = synth.scene_small(6)
    cam = synth.camera_small()
    pd = params_dev(p)
    a = fgs.render(ctx, pd, p.shape[1], cam, fgs.RenderOpts())
    b = fgs.render(ctx, pd, p.shape[1], cam, fgs.RenderOpts())
    for k in ("rgb", "depth", "alpha", "T_final", "n_contrib"):
        assert np.array_equal(host(a[k]), host(b[k]))


def test_profiling_levels_and_work_counters(fgs, ctx):
    """Levels 1 and 2 time without counting; level 3 counts exactly: the pairs blended are the sum
    of the per-pixel contributor counts, and profiling changes no output bit."""
    p = synth.scene_small(8)
    cam = synth.camera_small()
    pd = params_dev(p)
    plain = fgs.render(ctx, pd, p.shape[1], cam, fgs.RenderOpts())
    ctx.profile(1)
    a = fgs.render(ctx, pd, p.shape[1], cam, fgs.RenderOpts())
    rep1 = ctx.profile_report()
    ctx.profile(2)
    c2 = fgs.render(ctx, pd, p.shape[1], cam, fgs.RenderOpts())
    rep_2 = ctx.profile_report()
    ctx.profile(3)
    b = fgs.render(ctx, pd, p.shape[1], cam, fgs.RenderOpts())
    rep2 = ctx.profile_report()
    ctx.profile(0)
    assert rep1["raster_fwd"][1] == 1 and rep1["counts"]["forwards"] == 0
    assert rep1["counts"]["pairs_blended"] == 0 and rep1["counts"]["pairs_examined"] == 0
    assert rep_2["project"][1] == 1 and rep_2["raster_fwd"][1] == 1 and rep_2["counts"]["forwards"] == 0
    assert rep2["counts"]["forwards"] == 1
    assert rep2["counts"]["pairs_blended"] == int(host(b["n_contrib"]).sum()) > 0
    assert rep2["counts"]["pairs_examined"] >= rep2["counts"]["pairs_blended"]
    for k in ("rgb", "depth", "alpha", "T_final", "n_contrib"):
        for r in (a, b, c2):
            assert np.array_equal(host(r[k]), host(plain[k])), k


def test_backward_finds_the_forward_blends(fgs):
    """At profiling level 3 the mapping step's backward counts the (pixel, entry) pairs it finds
    blended by replaying the forward's decisions in reverse: exactly the forward's count, on a
    clamp-heavy scene of 3,000 gaussians over several tiles and a ragged edge."""
    import torch
    cam = synth.Camera(72, 52, 70.0, 70.0, 36.0, 26.0)
    p = synth.frustum_scene(21, 3000, cam, 1.0, 5.0)
    p[10] = np.abs(p[10]) + 2.0  # opacities near 1: many clamped alphas
    pd = params_dev(p)
    n = p.shape[1]
    ctx = fgs.Context()
    tgt = fgs.render(ctx, params_dev(synth.frustum_scene(22, 3000, cam, 1.0, 5.0)), n, cam, fgs.RenderOpts(), aux=False)
    adam = fgs.Adam.like(pd)
    ctx.profile(3)
    for _ in range(2):
        fgs.map_step(ctx, pd, n, adam, [cam], [(tgt["rgb"], tgt["depth"])], fgs.RenderOpts())
    ctx.check()
    c = ctx.profile_report()["counts"]
    ctx.profile(0)
    torch.cuda.synchronize()
    assert c["forwards"] == 2 and c["backwards"] == 2
    assert c["bwd_pairs_blended"] == c["pairs_blended"] > 0
    assert c["bwd_wave_takes"] <= c["bwd_wave_evals"] and c["bwd_wave_few"] <= c["bwd_wave_takes"]
    assert 64 * c["bwd_wave_takes"] >= c["bwd_pairs_blended"]


def test_work_counts_match_oracle(fgs):
    """The forward's work counters at profiling level 3 against the oracle's on a scene with no
    ambiguous pixel, 16x16 tiles: E_f (pairs examined within the cutoff before each pixel stops),
    E_c (pairs blended) and K_c ((tile, gaussian) entries some pixel blended) exactly; L_f and L_b
    (list entries consumed before each tile terminates, forward and backward) within 0.5% plus two
    per tile at most (the HIP tile boxes are padded by 1e-3 px so that FP32 cannot reach outside them,
    which can put an extra boundary entry in a list)."""
    from test_gpu_mapstep import zero_ambiguity_scene
    p, cam, _ = zero_ambiguity_scene(n=2000)
    n = p.shape[1]
    c = fgs.Context()
    c.profile(3)
    fgs.render(c, params_dev(p), n, cam, fgs.RenderOpts(), aux=False)
    rep = c.profile_report()
    c.profile(0)
    cnt = rep["counts"]
    assert cnt["forwards"] == 1
    ref = oracle.render_fwd(p.astype(np.float64), cam, oracle_opts(), amb_rel=1e-5)
    assert ref["n_amb"] == 0
    tc = oracle.tile_counts(p.astype(np.float64), cam, oracle_opts())
    assert cnt["pairs_examined"] == ref["E_f"]
    assert cnt["pairs_blended"] == ref["E_c"]
    assert cnt["K_c"] == tc["K_c"]
    tiles = ((cam.width + 15) // 16) * ((cam.height + 15) // 16)
    for k in ("L_f", "L_b"):
        assert abs(cnt[k] - tc[k]) <= 0.005 * tc[k] + 2 * tiles, (k, cnt[k], tc[k])
    assert tc["K_c"] <= tc["L_b"] <= tc["L_f"] <= tc["K"]
    c.close()
