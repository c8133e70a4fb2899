"""GPU tests of the keyframe window (fgs_window_*): several views of different sizes and tile
shapes mapped together by one persistent forward launch and one persistent backward launch.

The window must compute what the plain mapping step computes over the same views (whose parity
with the oracle is tested elsewhere): the per-view losses, the gradient summed over the views, and
the Adam update, here with the Adam step counter kept on the device. A graph replay must give what
an eager step gives. A pair overflow during a replay is reported by the next call, after which the
window has grown and steps are correct again.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import assert_close_rel, dev, host, need_gpu, oracle_opts, assert_grad_close, near_plane_splats

pytestmark = pytest.mark.gpu
LR = (1e-3, 5e-3, 1e-3, 5e-2, 2.5e-3)
GROUP = np.array([0, 0, 0, 1, 1, 1, 2, 2, 2, 2, 3, 4, 4, 4])


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


def small_views():
    cam0 = synth.camera_small()
    cams = [cam0, synth.centred_camera(70, 50, 55.0),
            synth.Camera(48, 40, 50.0, 50.0, 24.0, 20.0, t=[0.1, -0.05, 0.2]),
            synth.centred_camera(96, 64, 80.0)]
    tiles = [(16, 16), (32, 8), (8, 32), (16, 16)]
    return cams, tiles


def random_targets(cams, seed):
    out = []
    for k, c in enumerate(cams):
        g = synth.rng(seed + k)
        out.append((dev(g.uniform(size=(3, c.height, c.width))), dev(g.uniform(1, 4, (c.height, c.width)))))
    return out


def per_view_losses(fgs, ctx, pd, n, cams, targets, lopts):
    import torch
    ls = []
    for c, (tr, tdp) in zip(cams, targets):
        out = fgs.render(ctx, pd, n, c, fgs.RenderOpts(), aux=False)
        dr, dd = torch.empty_like(tr), torch.empty_like(tdp)
        loss = torch.zeros(1, device="cuda")
        fgs.loss_l1(ctx, out["rgb"], out["depth"], tr, tdp, lopts, dr, dd, loss)
        ls.append(float(loss))
    return np.array(ls)


@pytest.mark.parametrize("graph", [False, True])
def test_window_equals_plain_mapping_step(fgs, ctx, graph):
    """Losses per view, the summed gradient and the Adam update equal those of fgs_map_step over the
    same views (tiles 16x16, 32x8, 8x32 mixed in one window)."""
    import torch
    cams, tiles = small_views()
    p = synth.frustum_scene(3, 1500, cams[0], 1.0, 5.0)
    n = p.shape[1]
    targets = random_targets(cams, 50)
    lopts = fgs.LossOpts(1.0, 0.1)
    ref_loss = per_view_losses(fgs, ctx, dev(p), n, cams, targets, lopts)

    pa = dev(p)
    adam_a = fgs.Adam.like(pa, lr=LR)
    ga = torch.zeros_like(pa)
    fgs.map_step(ctx, pa, n, adam_a, cams, targets, fgs.RenderOpts(), lopts, grad_out=ga)

    pb = dev(p)
    adam_b = fgs.Adam.like(pb, lr=LR)
    gb = torch.full_like(pb, 3.0)  # overwritten
    loss = torch.zeros(len(cams), device="cuda")
    psnr = torch.zeros(len(cams), device="cuda")
    win = fgs.Window(ctx, cams, tiles)
    win.step(pb, n, adam_b, targets, fgs.RenderOpts(), lopts, loss, psnr, grad_out=gb, graph=graph)
    ctx.check()
    torch.cuda.synchronize()
    assert adam_b.step == 1
    np.testing.assert_allclose(host(loss), ref_loss, rtol=1e-5)
    assert np.all(np.isfinite(host(psnr)))
    assert_close_rel(host(gb), host(ga), 1e-5, what="window gradient", floor=1e-2)
    # first Adam step: -lr g / (|g| + eps), compared where |g| is well above the FP32 error
    g = host(ga).astype(np.float64)
    big = np.abs(g) >= 1e-2 * np.abs(g).max(axis=1, keepdims=True)
    np.testing.assert_allclose(host(pb)[big], host(pa)[big], rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(host(adam_b.m)[big], host(adam_a.m)[big], rtol=1e-4)
    win.close()


def test_window_first_view_matches_oracle(fgs, ctx):
    """A one-view window against the FP64 oracle directly (zero-ambiguity scene of the
    mapping-step test): loss, gradient."""
    import torch
    from test_gpu_mapstep import zero_ambiguity_scene
    p, cam, seed = zero_ambiguity_scene()
    n = p.shape[1]
    ref = oracle.render_fwd(p.astype(np.float64), cam, oracle_opts(), amb_rel=0)
    tgt = oracle.render_fwd(synth.frustum_scene(seed + 1000, n, cam, 1.0, 5.0).astype(np.float64), cam, amb_rel=0)
    trgb, td = tgt["rgb"].astype(np.float32), tgt["depth"].astype(np.float32)
    trgb[np.abs(ref["rgb"] - trgb) < 1e-3] += 0.01
    td[np.abs(ref["depth"] - td) < 1e-3] += 0.01
    L, ps, gr, gd = oracle.loss_l1(ref["rgb"], ref["depth"], trgb, td, 1.0, 0.1)
    gref, _, mass = oracle.render_bwd(p.astype(np.float64), cam, gr, gd, None, oracle_opts(), mass=True)
    pd = dev(p)
    adam = fgs.Adam.like(pd, lr=(0, 0, 0, 0, 0))
    grad = torch.zeros_like(pd)
    loss, psnr = torch.zeros(1, device="cuda"), torch.zeros(1, device="cuda")
    win = fgs.Window(ctx, [cam])
    win.step(pd, n, adam, [(dev(trgb), dev(td))], fgs.RenderOpts(), fgs.LossOpts(1.0, 0.1), loss, psnr, grad)
    ctx.check()
    assert abs(float(loss) - L) <= 1e-5 * L
    assert abs(float(psnr) - ps) <= 1e-5 * ps
    gg = host(grad)
    assert_grad_close(gg, gref, mass, "one-view window")
    np.testing.assert_array_equal(host(pd), p)  # lr = 0
    win.close()


@pytest.mark.parametrize("blocks_per_cu,graph", [(0, False), (0, True), (2, False), (2, True)])
def test_uneven_window_matches_oracle(fgs, ctx, blocks_per_cu, graph):
    """Four views of different sizes and poses with 16x16, 32x8, 8x32 and 16x16 tiles, one
    workgroup per item or a persistent grid, eager or graph-replayed: each view's loss against the
    oracle's forward and L1 terms of Eq. 16, and the gradient summed over the views and the first
    Adam update against the oracle's per-view backward (ambiguous pixels masked out of the targets
    on both sides)."""
    import torch
    from oracle_ref import mapping_reference
    cams, tiles = small_views()
    p = synth.frustum_scene(14, 1500, cams[0], 1.0, 5.0)
    n = p.shape[1]
    targets = [(host(a), host(b)) for a, b in random_targets(cams, 150)]
    R = mapping_reference(p, cams, targets)
    win = fgs.Window(ctx, cams, tiles, blocks_per_cu)
    pd = dev(p)
    loss, psnr = torch.zeros(len(cams), device="cuda"), torch.zeros(len(cams), device="cuda")
    win.step(pd, n, fgs.Adam.like(pd, lr=(0, 0, 0, 0, 0)), [(dev(a), dev(b)) for a, b in R["targets"]],
             fgs.RenderOpts(), fgs.LossOpts(1.0, 0.1), loss, psnr, graph=graph)
    ctx.check()
    np.testing.assert_allclose(host(loss), R["loss"], rtol=1e-5)
    np.testing.assert_allclose(host(psnr), R["psnr"], rtol=1e-5)
    adam = fgs.Adam.like(pd, lr=LR)
    grad = torch.zeros_like(pd)
    win.step(pd, n, adam, [(dev(a), dev(b)) for a, b in R["masked"]], fgs.RenderOpts(), fgs.LossOpts(1.0, 0.1),
             grad_out=grad, graph=graph)
    ctx.check()
    gg, gref = host(grad), R["grad"]
    assert_grad_close(gg, gref, R["mass"], "uneven window")
    lr = np.array(LR)[GROUP][:, None]
    expect = p - lr * gref / (np.abs(gref) + 1e-15)
    big = np.abs(gref) >= 1e-2 * np.abs(gref).max(axis=1, keepdims=True)
    np.testing.assert_allclose(host(pd)[big], expect[big], rtol=1e-6, atol=1e-6)
    win.close()


def test_full_window_matches_oracle(fgs):
    """The 8-view window at its real shapes (500k gaussians in a 6x6x4 m box, four 640x480 views
    with 32x8 tiles and four 1200x680 views with 16x16 tiles, graph replay) against the oracle's
    per-view forward, L1 terms of Eq. 16 and backward, summed over the views (random targets;
    ambiguous pixels masked out on both sides). Losses at 1e-5; gradients at the parity bar
    (assert_grad_close). The cameras stand inside the scene, so some 8% of the gaussians lie within
    25% of the near plane in some view; their projections are huge (radius up to ~27,000 px), very
    elongated and far off-centre, and the binary32 rounding of those projections, not the sums,
    decides their gradients to about 1e-3 (measured: up to 0.72% of the absolute mass): they are
    held to the near-plane allowance."""
    import torch
    from oracle_ref import mapping_reference
    c = fgs.Context()
    cams = synth.window_cameras(0)
    p = synth.scene_window(0)
    n = p.shape[1]
    targets = []
    for k, cam in enumerate(cams):
        g = synth.rng(900 + k)
        targets.append((g.uniform(size=(3, cam.height, cam.width)).astype(np.float32),
                        g.uniform(1, 4, (cam.height, cam.width)).astype(np.float32)))
    R = mapping_reference(p, cams, targets, log=lambda s: print(s, flush=True))
    near = near_plane_splats(p, cams)
    win = fgs.Window(c, cams, [(32, 8)] * 4 + [(16, 16)] * 4, 0)
    pd = dev(p)
    loss = torch.zeros(len(cams), device="cuda")
    win.step(pd, n, fgs.Adam.like(pd, lr=(0, 0, 0, 0, 0)), [(dev(a), dev(b)) for a, b in R["targets"]],
             fgs.RenderOpts(), fgs.LossOpts(1.0, 0.1), loss, graph=True)
    grad = torch.zeros_like(pd)
    win.step(pd, n, fgs.Adam.like(pd, lr=(0, 0, 0, 0, 0)), [(dev(a), dev(b)) for a, b in R["masked"]],
             fgs.RenderOpts(), fgs.LossOpts(1.0, 0.1), grad_out=grad, graph=True)
    c.check()
    np.testing.assert_allclose(host(loss), R["loss"], rtol=1e-5)
    gg, gref = host(grad).astype(np.float64), R["grad"]
    print(f"{int(near.sum())} near-plane splats of {n}", flush=True)
    assert_grad_close(gg, gref, R["mass"], "8-view window", near=near)
    win.close()
    c.close()


def test_graph_replays_match_eager_steps(fgs, ctx):
    """Five replays of one captured step, the target planes rewritten in place between them and
    other device work interleaved, each equal to an eager step on the same inputs."""
    import torch
    cams, tiles = small_views()
    p = synth.frustum_scene(4, 1500, cams[0], 1.0, 5.0)
    n = p.shape[1]
    pd = dev(p)
    targets = random_targets(cams, 70)
    zero = fgs.Adam.like(pd, lr=(0, 0, 0, 0, 0))
    we = fgs.Window(ctx, cams, tiles)
    wg = fgs.Window(ctx, cams, tiles, blocks_per_cu=2)
    ge, gg = torch.zeros_like(pd), torch.zeros_like(pd)
    le, lg = torch.zeros(len(cams), device="cuda"), torch.zeros(len(cams), device="cuda")
    for k in range(5):
        for j, (tr, tdp) in enumerate(targets):
            g = synth.rng(100 * k + j)
            tr.copy_(torch.as_tensor(g.uniform(size=tuple(tr.shape)), dtype=torch.float32))
            tdp.copy_(torch.as_tensor(g.uniform(1, 4, tuple(tdp.shape)), dtype=torch.float32))
        junk = torch.randn(1 << 20, device="cuda").sum()  # unrelated work on the same stream
        wg.step(pd, n, zero, targets, fgs.RenderOpts(), loss=lg, grad_out=gg, graph=True)
        we.step(pd, n, zero, targets, fgs.RenderOpts(), loss=le, grad_out=ge, graph=False)
        ctx.check()
        torch.cuda.synchronize()
        assert np.isfinite(float(junk))
        np.testing.assert_allclose(host(lg), host(le), rtol=1e-6, err_msg=f"replay {k}")
        assert_close_rel(host(gg), host(ge), 1e-5, what=f"replay {k} gradient", floor=1e-2)
    we.close()
    wg.close()


def test_graph_adam_reads_the_device_step(fgs, ctx):
    """After three captured steps, the fourth uses bias correction for step 4: its update equals one
    computed on the host from the snapshot before it and its own gradient. A step counter reset
    on the host is followed by the device."""
    import torch
    cams, tiles = small_views()
    p = synth.frustum_scene(5, 1500, cams[0], 1.0, 5.0)
    n = p.shape[1]
    pd = dev(p)
    targets = random_targets(cams, 90)
    adam = fgs.Adam.like(pd, lr=LR)
    grad = torch.zeros_like(pd)
    win = fgs.Window(ctx, cams, tiles)
    b1, b2 = float(np.float32(0.9)), float(np.float32(0.999))
    for k in range(6):
        if k == 4:
            adam.step = 10  # the host resets the counter; the device copy must follow
        snap = [host(t).astype(np.float64) for t in (pd, adam.m, adam.v)]
        t = adam.step + 1
        win.step(pd, n, adam, targets, fgs.RenderOpts(), grad_out=grad, graph=True)
        ctx.check()
        g = host(grad).astype(np.float64)
        p0, m0, v0 = snap
        m1 = b1 * m0 + (1 - b1) * g
        v1 = b2 * v0 + (1 - b2) * g * g
        lr = np.array(LR)[GROUP][:, None]
        expect = p0 - lr * (m1 / (1 - b1 ** t)) / (np.sqrt(v1 / (1 - b2 ** t)) + 1e-15)
        big = np.abs(g) >= 1e-3 * np.abs(g).max(axis=1, keepdims=True)
        step = np.abs(expect - p0)
        err = np.abs(host(pd).astype(np.float64) - expect)
        ulp = np.spacing(np.abs(expect).astype(np.float32)).astype(np.float64)
        assert np.all((err <= 1e-4 * step + 2 * ulp + 1e-5 * lr)[big]), f"step {k} (t = {t})"
    assert adam.step == 12
    win.close()


def test_overflow_in_a_replay_is_reported_and_recovered(fgs, ctx):
    """Gaussians grown in place after the window was sized: the replay overflows a view's state and
    leaves the parameters, the Adam moments and the device step count as they were (nonzero
    learning rates); the next call reports FGS_ERR_CAPACITY once and sets the host's step count
    back; the call after it resizes, equals the plain mapping step again and applies update
    number 2."""
    import torch
    cams, tiles = small_views()
    p = synth.frustum_scene(6, 2000, cams[0], 1.0, 5.0)
    p[3:6] = -6.0  # tiny: about one tile each
    n = p.shape[1]
    pd = dev(p)
    targets = random_targets(cams, 110)
    adam = fgs.Adam.like(pd, lr=LR)
    grad = torch.zeros_like(pd)
    win = fgs.Window(ctx, cams, tiles)
    win.step(pd, n, adam, targets, fgs.RenderOpts(), grad_out=grad, graph=True)
    ctx.check()
    assert adam.step == 1
    pd[3:6] = -1.5  # large footprints: many more (tile, gaussian) pairs
    snap = [host(t).copy() for t in (pd, adam.m, adam.v)]
    win.step(pd, n, adam, targets, fgs.RenderOpts(), grad_out=grad, graph=True)  # overflows, not yet known
    torch.cuda.synchronize()
    for name, t, s in zip(("params", "m", "v"), (pd, adam.m, adam.v), snap):
        np.testing.assert_array_equal(host(t), s, err_msg=f"{name} changed by the overflowed step")
    with pytest.raises(fgs.FgsError) as e:
        win.step(pd, n, adam, targets, fgs.RenderOpts(), grad_out=grad, graph=True)
    assert e.value.status == fgs.ERR_CAPACITY and "grown" in str(e.value) and "not applied" in str(e.value)
    assert adam.step == 1, "the overflowed step is not counted"
    ctx.check()  # the context's own overflow word was cleared by the window's report
    ref = torch.zeros_like(pd)
    fgs.map_step(ctx, pd, n, fgs.Adam.like(pd, lr=(0, 0, 0, 0, 0)), cams, targets, fgs.RenderOpts(), grad_out=ref)
    ctx.check()
    p0, m0, v0 = (s.astype(np.float64) for s in snap)
    win.step(pd, n, adam, targets, fgs.RenderOpts(), grad_out=grad, graph=True)
    ctx.check()
    assert adam.step == 2
    assert_close_rel(host(grad), host(ref), 1e-5, what="after recovery", floor=1e-2)
    # update number 2 from the state the overflowed step left
    g = host(grad).astype(np.float64)
    b1, b2 = float(np.float32(0.9)), float(np.float32(0.999))
    m1 = b1 * m0 + (1 - b1) * g
    v1 = b2 * v0 + (1 - b2) * g * g
    lr = np.array(LR)[GROUP][:, None]
    expect = p0 - lr * (m1 / (1 - b1 ** 2)) / (np.sqrt(v1 / (1 - b2 ** 2)) + 1e-15)
    err = np.abs(host(pd).astype(np.float64) - expect)
    ulp = np.spacing(np.abs(expect).astype(np.float32)).astype(np.float64)
    assert np.all(err <= 1e-4 * np.abs(expect - p0) + 2 * ulp + 1e-5 * lr), "update 2 after recovery"
    win.close()


def test_graph_recaptured_after_the_context_workspace_grows(fgs):
    """A captured window step bakes in the context's sort and binning buffers. A larger mapping step
    on the same context grows (reallocates) them; the next graphed window step must be captured
    again, not replay the old addresses. Each graphed step equals an eager step on the same
    inputs."""
    import torch
    c = fgs.Context()  # fresh: its workspace is sized by the small window first
    cams, tiles = small_views()
    p = synth.frustum_scene(7, 1500, cams[0], 1.0, 5.0)
    n = p.shape[1]
    pd = dev(p)
    targets = random_targets(cams, 130)
    zero = fgs.Adam.like(pd, lr=(0, 0, 0, 0, 0))
    wg, we = fgs.Window(c, cams, tiles), fgs.Window(c, cams, tiles)
    gg, ge = torch.zeros_like(pd), torch.zeros_like(pd)
    lg, le = torch.zeros(len(cams), device="cuda"), torch.zeros(len(cams), device="cuda")

    def compare(what):
        wg.step(pd, n, zero, targets, fgs.RenderOpts(), loss=lg, grad_out=gg, graph=True)
        we.step(pd, n, zero, targets, fgs.RenderOpts(), loss=le, grad_out=ge, graph=False)
        c.check()
        np.testing.assert_allclose(host(lg), host(le), rtol=1e-6, err_msg=what)
        assert_close_rel(host(gg), host(ge), 1e-5, what=f"{what} gradient", floor=1e-2)

    compare("before")
    compare("replay")
    big_cam = synth.camera_replica()
    big = dev(synth.frustum_scene(8, 200_000, big_cam, 0.5, 8.0))
    bt = [(dev(synth.rng(140).uniform(size=(3, big_cam.height, big_cam.width))),
           dev(synth.rng(141).uniform(1, 4, (big_cam.height, big_cam.width))))]
    fgs.map_step(c, big, 200_000, fgs.Adam.like(big, lr=(0, 0, 0, 0, 0)), [big_cam], bt, fgs.RenderOpts())
    c.check()
    del big, bt
    compare("after the workspace grew")
    compare("replay after the workspace grew")
    wg.close()
    we.close()
    c.close()


def test_profiled_window_step_runs_eagerly(fgs, ctx):
    import torch
    cams, tiles = small_views()
    p = synth.frustum_scene(7, 1000, cams[0], 1.0, 5.0)
    pd = dev(p)
    targets = random_targets(cams, 130)
    win = fgs.Window(ctx, cams, tiles)
    ctx.profile(3)
    adam = fgs.Adam.like(pd)
    for _ in range(3):
        win.step(pd, p.shape[1], adam, targets, fgs.RenderOpts(), graph=True)
    ctx.check()
    rep = ctx.profile_report()
    ctx.profile(0)
    assert rep["raster_fwd"][1] == 3 and rep["raster_bwd"][1] == 3 and rep["project_bwd"][1] == 3
    assert rep["counts"]["forwards"] == 3 * len(cams) and rep["counts"]["pairs_blended"] > 0
    torch.cuda.synchronize()
    win.close()


def test_empty_window(fgs, ctx):
    """No gaussians: every view renders the background, so each view's loss is the L1 loss of the
    background against its target, as the plain mapping step reports it, and nothing faults."""
    import torch
    cams, tiles = small_views()
    targets = random_targets(cams, 40)
    pd = dev(np.zeros((14, 1), np.float32))
    lw = torch.zeros(len(cams), device="cuda")
    lm = torch.zeros(len(cams), device="cuda")
    win = fgs.Window(ctx, cams, tiles, 0)
    win.step(pd, 0, fgs.Adam.like(pd), targets, fgs.RenderOpts(), loss=lw, graph=False)
    win.close()
    fgs.map_step(ctx, pd, 0, fgs.Adam.like(pd), cams, targets, fgs.RenderOpts(), loss=lm)
    ctx.check()
    assert np.all(np.isfinite(host(lw)))
    np.testing.assert_allclose(host(lw), host(lm), rtol=1e-6)


def test_full_window_workload(fgs, ctx):
    """The 8-view window over the 500k-gaussian box scene (four 640x480, four 1200x680 views) in the
    launch configuration the benchmark times.

    The window's losses equal single-view renders (1e-5). Its gradient is compared with the plain
    mapping step's over the same views, per parameter row. Opacity and colour gradients are well
    conditioned: relative L2 error 1e-5 and largest difference 1e-4 of the row's largest entry.
    The geometric rows (mean, log-scale, rotation) are not reproducible to that level by any FP32
    path at this size: L1-loss gradients are sums of +-1-weighted pixel terms that cancel heavily,
    and cameras inside the box see gaussians just past the near plane whose gradients cancel over
    most of a view, so the FP32 atomic order alone moves these rows by up to 5e-4 in relative L2
    (measured between two runs of the same plain step); they are held to 2e-3 in relative L2 and
    1e-2 of the row's largest entry, which any missing view, tile or term would exceed by orders
    of magnitude. Elementwise parity with the oracle is asserted on the small windows above. A
    graph replay is compared with an eager step the same way."""
    import torch
    cams = synth.window_cameras(0)
    p = synth.scene_window(0)
    n = p.shape[1]
    pd = dev(p)
    tscene = dev(synth.scene_window(1))
    targets = []
    for c in cams:
        t = fgs.render(ctx, tscene, n, c, fgs.RenderOpts(), aux=False)
        targets.append((t["rgb"], t["depth"]))
    del tscene
    lopts = fgs.LossOpts()
    ref_loss = per_view_losses(fgs, ctx, pd, n, cams, targets, lopts)
    zero = fgs.Adam.like(pd, lr=(0, 0, 0, 0, 0))
    ref = torch.zeros_like(pd)
    fgs.map_step(ctx, pd, n, zero, cams, targets, fgs.RenderOpts(), lopts, grad_out=ref)
    ctx.check()
    ref = host(ref).astype(np.float64)
    win = fgs.Window(ctx, cams)
    loss = torch.zeros(8, device="cuda")
    ga, gb = torch.zeros_like(pd), torch.zeros_like(pd)
    win.step(pd, n, zero, targets, fgs.RenderOpts(), lopts, loss=loss, grad_out=ga, graph=False)
    ctx.check()
    np.testing.assert_allclose(host(loss), ref_loss, rtol=1e-5)
    win.step(pd, n, zero, targets, fgs.RenderOpts(), lopts, loss=loss, grad_out=gb, graph=True)
    win.step(pd, n, zero, targets, fgs.RenderOpts(), lopts, loss=loss, grad_out=gb, graph=True)
    ctx.check()
    np.testing.assert_allclose(host(loss), ref_loss, rtol=1e-5)
    g_a, g_b = host(ga).astype(np.float64), host(gb).astype(np.float64)
    l2_tol = np.array([2e-3] * 10 + [1e-5] * 4)
    max_tol = np.array([1e-2] * 10 + [1e-4] * 4)
    for what, x, y in (("window vs map_step", g_a, ref), ("replay vs eager", g_b, g_a)):
        l2 = np.linalg.norm(x - y, axis=1) / np.linalg.norm(y, axis=1)
        worst = np.abs(x - y).max(axis=1) / np.abs(y).max(axis=1)
        assert np.all(l2 <= l2_tol), (what, "relative L2 per row", l2)
        assert np.all(worst <= max_tol), (what, "max error / row max", worst)
    win.close()
