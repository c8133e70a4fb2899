"""The structural-similarity term and the scale regulariser of the mapping loss (Sec. III-D,
Eq. 15 and Eq. 16) on the GPU against the oracle: the SSIM kernel on identical FP32 inputs, and
the mapping step with the full loss end to end."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import U32, assert_grad_close, dev, host, need_gpu, oracle_opts

pytestmark = pytest.mark.gpu

LR = (1e-3, 5e-3, 1e-3, 5e-2, 2.5e-3)


@pytest.fixture(scope="module")
def fgs():
    need_gpu()
    import paper_2503_01109_amd as F
    return F


@pytest.fixture(scope="module")
def ctx(fgs):
    return fgs.Context()


def ssim_errors(gpu_grad, ref_grad):
    e = np.abs(np.asarray(gpu_grad, np.float64) - ref_grad)
    scale = np.abs(ref_grad).max()
    return e.max() / scale, e


@pytest.mark.parametrize("shape,seed", [((48, 64), 1), ((45, 70), 2), ((680, 1200), 3)])
def test_ssim_matches_oracle(fgs, ctx, shape, seed):
    """Random images with smooth and noisy parts (several 16x16 tiles, ragged edges at 70x45, the
    full 1200x680 frame): the index within 5e-7 (FP32 window moments, FP64 final sum; measured up to
    6e-8), the gradient within 2e-5 of its largest entry (measured 3e-6) and 5e-4 relative where it
    exceeds 1e-2 of it (measured 1.2e-4: the index's partials subtract terms up to 2 mu / C2 ~ 2e3
    times the index, so FP32 rounding of the moments is amplified where the contrast is low)."""
    import torch
    H, W = shape
    g = synth.rng(seed)
    yy, xx = np.mgrid[0:H, 0:W] / max(H, W)
    base = 0.5 + 0.3 * np.sin(6 * xx)[None] * np.cos(4 * yy)[None]
    img = np.clip(base + 0.1 * g.normal(size=(3, H, W)), 0, 1).astype(np.float32)
    tgt = np.clip(base + 0.15 * g.normal(size=(3, H, W)), 0, 1).astype(np.float32)
    v = torch.zeros(1, device="cuda")
    grad = torch.empty((3, H, W), device="cuda")
    fgs.ssim(ctx, dev(img), dev(tgt), v, grad)
    ctx.check()
    s_ref, g_ref, _ = oracle.ssim(img.astype(np.float64), tgt.astype(np.float64))
    assert abs(float(v) - s_ref) <= 5e-7, (float(v), s_ref)
    rel, e = ssim_errors(host(grad), g_ref)
    scale = np.abs(g_ref).max()
    big = np.abs(g_ref) > 1e-2 * scale
    worst = (e[big] / np.abs(g_ref[big])).max()
    print(f"ssim {W}x{H}: |dv| {abs(float(v) - s_ref):.2e}, grad max err / max {rel:.2e}, worst rel (>1e-2 max) {worst:.2e}")
    assert rel <= 2e-5
    assert worst <= 5e-4


def test_ssim_of_an_image_with_itself(fgs, ctx):
    import torch
    img = synth.rng(4).uniform(0, 1, (3, 40, 56)).astype(np.float32)
    v = torch.zeros(1, device="cuda")
    grad = torch.empty((3, 40, 56), device="cuda")
    fgs.ssim(ctx, dev(img), dev(img), v, grad)
    assert abs(float(v) - 1.0) < 1e-6
    # the gradient vanishes up to FP32 rounding of terms that cancel exactly
    assert np.abs(host(grad)).max() < 1e-9


def full_loss_reference(p, cam, trgb, td, li, ld, lr_):
    """Oracle mapping step terms with the full loss: image loss, regulariser value, gradient and its
    absolute mass (the regulariser's gradient counted in the mass of the log-scale rows)."""
    p64 = p.astype(np.float64)
    ref = oracle.render_fwd(p64, cam, oracle_opts(), amb_rel=0)
    L1, _, gr, gd = oracle.loss_l1(ref["rgb"], ref["depth"], trgb, td, li, ld)
    s, gs, _ = oracle.ssim(ref["rgb"], trgb)
    L = L1 + (1 - li) * (1 - s)
    gr = gr - (1 - li) * gs
    grad, _, mass = oracle.render_bwd(p64, cam, gr, gd, None, oracle_opts(), mass=True)
    reg, greg = oracle.scale_reg(p64[3:6])
    grad[3:6] += lr_ * greg
    mass[3:6] += np.abs(lr_ * greg)
    return L, reg, grad, mass


def test_map_step_with_full_loss_matches_oracle(fgs, ctx):
    """lambda_i = 0.8 (SSIM weight 0.2), lambda_d = 0.1, lambda_r = 0.05 on the 400-gaussian 64x48
    scene without ambiguous pixels: the view's loss, the regulariser's value and the summed
    gradient (all 14 rows, the same bar as the L1 step)."""
    import torch
    from test_gpu_mapstep import zero_ambiguity_scene
    p, cam, seed = zero_ambiguity_scene()
    n = p.shape[1]
    ref = oracle.render_fwd(p.astype(np.float64), cam, oracle_opts(), amb_rel=0)
    tgt = oracle.render_fwd(synth.frustum_scene(seed + 1000, n, cam, 1.0, 5.0).astype(np.float64), cam, amb_rel=0)
    trgb, td = tgt["rgb"].astype(np.float32), tgt["depth"].astype(np.float32)
    trgb[np.abs(ref["rgb"] - trgb) < 1e-3] += 0.01  # residuals away from the L1 kink
    td[np.abs(ref["depth"] - td) < 1e-3] += 0.01
    li, ld, lr_ = 0.8, 0.1, 0.05
    L, reg, gref, mass = full_loss_reference(p, cam, trgb, td, li, ld, lr_)
    pd = dev(p)
    adam = fgs.Adam.like(pd, lr=LR)
    grad = torch.zeros_like(pd)
    loss = torch.zeros(1, device="cuda")
    rv = torch.zeros(1, device="cuda")
    fgs.map_step(ctx, pd, n, adam, [cam], [(dev(trgb), dev(td))], fgs.RenderOpts(),
                 fgs.LossOpts(li, ld, lr_, rv), loss, None, grad_out=grad)
    ctx.check()
    assert float(loss) == pytest.approx(L, rel=2e-5), (float(loss), L)
    assert float(rv) == pytest.approx(reg, rel=1e-5), (float(rv), reg)
    assert_grad_close(host(grad), gref, mass, "full-loss step")


def test_regulariser_value_alone_changes_no_gradient(fgs, ctx):
    """With lambda_r = 0 and a value output the step's gradient equals the plain one to within the
    spread of the backward's float-atomic order (a regulariser gradient of lambda / n would move the
    log-scale rows by about a quarter of their size), and the value matches the oracle's."""
    import torch
    p = synth.scene_small(5)
    cam = synth.camera_small()
    n = p.shape[1]
    tg = fgs.render(ctx, dev(synth.scene_small(6)), n, cam, fgs.RenderOpts(), aux=False)
    targets = [(tg["rgb"], tg["depth"])]
    grads = []
    rv = torch.zeros(1, device="cuda")
    for lo in (fgs.LossOpts(1.0, 0.1), fgs.LossOpts(1.0, 0.1, 0.0, rv)):
        pd = dev(p)
        grad = torch.zeros_like(pd)
        fgs.map_step(ctx, pd, n, fgs.Adam.like(pd, lr=LR), [cam], targets, fgs.RenderOpts(), lo, grad_out=grad)
        grads.append(host(grad))
    ctx.check()
    for name, rows in (("log_scale", slice(3, 6)), ("all", slice(0, 14))):
        d = np.abs(grads[0][rows] - grads[1][rows]).max()
        assert d <= 1e-5 * np.abs(grads[0][rows]).max(), (name, d)
    assert float(rv) == pytest.approx(oracle.scale_reg(p[3:6].astype(np.float64))[0], rel=1e-5)


def test_window_rejects_the_ssim_and_regulariser_terms(fgs, ctx):
    import torch
    cam = synth.camera_small()
    p = synth.scene_small(7)
    pd = dev(p)
    tg = fgs.render(ctx, dev(synth.scene_small(8)), p.shape[1], cam, fgs.RenderOpts(), aux=False)
    win = fgs.Window(ctx, [cam])
    for lo in (fgs.LossOpts(0.8, 0.1), fgs.LossOpts(1.0, 0.1, 0.01)):
        with pytest.raises(fgs.FgsError) as ei:
            win.step(pd, p.shape[1], fgs.Adam.like(pd), [(tg["rgb"], tg["depth"])], fgs.RenderOpts(), lo)
        assert ei.value.status == fgs.ERR_UNSUPPORTED
    win.close()
    torch.cuda.synchronize()


def test_map_step_rejects_out_of_range_weights(fgs, ctx):
    p = synth.scene_small(9)
    cam = synth.camera_small()
    pd = dev(p)
    tg = fgs.render(ctx, dev(synth.scene_small(10)), p.shape[1], cam, fgs.RenderOpts(), aux=False)
    for lo in (fgs.LossOpts(1.2, 0.1), fgs.LossOpts(-0.1, 0.1), fgs.LossOpts(1.0, 0.1, -1.0)):
        with pytest.raises(fgs.FgsError) as ei:
            fgs.map_step(ctx, pd, p.shape[1], fgs.Adam.like(pd), [cam], [(tg["rgb"], tg["depth"])],
                         fgs.RenderOpts(), lo)
        assert ei.value.status == fgs.ERR_INVALID_ARG
