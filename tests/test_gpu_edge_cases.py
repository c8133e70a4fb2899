"""GPU parity on the method's degenerate and boundary cases, against the FP64 oracle through the
C ABI: opacities that hit the alpha clamp, gaussians at exactly equal depth (whose blending order is
the index order), and invalid parameters (zero quaternion, NaN or infinite entries) that both sides
must cull alike. Tolerances as in the render tests: 1e-5 relative for rendered planes; gradients 1e-4
relative plus the rounding allowance on each sum's absolute mass (gpu_helpers.assert_grad_close)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import assert_close_rel, dev, host, need_gpu, oracle_opts, assert_grad_close

pytestmark = pytest.mark.gpu

FWD_TOL, GRAD_TOL = 1e-5, 1e-4
ROWS = (("mean", slice(0, 3)), ("log_scale", slice(3, 6)), ("quat", slice(6, 10)), ("opacity", slice(10, 11)),
        ("rgb", slice(11, 14)))


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


def compare(fgs, ctx, p, cam, skip, seed, what, check_nan_free=True):
    """Forward planes and all 14 gradient rows against the oracle; `skip` (H, W) marks the pixels
    left out of the forward comparison, whose upstream gradient is set to zero."""
    n = p.shape[1]
    pd = dev(p)
    out = fgs.render(ctx, pd, n, cam, fgs.RenderOpts())
    ref = oracle.render_fwd(p.astype(np.float64), cam, oracle_opts(), mode=0, amb_rel=1e-5)
    ok = ~skip
    for k in ("depth", "alpha", "T_final"):
        assert_close_rel(host(out[k]), ref[k], FWD_TOL, ok, f"{what}: {k}")
    assert_close_rel(host(out["rgb"]), ref["rgb"], FWD_TOL, ok, f"{what}: rgb")
    np.testing.assert_array_equal(host(out["n_contrib"])[ok], ref["n_contrib"][ok], err_msg=f"{what}: n_contrib")
    P = cam.width * cam.height
    g = synth.rng(2000 + seed)
    gr = g.normal(size=(3, P))
    gd = g.normal(size=P)
    ga = g.normal(size=P)
    s = skip.ravel()
    gr[:, s] = 0
    gd[s] = 0
    ga[s] = 0
    gr, gd, ga = (a.astype(np.float32) for a in (gr, gd, ga))
    H, W = cam.height, cam.width
    import torch
    grad = torch.zeros_like(pd)
    fgs.render_bwd(ctx, pd, n, cam, fgs.RenderOpts(), out["state"], dev(gr.reshape(3, H, W)), dev(gd.reshape(H, W)),
                   dev(ga.reshape(H, W)), grad)
    ctx.check()
    gref, _, mass = oracle.render_bwd(p.astype(np.float64), cam, gr, gd, ga, oracle_opts(), mode=0, mass=True)
    gg = host(grad)
    if check_nan_free:
        assert np.isfinite(gg).all(), f"{what}: non-finite gradient"
    assert_grad_close(gg, gref, mass, what, tol=GRAD_TOL)
    return ref, gg, gref


@pytest.mark.parametrize("seed", [0, 1])
def test_clamped_opacities(fgs, ctx, seed):
    """Logits around 6 (opacity 0.99-0.999): most pairs at a gaussian's centre hit the alpha <= 0.99
    clamp, which passes no gradient to opacity, 2D mean or conic. At least a few hundred pixels are
    checked through clamped pairs."""
    cam = synth.camera_small()
    p = synth.scene_small(20 + seed)
    p[10] = synth.rng(30 + seed).normal(6.0, 0.5, size=p.shape[1])
    ref = oracle.render_fwd(p.astype(np.float64), cam, oracle_opts(), amb_rel=1e-5)
    assert ref["n_amb"] <= 0.02 * cam.width * cam.height
    # gaussians clamped at the pixel centre nearest their projected mean
    pr = oracle.project(p.astype(np.float64), cam)
    v = pr[:, 0] > 0
    m2 = pr[v][:, 10:12]
    d = np.floor(m2) + 0.5 - m2
    a, b, c = pr[v][:, 7], pr[v][:, 8], pr[v][:, 9]
    Q = a * d[:, 0] ** 2 + 2 * b * d[:, 0] * d[:, 1] + c * d[:, 1] ** 2
    assert (pr[v][:, 13] * np.exp(-0.5 * Q) > 0.99).sum() >= 100
    compare(fgs, ctx, p, cam, ref["amb"], seed, f"clamped seed {seed}")


def tie_scene(seed, n=1000):
    """n pairs of gaussians; the two members of pair i share one mean (so one camera depth) and
    differ in shape, rotation, opacity and colour. Depths are multiples of 2^-10 m, so the depths
    of different pairs differ by at least 2^-10 m (no near-ties) while a pair's are exactly equal.
    Member a of pair i has index i, member b index n + i."""
    cam = synth.camera_small()
    a = synth.frustum_scene(seed, n, cam, 1.0, 5.0)
    b = synth.frustum_scene(seed + 500, n, cam, 1.0, 5.0)
    a[2] = np.round(a[2] * 1024.0) / 1024.0
    b[0:3] = a[0:3]
    b[10] = a[10] + 1.0  # more opaque: the order visibly changes the colour
    return cam, np.concatenate([a, b], axis=1)


def test_exact_depth_ties_blend_in_index_order(fgs, ctx):
    """Equal depths blend in ascending index (both the oracle and the HIP path). Pixels where two
    contributors tie are compared, not masked: only cutoff ambiguities are left out."""
    cam, p = tie_scene(40)
    ref = oracle.render_fwd(p.astype(np.float64), cam, oracle_opts(), amb_rel=1e-5)
    assert ref["amb_tie"].sum() >= 1000, "the scene must put tied pairs on most pixels"
    assert ref["amb_cut"].sum() <= 0.02 * cam.width * cam.height
    # the order matters: with the members' indices swapped the oracle's image changes
    n = p.shape[1] // 2
    sw = np.concatenate([p[:, n:], p[:, :n]], axis=1)
    ref_sw = oracle.render_fwd(sw.astype(np.float64), cam, oracle_opts(), amb_rel=0)
    ok = ~ref["amb_cut"]
    assert np.abs(ref_sw["rgb"] - ref["rgb"])[:, ok].max() > 1e-2
    compare(fgs, ctx, p, cam, ref["amb_cut"], 3, "ties")
    compare(fgs, ctx, sw, cam, ref["amb_cut"] | oracle.render_fwd(sw.astype(np.float64), cam, oracle_opts(), amb_rel=1e-5)["amb_cut"],
            4, "ties, swapped")


def test_invalid_parameters_are_culled_like_the_oracle(fgs, ctx):
    """Zero quaternions and NaN means, log-scales, quaternions or logits, and +inf log-scales are
    culled by both sides (no contribution, zero gradient); -inf log-scales (a point whose footprint
    is the screen low-pass alone) and +-inf logits (opacity 1 or 0) stay valid and match."""
    cam = synth.camera_small()
    p = synth.scene_small(9).copy()
    nan = np.float32(np.nan)
    p[6:10, 0:20] = 0.0
    p[0, 20:40] = nan
    p[4, 40:60] = nan
    p[7, 60:80] = nan
    p[10, 80:100] = nan
    p[3:6, 100:120] = np.inf
    p[3:6, 120:140] = -np.inf
    p[10, 140:160] = np.inf
    p[10, 160:180] = -np.inf
    culled = np.zeros(p.shape[1], bool)
    culled[0:120] = True
    proj = oracle.project(p.astype(np.float64), cam)
    assert not proj[culled, 0].any(), "the oracle culls every invalid gaussian"
    assert proj[120:180, 0].all(), "-inf log-scales and +-inf logits stay valid"
    ref = oracle.render_fwd(p.astype(np.float64), cam, oracle_opts(), amb_rel=1e-5)
    _, gg, gref = compare(fgs, ctx, p, cam, ref["amb"], 5, "invalid parameters")
    assert np.all(gg[:, culled] == 0), "culled gaussians receive no gradient"
    assert np.all(gref[:, culled] == 0)
    # the same scene without the culled gaussians renders the same image
    keep = ~culled
    pk = p[:, keep].copy()
    out_k = fgs.render(ctx, dev(pk), pk.shape[1], cam, fgs.RenderOpts())
    out_a = fgs.render(ctx, dev(p), p.shape[1], cam, fgs.RenderOpts())
    np.testing.assert_array_equal(host(out_k["rgb"]), host(out_a["rgb"]))
    np.testing.assert_array_equal(host(out_k["n_contrib"]), host(out_a["n_contrib"]))
