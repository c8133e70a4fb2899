"""Worked examples derived by hand from the paper's definitions (tests/golden/*.json, each with its
citation and derivation): the oracle must reproduce them exactly, and the HIP path within FP32
rounding."""
import json
import os

import numpy as np
import pytest

import oracle
from gpu_helpers import dev, host, need_gpu
from synth import Camera

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def blend_case():
    g = load("blend_three_on_axis.json")
    c = g["camera"]
    cam = Camera(c["width"], c["height"], c["fx"], c["fy"], c["cx"], c["cy"])
    p = np.zeros((14, len(g["gaussians"])))
    for i, q in enumerate(g["gaussians"]):
        p[0:3, i] = q["mean"]
        p[3:6, i] = q["log_scale"]
        p[6:10, i] = q["quat"]
        p[10, i] = q["opacity_logit"]
        p[11:14, i] = q["rgb"]
    return g, cam, p


def test_oracle_blend_three_on_axis():
    """Eq. 1 worked example: three gaussians projecting onto one pixel centre (G = 1)."""
    g, cam, p = blend_case()
    o = oracle.RenderOpts(bg=tuple(g["render_opts"]["bg"]), bg_depth=g["render_opts"]["bg_depth"])
    out = oracle.render_fwd(p, cam, o, mode=1)
    x, y = g["pixel"]
    e = g["expected"]
    np.testing.assert_allclose(out["rgb"][:, y, x], e["rgb"], rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(out["depth"][y, x], e["depth"], rtol=1e-14)
    np.testing.assert_allclose(out["alpha"][y, x], e["alpha"], rtol=1e-14)
    np.testing.assert_allclose(out["T_final"][y, x], e["T_final"], rtol=1e-14)
    assert out["n_contrib"][y, x] == e["n_contrib"]


def test_oracle_triangle_threshold_cases():
    """Triangle threshold worked examples, and their mirror images."""
    g = load("triangle_threshold.json")
    for case in g["cases"]:
        h = np.asarray(case["hist"], np.int64)
        assert len(h) == 256
        assert oracle.triangle(h) == case["threshold"], case["name"]
        assert oracle.triangle(h[::-1].copy()) == 255 - case["threshold"], case["name"]


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


@pytest.mark.gpu
def test_gpu_blend_three_on_axis(fgs, ctx):
    """The HIP path on the Eq. 1 worked example, through the C ABI (FP32: the opacities carry the
    rounding of the sigmoid of an FP32 logit)."""
    g, cam, p = blend_case()
    o = fgs.RenderOpts(bg=tuple(g["render_opts"]["bg"]), bg_depth=g["render_opts"]["bg_depth"])
    out = fgs.render(ctx, dev(p), p.shape[1], cam, o)
    x, y = g["pixel"]
    e = g["expected"]
    np.testing.assert_allclose(host(out["rgb"])[:, y, x], e["rgb"], rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(host(out["depth"])[y, x], e["depth"], rtol=1e-6)
    np.testing.assert_allclose(host(out["alpha"])[y, x], e["alpha"], rtol=1e-6)
    np.testing.assert_allclose(host(out["T_final"])[y, x], e["T_final"], rtol=1e-6)
    assert int(host(out["n_contrib"])[y, x]) == e["n_contrib"]


# ------------------------------------------------------------------ alpha clamp (R-P8)

def params_of(gs):
    p = np.zeros((14, len(gs)))
    for i, q in enumerate(gs):
        p[0:3, i] = q["mean"]
        p[3:6, i] = q["log_scale"]
        p[6:10, i] = q.get("quat", [1, 0, 0, 0])
        p[10, i] = q.get("opacity_logit", 0.0)
        p[11:14, i] = q.get("rgb", [0.5, 0.5, 0.5])
    return p


def camera_of(g):
    c = g["camera"]
    return Camera(c["width"], c["height"], c["fx"], c["fy"], c["cx"], c["cy"])


def clamp_case():
    g = load("alpha_clamp_pair.json")
    cam = camera_of(g)
    p = params_of(g["gaussians"])
    P = cam.width * cam.height
    x, y = g["pixel"]
    u = g["upstream"]
    gr = np.zeros((3, P))
    gd = np.zeros(P)
    ga = np.zeros(P)
    gr[:, y * cam.width + x] = u["rgb"]
    gd[y * cam.width + x] = u["depth"]
    ga[y * cam.width + x] = u["alpha"]
    exp_grad = np.zeros((14, 2))
    for i, q in enumerate(g["expected"]["grad"]):
        exp_grad[:, i] = q["mean"] + q["log_scale"] + q["quat"] + [q["opacity_logit"]] + q["rgb"]
    return g, cam, p, (gr, gd, ga), exp_grad


def pixel_loss(p, cam, g, up):
    out = oracle.render_fwd(p, cam, mode=1, amb_rel=0)
    x, y = g["pixel"]
    u = g["upstream"]
    return float(np.dot(u["rgb"], out["rgb"][:, y, x]) + u["depth"] * out["depth"][y, x] +
                 u["alpha"] * out["alpha"][y, x])


def test_oracle_alpha_clamp_pair():
    """A pair clamped at alpha = 0.99 in front of an unclamped one: the forward values and the
    analytic gradient worked out by hand (the clamped pair passes gradient to its colour and depth
    only), and central finite differences of the oracle's own forward agreeing with both."""
    g, cam, p, up, exp_grad = clamp_case()
    e = g["expected"]
    x, y = g["pixel"]
    for mode in (0, 1):
        out = oracle.render_fwd(p, cam, mode=mode, amb_rel=0)
        np.testing.assert_allclose(out["rgb"][:, y, x], e["rgb"], rtol=1e-14, atol=1e-15)
        np.testing.assert_allclose(out["depth"][y, x], e["depth"], rtol=1e-14)
        np.testing.assert_allclose(out["alpha"][y, x], e["alpha"], rtol=1e-14)
        np.testing.assert_allclose(out["T_final"][y, x], e["T_final"], rtol=1e-12)
        assert out["n_contrib"][y, x] == e["n_contrib"]
    grad, _ = oracle.render_bwd(p, cam, *up, mode=1)
    np.testing.assert_allclose(grad, exp_grad, rtol=1e-12, atol=1e-15)
    h = 1e-6
    fd = np.zeros_like(grad)
    for r in range(14):
        for i in range(2):
            pp, pm = p.copy(), p.copy()
            pp[r, i] += h
            pm[r, i] -= h
            fd[r, i] = (pixel_loss(pp, cam, g, up) - pixel_loss(pm, cam, g, up)) / (2 * h)
    np.testing.assert_allclose(fd, exp_grad, rtol=0, atol=1e-8)
    # the pin has teeth: without the clamp the front gaussian's opacity and 2D position would
    # receive gradient
    o = oracle.RenderOpts(alpha_max=0.999)
    free, _ = oracle.render_bwd(p, cam, *up, opts=o, mode=1)
    assert abs(free[10, 0]) > 1e-4 and abs(free[0, 0]) > 1e-4


# ------------------------------------------------------------------ duplicate count

def duplicates_case():
    g = load("duplicates_six_gaussians.json")
    return g, camera_of(g), params_of(g["gaussians"])


def test_oracle_duplicates_counted_by_hand():
    """(tile, gaussian) pairs of six gaussians across tile borders, off screen and behind the near
    plane, counted by hand for 16x16 and 32x8 tiles, in total and gaussian by gaussian."""
    g, cam, p = duplicates_case()
    for shape, (tw, th) in (("16x16", (16, 16)), ("32x8", (32, 8))):
        e = g["expected"][shape]
        assert oracle.count_duplicates(p, cam, tw, th) == e["total"], shape
        for i, k in enumerate(e["per_gaussian"]):
            assert oracle.count_duplicates(p[:, i:i + 1].copy(), cam, tw, th) == k, (shape, g["gaussians"][i]["name"])


# ------------------------------------------------------------------ bf16 rounding in the MLP backward

MLP_OFFS = dict(zip(("W1", "b1", "W2", "b2", "W3", "b3"), np.cumsum([0, 256 * 260, 256, 256 * 256, 256, 4 * 256])))
MLP_COLS = {"W1": 260, "W2": 256, "W3": 256}


def mlp_index(name, entry):
    if name in MLP_COLS:
        return int(MLP_OFFS[name] + entry[0] * MLP_COLS[name] + entry[1])
    return int(MLP_OFFS[name] + entry[0])


def mlp_case():
    g = load("mlp_bf16_backward.json")
    w = np.zeros(oracle.MLP_PARAMS)
    for name, entries in g["weights"].items():
        for e in entries:
            w[mlp_index(name, e[:-1])] = e[-1]
    x = np.zeros((1, 260))
    for k, v in g["x"].items():
        x[0, int(k)] = v
    t = np.asarray([g["target"]], np.float64)
    expect = np.zeros(oracle.MLP_PARAMS)
    for name, entries in g["expected_bf16"].items():
        if name == "loss":
            continue
        for e in entries:
            expect[mlp_index(name, e[:-1])] = e[-1]
    return g, w, x, t, expect


def test_oracle_mlp_backward_bf16_rounding_points():
    """A network with one active unit per layer whose upstream gradients are not bfloat16 values:
    every weight gradient carries the rounding of its upstream-gradient operand (and of the input),
    the bias gradients do not; the values are worked out by hand, and the unrounded network gives
    the different values the derivation lists."""
    g, w, x, t, expect = mlp_case()
    grad, L = oracle.mlp_bwd(x, w, t, bf16=True)
    assert abs(L - g["expected_bf16"]["loss"]) <= 1e-15
    np.testing.assert_allclose(grad, expect, rtol=1e-12, atol=0)
    plain, _ = oracle.mlp_bwd(x, w, t, bf16=False)
    c = g["unrounded_for_contrast"]
    np.testing.assert_allclose(plain[mlp_index("W3", (0, 0))], c["W3"], rtol=1e-12)
    np.testing.assert_allclose(plain[mlp_index("W2", (0, 0))], c["W2"], rtol=1e-12)
    np.testing.assert_allclose(plain[mlp_index("W1", (0, 0))], c["W1_0"], rtol=1e-12)


@pytest.mark.gpu
def test_gpu_alpha_clamp_pair(fgs, ctx):
    """The HIP path on the clamped-pair example through the C ABI: forward values and all 28
    parameter gradients within FP32 rounding of the hand-derived ones (zero stays zero)."""
    import torch
    g, cam, p, up, exp_grad = clamp_case()
    e = g["expected"]
    x, y = g["pixel"]
    pd = dev(p)
    out = fgs.render(ctx, pd, 2, cam, fgs.RenderOpts())
    np.testing.assert_allclose(host(out["rgb"])[:, y, x], e["rgb"], rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(host(out["depth"])[y, x], e["depth"], rtol=1e-6)
    np.testing.assert_allclose(host(out["alpha"])[y, x], e["alpha"], rtol=1e-6)
    np.testing.assert_allclose(host(out["T_final"])[y, x], e["T_final"], rtol=1e-4)
    assert int(host(out["n_contrib"])[y, x]) == e["n_contrib"]
    grad = torch.zeros_like(pd)
    H, W = cam.height, cam.width
    fgs.render_bwd(ctx, pd, 2, cam, fgs.RenderOpts(), out["state"], dev(up[0].reshape(3, H, W)),
                   dev(up[1].reshape(H, W)), dev(up[2].reshape(H, W)), grad)
    ctx.check()
    np.testing.assert_allclose(host(grad), exp_grad, rtol=1e-5, atol=1e-7 * np.abs(exp_grad).max())


@pytest.mark.gpu
def test_gpu_duplicates_counted_by_hand(fgs, ctx):
    """The HIP binning lists exactly the hand-counted (tile, gaussian) pairs for both tile shapes."""
    g, cam, p = duplicates_case()
    for shape, (tw, th) in (("16x16", (16, 16)), ("32x8", (32, 8))):
        fgs.render(ctx, dev(p), p.shape[1], cam, fgs.RenderOpts(tile_w=tw, tile_h=th))
        assert ctx.stats()["pairs"] == g["expected"][shape]["total"], shape


@pytest.mark.gpu
def test_gpu_mlp_backward_bf16_rounding_points(fgs, ctx):
    """The HIP network's gradient (bf16 MFMA operands, FP32 accumulation) on the hand-worked
    example: every entry within FP32 rounding of the derived values, all others zero."""
    import torch
    g, w, x, t, expect = mlp_case()
    wd = dev(w)
    adam = fgs.PriorAdam.like(wd, lr=0.0)
    grad = torch.zeros_like(wd)
    loss = torch.zeros(1, device="cuda")
    fgs.prior_train_step(ctx, dev(x), dev(t), wd, adam, loss=loss, grad_out=grad)
    ctx.check()
    assert abs(float(loss) - g["expected_bf16"]["loss"]) <= 1e-6
    np.testing.assert_allclose(host(grad), expect, rtol=1e-6, atol=1e-6)
