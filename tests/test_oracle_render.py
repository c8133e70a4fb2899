"""Pins of the FP64 oracle's rendering (projection + Eq. 1 compositing + backward).

Each test fixes the oracle against something other than itself: a closed form, an
invariant, a symmetry, the brute-force definition, or finite differences.
"""
import numpy as np
import pytest

import oracle
import synth
from synth import Camera

O = oracle.RenderOpts()


def one_gaussian(mu, log_s, q=(1, 0, 0, 0), logit=0.0, rgb=(0.2, 0.5, 0.9)):
    p = np.zeros((14, 1))
    p[0:3, 0] = mu
    p[3:6, 0] = log_s
    p[6:10, 0] = q
    p[10, 0] = logit
    p[11:14, 0] = rgb
    return p


def stack(*gs):
    return np.concatenate(gs, axis=1)


def test_closed_form_single_isotropic_gaussian():
    """P1: one isotropic gaussian on the optical axis, identity pose: sigma^2 = (f s / z)^2 + lowpass."""
    cam = Camera(40, 30, 50.0, 50.0, 20.0, 15.0)
    z, s, logit = 2.0, 0.04, 0.7
    p = one_gaussian((0, 0, z), [np.log(s)] * 3, q=(0.3, -0.2, 0.5, 0.4), logit=logit)
    out = oracle.render_fwd(p, cam, O, mode=1)
    sig2 = (cam.fx * s / z) ** 2 + O.lowpass
    o = 1 / (1 + np.exp(-logit))
    xs = np.arange(cam.width) + 0.5 - cam.cx
    ys = np.arange(cam.height) + 0.5 - cam.cy
    d2 = xs[None, :] ** 2 + ys[:, None] ** 2
    Q = d2 / sig2
    a = np.minimum(0.99, o * np.exp(-Q / 2))
    a = np.where((Q <= 9) & (a >= 1 / 255), a, 0.0)
    np.testing.assert_allclose(out["alpha"], a, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(out["depth"], a * z, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(out["T_final"], 1 - a, rtol=1e-12, atol=1e-15)
    for c in range(3):
        np.testing.assert_allclose(out["rgb"][c], a * p[11 + c, 0], rtol=1e-12, atol=1e-15)
    assert out["n_contrib"].sum() == (a > 0).sum()


def test_closed_form_gradients_axis_aligned():
    """P1 (backward): identity rotation, axis-aligned scales; d/d(logit, rgb, log s_x, log s_y)."""
    cam = Camera(40, 30, 50.0, 50.0, 20.0, 15.0)
    z, sx, sy, logit = 2.0, 0.05, 0.03, -0.3
    rgb = np.array([0.2, 0.5, 0.9])
    p = one_gaussian((0, 0, z), [np.log(sx), np.log(sy), np.log(0.02)], logit=logit, rgb=rgb)
    g = synth.rng(3)
    gr = g.normal(size=(3, cam.height, cam.width))
    gd = g.normal(size=(cam.height, cam.width))
    ga = g.normal(size=(cam.height, cam.width))
    grad, _ = oracle.render_bwd(p, cam, gr, gd, ga, O, mode=1)
    o = 1 / (1 + np.exp(-logit))
    vx = (cam.fx * sx / z) ** 2 + O.lowpass
    vy = (cam.fy * sy / z) ** 2 + O.lowpass
    xs = np.arange(cam.width) + 0.5 - cam.cx
    ys = np.arange(cam.height) + 0.5 - cam.cy
    Q = xs[None, :] ** 2 / vx + ys[:, None] ** 2 / vy
    a = o * np.exp(-Q / 2)
    act = (Q <= 9) & (a >= 1 / 255)
    a = np.where(act, a, 0.0)
    # outputs: rgb = a c, depth = a z, alpha = a  =>  dL/da per pixel
    dLda = (gr * rgb[:, None, None]).sum(0) + gd * z + ga
    np.testing.assert_allclose(grad[11:14, 0], (gr * a[None]).sum((1, 2)), rtol=1e-10)
    np.testing.assert_allclose(grad[10, 0], (dLda * a * (1 - o)).sum(), rtol=1e-10)
    # dQ/dlog s_x = -xs^2/vx^2 * 2 (f sx/z)^2 ; da/dQ = -a/2
    dQx = -(xs[None, :] ** 2) / vx ** 2 * 2 * (cam.fx * sx / z) ** 2
    dQy = -(ys[:, None] ** 2) / vy ** 2 * 2 * (cam.fy * sy / z) ** 2
    np.testing.assert_allclose(grad[3, 0], (dLda * (-a / 2) * dQx).sum(), rtol=1e-9)
    np.testing.assert_allclose(grad[4, 0], (dLda * (-a / 2) * dQy).sum(), rtol=1e-9)
    assert abs(grad[5, 0]) < 1e-12 * abs(grad[3, 0])  # z-axis scale does not reach the image


def test_two_gaussian_ordering_and_ties():
    """P2: C = a1 c1 + a2 (1 - a1) c2 at the principal point; swapping depths swaps roles;
    equal depths composite the lower index first."""
    cam = Camera(16, 16, 40.0, 40.0, 8.5, 8.5)  # pixel (8, 8) centre sits on the axis
    c1, c2 = (1.0, 0.0, 0.0), (0.0, 0.0, 1.0)
    l1, l2 = 0.4, -0.2
    o1, o2 = 1 / (1 + np.exp(-l1)), 1 / (1 + np.exp(-l2))
    pix = [8 * 16 + 8]
    for z1, z2, first in ((1.0, 2.0, 1), (2.0, 1.0, 2), (1.5, 1.5, 1)):
        p = stack(one_gaussian((0, 0, z1), [np.log(0.05)] * 3, logit=l1, rgb=c1),
                  one_gaussian((0, 0, z2), [np.log(0.05)] * 3, logit=l2, rgb=c2))
        out = oracle.render_fwd(p, cam, O, mode=1, pix=pix)
        if first == 1:
            expect = o1 * np.array(c1) + o2 * (1 - o1) * np.array(c2)
        else:
            expect = o2 * np.array(c2) + o1 * (1 - o2) * np.array(c1)
        np.testing.assert_allclose(out["rgb"][:, 0], expect, rtol=1e-13)


def test_order_takes_the_binary32_depth():
    """The blending order is decided on the depth rounded to binary32 (the precision of the
    rasterizer's sort key), ties in index order: depths 2 + 2^-30 and 2 round to the same binary32
    value, so index 0 (the deeper one in FP64) blends first; 2 + 2^-20 is four binary32 steps
    above 2, so index 1 (at 2) blends first. The blended depth value stays FP64."""
    cam = Camera(16, 16, 40.0, 40.0, 8.5, 8.5)
    c1, c2 = (1.0, 0.0, 0.0), (0.0, 0.0, 1.0)
    l1, l2 = 0.4, -0.2
    o1, o2 = 1 / (1 + np.exp(-l1)), 1 / (1 + np.exp(-l2))
    pix = [8 * 16 + 8]
    for dz, first in ((2.0 ** -30, 1), (2.0 ** -20, 2)):
        z1 = 2.0 + dz
        p = stack(one_gaussian((0, 0, z1), [np.log(0.05)] * 3, logit=l1, rgb=c1),
                  one_gaussian((0, 0, 2.0), [np.log(0.05)] * 3, logit=l2, rgb=c2))
        out = oracle.render_fwd(p, cam, O, mode=1, pix=pix, amb_rel=1e-5)
        if first == 1:
            w1, w2 = o1, o2 * (1 - o1)
        else:
            w1, w2 = o1 * (1 - o2), o2
        np.testing.assert_allclose(out["rgb"][:, 0], w1 * np.array(c1) + w2 * np.array(c2), rtol=1e-13)
        np.testing.assert_allclose(out["depth"][0], w1 * z1 + w2 * 2.0, rtol=1e-15)
        assert bool(out["amb_tie"][0]) == (first == 1) and not out["amb"][0]


def test_termination_semantics():
    """P3: identical alpha = 0.5 contributors: 2^-14 < 1e-4 <= 2^-13, so 13 composite and the
    14th is dropped (not composited) when the pixel stops."""
    cam = Camera(16, 16, 40.0, 40.0, 8.5, 8.5)
    gs = [one_gaussian((0, 0, 1.0 + 0.1 * k), [np.log(0.05)] * 3, logit=0.0, rgb=(k / 20, 0.5, 1 - k / 20))
          for k in range(20)]
    p = stack(*gs)
    out = oracle.render_fwd(p, cam, O, mode=1, pix=[8 * 16 + 8])
    assert out["n_contrib"][0] == 13
    assert out["T_final"][0] == 2.0 ** -13
    expect = sum(0.5 * 2.0 ** -k * p[11:14, k] for k in range(13))
    np.testing.assert_allclose(out["rgb"][:, 0], expect, rtol=1e-14)


@pytest.mark.parametrize("mode", [0, 1])
def test_weights_sum_to_one(mode):
    """P4: sum_i w_i + T_final = 1 per pixel, and alpha = 1 - T_final."""
    p = synth.scene_small(0)
    cam = synth.camera_small()
    out = oracle.render_fwd(p, cam, O, mode=mode)
    np.testing.assert_allclose(out["alpha"] + out["T_final"], 1.0, atol=1e-12)
    assert out["n_contrib"].max() > 10


def test_mirror_symmetry():
    """P5: mirroring the scene in x (mu_x -> -mu_x, q -> (w, x, -y, -z)) mirrors the image
    when the principal point is the image centre."""
    p = synth.scene_small(1).astype(np.float64)
    cam = synth.camera_small()
    m = p.copy()
    m[0] = -m[0]
    m[8] = -m[8]
    m[9] = -m[9]
    a = oracle.render_fwd(p, cam, O, mode=0)
    b = oracle.render_fwd(m, cam, O, mode=0)
    np.testing.assert_allclose(b["rgb"], a["rgb"][:, :, ::-1], atol=1e-12)
    np.testing.assert_allclose(b["depth"], a["depth"][:, ::-1], atol=1e-12)


def quat_mul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def rot_of(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def test_rigid_motion_invariance():
    """Moving the world and the camera by the same rigid motion leaves the image unchanged
    (pins the use of the camera rotation and its transposes)."""
    p = synth.scene_small(2).astype(np.float64)
    cam = synth.camera_small()
    qg = np.array([0.8, 0.3, -0.4, 0.2])
    qg /= np.linalg.norm(qg)
    Rg = rot_of(qg)
    tg = np.array([0.3, -1.2, 0.7])
    m = p.copy()
    m[0:3] = Rg @ p[0:3] + tg[:, None]
    for i in range(p.shape[1]):
        m[6:10, i] = quat_mul(qg, p[6:10, i])
    cam2 = Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy)
    R2 = np.asarray(cam.R, np.float64) @ Rg.T
    t2 = np.asarray(cam.t, np.float64) - R2 @ tg

    class Cam64:  # keep the moved pose in FP64
        pass
    c = Cam64()
    for k in ("width", "height", "fx", "fy", "cx", "cy", "z_near"):
        setattr(c, k, getattr(cam2, k))
    c.R, c.t = R2, t2
    a = oracle.render_fwd(p, cam, O, mode=0)
    b = oracle.render_fwd(m, c, O, mode=0)
    ok = ~(a["amb"] | b["amb"])
    np.testing.assert_allclose(b["rgb"][:, ok], a["rgb"][:, ok], atol=1e-9)
    np.testing.assert_allclose(b["depth"][ok], a["depth"][ok], atol=1e-9)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bucketed_equals_brute_force(seed):
    """P7: the tile-bucketed pre-cull gives exactly the brute-force result (50 gaussians)."""
    cam = synth.camera_small()
    p = synth.frustum_scene(seed + 10, 50, cam, 1.0, 5.0).astype(np.float64)
    a = oracle.render_fwd(p, cam, O, mode=0)
    b = oracle.render_fwd(p, cam, O, mode=1)
    for k in ("rgb", "depth", "alpha", "T_final"):
        np.testing.assert_array_equal(a[k], b[k])
    np.testing.assert_array_equal(a["n_contrib"], b["n_contrib"])


def fd_scene(seed, n):
    g = synth.rng(seed)
    cam = Camera(24, 20, 30.0, 32.0, 12.0, 10.0)
    p = np.zeros((14, n))
    p[2] = g.uniform(1.0, 2.0, n)
    p[0] = g.uniform(-0.4, 0.4, n) * p[2]
    p[1] = g.uniform(-0.3, 0.3, n) * p[2]
    p[3:6] = g.normal(-2.2, 0.3, (3, n))
    q = g.normal(size=(4, n))
    p[6:10] = q / np.linalg.norm(q, axis=0) * g.uniform(0.5, 2.0, n)  # not unit: normalisation path
    p[10] = g.normal(0.5, 1.0, n)
    p[11:14] = g.uniform(0, 1, (3, n))
    return p, cam


def posed(cam):
    qg = np.array([0.95, 0.1, -0.2, 0.15])
    R = rot_of(qg)
    c = Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy)

    class Cam64:
        pass
    o = Cam64()
    for k in ("width", "height", "fx", "fy", "cx", "cy", "z_near"):
        setattr(o, k, getattr(c, k))
    # world -> camera with rotation R and a translation; the scene is moved to stay in view
    o.R, o.t = R, np.array([0.05, -0.02, 0.1])
    return o, R


@pytest.mark.parametrize("seed,n,use_pose,lowpass,bg", [
    (0, 1, False, 0.3, (0, 0, 0)),
    (1, 3, False, 0.0, (0.2, 0.4, 0.1)),
    (2, 5, True, 0.3, (0, 0, 0)),
    (3, 4, True, 0.3, (0.5, 0.5, 0.5)),
])
def test_backward_matches_finite_differences(seed, n, use_pose, lowpass, bg):
    """P8: central differences (h = 1e-6, FP64) of L = sum g * out on tiny scenes."""
    p, cam = fd_scene(seed, n)
    if use_pose:
        cam, R = posed(cam)
        p[0:3] = R.T @ (p[0:3] - cam.t[:, None])  # keep gaussians in front of the camera
    opts = oracle.RenderOpts(lowpass=lowpass, bg=bg, bg_depth=0.3 if any(bg) else 0.0)
    g = synth.rng(100 + seed)
    P = cam.width * cam.height
    gr = g.normal(size=(3, P))
    gd = g.normal(size=P)
    ga = g.normal(size=P)
    amb = oracle.render_fwd(p, cam, opts, mode=1, amb_rel=1e-3)["amb"].ravel()
    gr[:, amb] = 0
    gd[amb] = 0
    ga[amb] = 0

    def L(pp):
        o = oracle.render_fwd(pp, cam, opts, mode=1, amb_rel=0)
        return (gr * o["rgb"].reshape(3, P)).sum() + (gd * o["depth"].ravel()).sum() + (
            ga * o["alpha"].ravel()).sum()

    grad, _ = oracle.render_bwd(p, cam, gr, gd, ga, opts, mode=1)
    h = 1e-6
    fd = np.zeros_like(p)
    for r in range(14):
        for i in range(n):
            pp = p.copy(); pp[r, i] += h
            pm = p.copy(); pm[r, i] -= h
            fd[r, i] = (L(pp) - L(pm)) / (2 * h)
    scale = np.abs(fd).max()
    assert scale > 1e-3
    np.testing.assert_allclose(grad, fd, atol=2e-6 * scale, rtol=1e-5)


def test_backward_bucketed_equals_brute():
    p = synth.frustum_scene(7, 60, synth.camera_small(), 1.0, 5.0).astype(np.float64)
    cam = synth.camera_small()
    g = synth.rng(8)
    gr = g.normal(size=(3, cam.n_pixels)); gd = g.normal(size=cam.n_pixels)
    a, a2 = oracle.render_bwd(p, cam, gr, gd, None, O, mode=0)
    b, b2 = oracle.render_bwd(p, cam, gr, gd, None, O, mode=1)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(a2, b2, rtol=1e-12, atol=1e-14)


def test_pixel_list_matches_full_image():
    p = synth.scene_small(4).astype(np.float64)
    cam = synth.camera_small()
    full = oracle.render_fwd(p, cam, O, mode=0)
    pix = np.array([0, 5, 700, 1500, 3071])
    for mode in (0, 1):
        part = oracle.render_fwd(p, cam, O, mode=mode, pix=pix)
        np.testing.assert_allclose(part["rgb"], full["rgb"].reshape(3, -1)[:, pix], rtol=1e-13, atol=1e-15)
        np.testing.assert_array_equal(part["n_contrib"], full["n_contrib"].ravel()[pix])


def test_culling_and_invalid_inputs():
    cam = Camera(16, 16, 40.0, 40.0, 8.0, 8.0)
    behind = one_gaussian((0, 0, 0.1), [np.log(0.05)] * 3)   # z <= z_near
    zero_q = one_gaussian((0, 0, 1.0), [np.log(0.05)] * 3, q=(0, 0, 0, 0))
    nan_mu = one_gaussian((np.nan, 0, 1.0), [np.log(0.05)] * 3)
    p = stack(behind, zero_q, nan_mu)
    out = oracle.render_fwd(p, cam, O, mode=1)
    assert out["alpha"].max() == 0
    assert (out["T_final"] == 1).all()
    proj = oracle.project(p, cam, O)
    assert (proj[:, 0] == 0).all()
    with pytest.raises(ValueError):
        oracle.render_fwd(p, Camera(0, 16, 40.0, 40.0, 8.0, 8.0), O)


def test_duplicate_count_matches_buckets():
    """K under 16x16 binning equals the sum of the per-tile candidate lists."""
    p = synth.scene_small(5).astype(np.float64)
    cam = synth.camera_small()
    K = oracle.count_duplicates(p, cam, 16, 16, O)
    proj = oracle.project(p, cam, O)
    k2 = 0
    for row in proj:
        if not row[0]:
            continue
        rx, ry = 3 * np.sqrt(row[4]), 3 * np.sqrt(row[6])
        x0, x1 = np.ceil(row[10] - rx - 0.5), np.floor(row[10] + rx - 0.5)
        y0, y1 = np.ceil(row[11] - ry - 0.5), np.floor(row[11] + ry - 0.5)
        x0, x1 = max(x0, 0), min(x1, cam.width - 1)
        y0, y1 = max(y0, 0), min(y1, cam.height - 1)
        if x0 > x1 or y0 > y1:
            continue
        k2 += (int(x1) // 16 - int(x0) // 16 + 1) * (int(y1) // 16 - int(y0) // 16 + 1)
    assert K == k2 and K > 0


def test_tile_counts_invariants_and_limits():
    """Work counts of the 16x16-tile formulation: K_c <= L_b <= L_f <= K (a contributing pair lies
    before the last blended entry, which lies before the last examined one); with no termination
    (T_min = 0) every pixel examines the whole list, L_f = K; with nothing above alpha_min nothing
    blends, K_c = L_b = 0 and L_f = K; one small gaussian inside one tile gives 1 everywhere."""
    cam = Camera(64, 48, 60.0, 60.0, 32.0, 24.0)
    import synth
    p = synth.scene_small(4).astype(np.float64)
    c = oracle.tile_counts(p, cam)
    K = oracle.count_duplicates(p, cam, 16, 16)
    assert c["K"] == K
    assert 0 < c["K_c"] <= c["L_b"] <= c["L_f"] <= K
    c0 = oracle.tile_counts(p, cam, O.__class__(T_min=0.0))
    assert c0["L_f"] == K
    q = p.copy()
    q[10] = -12.0  # opacity 6e-6 < 1/255
    cn = oracle.tile_counts(q, cam)
    assert cn["K_c"] == 0 and cn["L_b"] == 0 and cn["L_f"] == K
    one = one_gaussian(((24.5 - 32.0) * 2 / 60.0, (8.5 - 24.0) * 2 / 60.0, 2.0), [np.log(0.02)] * 3, logit=2.0)
    c1 = oracle.tile_counts(stack(one), cam)
    assert c1 == {"K_c": 1, "L_f": 1, "L_b": 1, "K": 1}
