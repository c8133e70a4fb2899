"""Pins of the FP64 oracle's Fourier seeding (Eq. 2-8, the triangle threshold, Eq. 11)."""
import numpy as np
import pytest

import oracle
import synth
from synth import Camera

W, H = 64, 48


def grey(Y):
    """RGB planes whose BT.601 luma is Y (R = G = B = Y)."""
    return np.repeat(np.asarray(Y, np.float32)[None], 3, axis=0)


def luma(rgb):
    r = rgb.astype(np.float64)
    return 0.299 * r[0] + 0.587 * r[1] + 0.114 * r[2]


def hp_filter(W, H, D0):
    u = np.arange(W)
    v = np.arange(H)
    ub = np.where(u < W / 2, u, u - W)
    vb = np.where(v < H / 2, v, v - H)
    D2 = ub[None, :] ** 2 + vb[:, None] ** 2
    return 1 - np.exp(-D2 / (2 * D0 ** 2))


@pytest.mark.parametrize("D0", [3.0, 10.0, 30.0])
def test_highpass_matches_numpy_fft(D0):
    """P9: the naive separable DFT pipeline equals numpy's FFT (a library routine) with the
    Gaussian high-pass of Eq. 5 centred on DC."""
    rgb, _ = synth.rgbd_frame(0, W, H, n_rect=6)
    E, hist, t, margin = oracle.highpass(rgb, D0)
    ref = np.abs(np.fft.ifft2(np.fft.fft2(luma(rgb)) * hp_filter(W, H, D0)))
    np.testing.assert_allclose(E, ref, rtol=1e-9, atol=1e-12 * ref.max())
    q = np.minimum(np.floor(255 * (ref / ref.max())), 255).astype(int)
    np.testing.assert_array_equal(hist, np.bincount(q.ravel(), minlength=256))
    assert hist.sum() == W * H


def test_highpass_of_a_cosine():
    """P10: a single cosine is an eigenfunction of the filter: I_h = H(k, l) * the cosine."""
    k, l, D0 = 5, 3, 4.0
    x = np.arange(W)[None, :]
    y = np.arange(H)[:, None]
    Y = 0.5 + 0.25 * np.cos(2 * np.pi * (k * x / W + l * y / H))
    rgb = grey(Y)
    E, _, _, _ = oracle.highpass(rgb, D0)
    Hkl = 1 - np.exp(-(k * k + l * l) / (2 * D0 * D0))
    Y32 = luma(rgb) - 0.5
    np.testing.assert_allclose(E, np.abs(Hkl * Y32), atol=2e-7)


def test_tiny_cutoff_removes_only_dc():
    """D0 -> 0 leaves H = 1 except at DC, so I_h = I - mean(I)."""
    rgb, _ = synth.rgbd_frame(1, W, H, n_rect=6)
    E, _, _, _ = oracle.highpass(rgb, 1e-3)
    Y = luma(rgb)
    np.testing.assert_allclose(E, np.abs(Y - Y.mean()), atol=1e-10)


def test_constant_frame_has_no_high_frequency():
    """P10: a constant frame has E == 0, so M_h is empty and only the stride-n lattice seeds."""
    rgb = grey(np.full((H, W), 0.4))
    depth = np.full((H, W), 2.0, np.float32)
    cam = Camera(W, H, 60.0, 60.0, W / 2, H / 2)
    E, hist, t, _ = oracle.highpass(rgb, 30.0)
    assert np.abs(E).max() < 1e-12 and t == -1
    s = oracle.seed(rgb, depth, cam, oracle.SeedOpts(D0=30.0))
    assert not s["is_high"].any()
    assert s["n"] == -(-W // 8) * -(-H // 8)
    assert (s["tile_count"] == 4).all()


def test_lattice_counts():
    """P12: with m = n the lattice is the same everywhere: ceil(W/m) ceil(H/m) seeds, m^-2 of a tile."""
    rgb = grey(np.full((H, W), 0.4))
    depth = np.full((H, W), 2.0, np.float32)
    cam = Camera(W, H, 60.0, 60.0, W / 2, H / 2)
    s = oracle.seed(rgb, depth, cam, oracle.SeedOpts(m=2, n=2))
    assert s["n"] == (W // 2) * (H // 2)
    assert (s["tile_count"] == 64).all()
    # ragged size: 70 x 50 -> ceil(70/4) * ceil(50/4)
    rgb2 = grey(np.full((50, 70), 0.4))
    d2 = np.full((50, 70), 2.0, np.float32)
    s2 = oracle.seed(rgb2, d2, Camera(70, 50, 60.0, 60.0, 35.0, 25.0), oracle.SeedOpts(m=4, n=4))
    assert s2["n"] == 18 * 13
    assert s2["tile_count"].sum() == s2["n"]


def test_invalid_depth_is_not_seeded():
    rgb = grey(np.full((H, W), 0.4))
    depth = np.full((H, W), 2.0, np.float32)
    depth[:, :W // 2] = 0.0            # below depth_min
    depth[0, W // 2 + 8] = np.nan     # not finite
    depth[8, W // 2 + 8] = 50.0       # beyond depth_max
    cam = Camera(W, H, 60.0, 60.0, W / 2, H / 2)
    s = oracle.seed(rgb, depth, cam, oracle.SeedOpts())
    xs = s["pixel"] % W
    assert (xs >= W // 2).all()
    assert s["n"] == (W // 2 // 8) * (H // 8) - 2


def test_high_frequency_patch_gets_dense_small_seeds():
    """A textured patch on a flat frame lands in M_h: stride-m lattice there, stride-n elsewhere,
    and Eq. 11 radii alpha_h d/f vs alpha_l d/f."""
    Y = np.full((H, W), 0.5)
    g = synth.rng(4)
    Y[16:32, 16:48] += 0.3 * g.uniform(-1, 1, (16, 32))
    rgb = grey(Y)
    depth = np.full((H, W), 2.0, np.float32)
    cam = Camera(W, H, 60.0, 60.0, W / 2, H / 2)
    o = oracle.SeedOpts(D0=8.0)
    s = oracle.seed(rgb, depth, cam, o)
    x, y = s["pixel"] % W, s["pixel"] // W
    hi = s["is_high"]
    assert hi.sum() > 50 and (~hi).sum() > 10
    assert ((x[hi] % 2 == 0) & (y[hi] % 2 == 0)).all()
    assert ((x[~hi] % 8 == 0) & (y[~hi] % 8 == 0)).all()
    inside = (x >= 14) & (x < 50) & (y >= 14) & (y < 34)
    assert inside[hi].mean() > 0.9
    np.testing.assert_array_equal(s["radius"][hi], np.float32(np.float32(1.0) * np.float32(2.0)) / np.float32(60.0))
    np.testing.assert_array_equal(s["radius"][~hi], np.float32(np.float32(4.0) * np.float32(2.0)) / np.float32(60.0))
    assert np.all(np.diff(s["pixel"]) > 0)  # row-major emission


def tri_right(h):
    return oracle.triangle(np.asarray(h, np.int64))


def test_triangle_threshold_hand_cases():
    """P11: hand-computed answers. (a) a linear ramp with one dip: the dip. (b) a two-segment
    ramp: its knee. Mirroring the histogram mirrors the threshold."""
    h = np.zeros(256, np.int64)
    h[:51] = 1000 - 10 * np.arange(51)
    h[20] = 100
    assert tri_right(h) == 20
    assert tri_right(h[::-1].copy()) == 255 - 20
    h = np.zeros(256, np.int64)
    h[:11] = 1000 - 90 * np.arange(11)
    h[10:51] = 100 - 2 * (np.arange(10, 51) - 10)
    assert tri_right(h) == 10
    assert tri_right(h[::-1].copy()) == 255 - 10
    # peak away from the edges, longer right tail, offset start
    h = np.zeros(256, np.int64)
    h[5:10] = [10, 40, 200, 500, 800]
    h[10:40] = np.maximum(900 - 60 * np.arange(30), 30)
    # below(i) = 29 (900 - h_i) - 870 (i - 10): bins 24 and 25 tie at 12180; the nearer one wins
    d = [29 * (900 - h[i]) - 870 * (i - 10) for i in range(11, 39)]
    assert d[24 - 11] == d[25 - 11] == max(d) == 12180
    assert tri_right(h) == 24
    assert tri_right(h[::-1].copy()) == 255 - 24


def test_seed_floats_are_binary32():
    """P13/P14: seed floats equal numpy binary32 arithmetic (IEEE single, no FMA) for the same
    operation sequence; re-projecting a seed lands on its pixel centre; its projected size is
    alpha pixels (Eq. 11)."""
    rgb, depth = synth.rgbd_frame(2, W, H, n_rect=8)
    qg = np.array([0.9, 0.2, -0.3, 0.1]); qg /= np.linalg.norm(qg)
    w, x, y, z = qg
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                  [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                  [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    cam = Camera(W, H, 61.0, 59.0, W / 2, H / 2, R=R, t=[0.1, -0.2, 0.3])
    o = oracle.SeedOpts(D0=8.0)
    s = oracle.seed(rgb, depth, cam, o)
    f = np.float32
    px = s["pixel"]
    xs, ys = (px % W).astype(f), (px // W).astype(f)
    d = depth.ravel()[px]
    X = ((xs + f(0.5)) - f(cam.cx)) * d / f(cam.fx)
    Y = ((ys + f(0.5)) - f(cam.cy)) * d / f(cam.fy)
    Rf, tf = cam.R.astype(f), cam.t.astype(f)
    u = [X - tf[0], Y - tf[1], d - tf[2]]
    for r in range(3):
        mu = (Rf[0, r] * u[0] + Rf[1, r] * u[1]) + Rf[2, r] * u[2]
        np.testing.assert_array_equal(s["mean"][r], mu)
    a = np.where(s["is_high"], f(o.alpha_h), f(o.alpha_l))
    np.testing.assert_array_equal(s["radius"], (a * d) / f(cam.fx))
    np.testing.assert_array_equal(s["rgb"], rgb.reshape(3, -1)[:, px])
    # re-projection through the render oracle's projection
    params = np.zeros((14, len(px)))
    params[0:3] = s["mean"]
    params[3:6] = np.log(s["radius"].astype(np.float64))[None]
    params[6] = 1.0
    pr = oracle.project(params, cam, oracle.RenderOpts(lowpass=0.3))
    np.testing.assert_allclose(pr[:, 10], px % W + 0.5, atol=2e-4)
    np.testing.assert_allclose(pr[:, 11], px // W + 0.5, atol=2e-4)
    # isotropic gaussian of radius r = alpha d / fx at camera point (X, Y, d): the EWA screen
    # variance along x is (fx r / d)^2 (1 + (X/d)^2) + lowpass = alpha^2 (1 + (X/d)^2) + lowpass
    xd = (px % W + 0.5 - cam.cx) / cam.fx
    np.testing.assert_allclose(pr[:, 4], a.astype(np.float64) ** 2 * (1 + xd ** 2) + 0.3, rtol=1e-4)


def test_margin_reports_quantisation_distance():
    rgb, _ = synth.rgbd_frame(3, W, H, n_rect=6)
    E, hist, t, margin = oracle.highpass(rgb, 30.0)
    r = 255 * (E / E.max())
    m = np.abs(r - np.rint(r))
    m[np.rint(r) < 1] = np.inf
    m[np.unravel_index(np.argmax(E), E.shape)] = np.inf
    assert margin == pytest.approx(m.min(), abs=1e-12)


def test_full_size_frame_seeds():
    """A 640x480 synthetic frame (the TUM-sized workload): seeds are plentiful, both classes occur,
    counts per 16x16 tile add up."""
    rgb, depth = synth.rgbd_frame(0)
    cam = synth.camera_tum()
    s = oracle.seed(rgb, depth, cam, oracle.SeedOpts())
    assert 5_000 < s["n"] < 80_000
    assert s["is_high"].any() and (~s["is_high"]).any()
    assert s["tile_count"].shape == (30, 40) and s["tile_count"].sum() == s["n"]


def test_seed_set_from_numpy_mask():
    """The seeded set is exactly: stride-m lattice points with q > t, stride-n lattice points with
    q <= t, valid depth; with q from numpy's FFT and t the triangle threshold of its histogram."""
    rgb, depth = synth.rgbd_frame(6, W, H, n_rect=8)
    cam = Camera(W, H, 60.0, 60.0, W / 2, H / 2)
    o = oracle.SeedOpts(D0=10.0)
    s = oracle.seed(rgb, depth, cam, o)
    assert s["margin"] > 1e-9
    E = np.abs(np.fft.ifft2(np.fft.fft2(luma(rgb)) * hp_filter(W, H, o.D0)))
    q = np.minimum(np.floor(255 * (E / E.max())), 255).astype(int)
    t = oracle.triangle(np.bincount(q.ravel(), minlength=256))
    assert t == s["threshold"]
    hi = q > t
    yy, xx = np.mgrid[0:H, 0:W]
    lat = np.where(hi, (xx % o.m == 0) & (yy % o.m == 0), (xx % o.n == 0) & (yy % o.n == 0))
    ok = (depth >= o.depth_min) & (depth <= o.depth_max)
    expect = np.flatnonzero(lat & ok)
    np.testing.assert_array_equal(s["pixel"], expect)
    np.testing.assert_array_equal(s["is_high"], hi.ravel()[expect])
    assert 0 < s["is_high"].sum() < len(expect)


# ------------------------------------------------ missing-region check (Eq. 9, 10)

def missing_frame():
    rgb, depth = synth.rgbd_frame(11, W, H, n_rect=8)
    depth[:4, :] = 0.0  # a band without depth measurements
    return rgb, depth, Camera(W, H, 60.0, 60.0, W / 2, H / 2)


def rendered_like(rgb, depth, alpha=1.0):
    """A map that explains the frame exactly: opacity `alpha`, the frame's own colour and depth."""
    return oracle.MissingCheck(np.full(depth.shape, alpha, np.float32), depth.copy(), rgb.copy())


def test_missing_check_first_frame_is_the_identity():
    """No map yet, or a map whose rendered opacity is 0 everywhere (M_i is the whole frame): the
    seeds are those of the plain seeding, and M_m is every pixel."""
    rgb, depth, cam = missing_frame()
    plain = oracle.seed(rgb, depth, cam)
    assert plain["missing"].all()
    empty = oracle.seed(rgb, depth, cam, miss=oracle.MissingCheck(np.zeros_like(depth), np.zeros_like(depth),
                                                                   np.zeros_like(rgb)))
    assert empty["missing"].all()
    for k in ("pixel", "is_high", "mean", "radius", "rgb", "tile_count"):
        np.testing.assert_array_equal(empty[k], plain[k], err_msg=k)


def test_missing_check_fully_explained_frame_seeds_nothing():
    rgb, depth, cam = missing_frame()
    s = oracle.seed(rgb, depth, cam, miss=rendered_like(rgb, depth))
    assert s["n"] == 0 and not s["missing"].any() and s["tile_count"].sum() == 0


def test_missing_check_compares_the_surface_over_its_opacity():
    """A translucent map (opacity 0.75 everywhere, above tau_alpha) whose depth and colour
    renderings are 0.75 times the frame's explains the frame: nothing is missing. The same planes
    taken as surface values (opacity 1) would put every pixel in M_d."""
    rgb, depth, cam = missing_frame()
    a = np.float32(0.75)
    m = oracle.MissingCheck(np.full(depth.shape, a, np.float32), depth * a, rgb * a)
    s = oracle.seed(rgb, depth, cam, miss=m)
    # 0.75 x rounds; the quotient is within one binary32 step of the frame's value
    assert not s["missing"].any() and s["n"] == 0
    opaque = oracle.seed(rgb, depth, cam, miss=oracle.MissingCheck(np.ones_like(depth), depth * a, rgb * a))
    valid = (depth >= 0.1) & (depth <= 10.0)
    assert opaque["missing"][valid].all()


def test_missing_check_masks_and_the_seeds_they_keep():
    """Three disjoint rectangles, each missing for one reason: low rendered opacity (M_i), a
    rendered depth 0.3 m off the frame's (M_d), a rendered colour 0.2 off per channel (M_c). M_m is
    exactly their union (Eq. 9), and the seeds are exactly the plain seeds inside it (Eq. 10: both
    frequency masks restricted to M_m, the lattices and radii unchanged)."""
    rgb, depth, cam = missing_frame()
    plain = oracle.seed(rgb, depth, cam)
    m = rendered_like(rgb, depth)
    A, B, Cr = (slice(8, 20), slice(5, 30)), (slice(24, 40), slice(10, 50)), (slice(2, 12), slice(40, 70))
    m.alpha[A] = 0.2
    m.depth[B] += 0.3
    m.rgb[(slice(None),) + Cr] = np.clip(m.rgb[(slice(None),) + Cr] + 0.2, 0.0, 1.2)
    s = oracle.seed(rgb, depth, cam, miss=m)
    expect_mask = np.zeros(depth.shape, bool)
    expect_mask[A] = True
    valid = (depth >= 0.1) & (depth <= 10.0)
    expect_mask[B] |= valid[B]  # the depth mask needs a depth measurement
    expect_mask[Cr] = True
    np.testing.assert_array_equal(s["missing"], expect_mask)
    keep = expect_mask.ravel()[plain["pixel"]]
    assert keep.sum() > 20 and (~keep).sum() > 50
    np.testing.assert_array_equal(s["pixel"], plain["pixel"][keep])
    np.testing.assert_array_equal(s["is_high"], plain["is_high"][keep])
    np.testing.assert_array_equal(s["mean"], plain["mean"][:, keep])
    np.testing.assert_array_equal(s["radius"], plain["radius"][keep])
    assert s["tile_count"].sum() == s["n"]


def test_missing_check_thresholds_are_strict():
    """An opacity equal to tau_alpha is not missing; a depth difference equal to tau_depth is not;
    a colour difference summing to exactly tau_rgb is not (values exact in binary32); just past each
    threshold is; a huge depth difference at a pixel without a depth measurement is not. Depth and
    colour are compared as the surface the map shows (rendered value over rendered opacity: at
    opacity 0.5 a render of half the frame's depth and colour matches the frame)."""
    rgb, depth, cam = missing_frame()
    rgb = np.full_like(rgb, 0.5)
    depth = np.where(depth > 0, 2.0, 0.0).astype(np.float32)
    m = rendered_like(rgb, depth)
    m.alpha[10, 10], m.alpha[10, 11] = 0.5, np.nextafter(np.float32(0.5), np.float32(0))
    m.depth[10, 10:12] *= m.alpha[10, 10:12]  # the surface the map shows: depth and colour / opacity
    m.rgb[:, 10, 10] *= 0.5
    m.depth[12, 10], m.depth[12, 11] = 2.125, np.nextafter(np.float32(2.125), np.float32(3))
    m.rgb[:, 14, 10] = 0.5 + np.float32(0.125)           # (0.125 + 0.125) + 0.125 = 0.375 exactly
    m.rgb[:, 14, 11] = [0.625, 0.625, np.nextafter(np.float32(0.625), np.float32(1))]
    m.depth[1, 20] = 50.0                                 # row 1 has no depth measurement
    s = oracle.seed(rgb, depth, cam, miss=oracle.MissingCheck(m.alpha, m.depth, m.rgb, 0.5, 0.125, 0.375))
    mm = s["missing"]
    assert not mm[10, 10] and mm[10, 11]
    assert not mm[12, 10] and mm[12, 11]
    assert not mm[14, 10] and mm[14, 11]
    assert not mm[1, 20]
    assert mm.sum() == 3
