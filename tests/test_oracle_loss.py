"""Pins of the oracle's structural-similarity term and scale regulariser (Sec. III-D, Eq. 15 and
Eq. 16) against facts that do not come from the oracle itself."""
import numpy as np
import pytest

import oracle

C1, C2 = 0.01 ** 2, 0.03 ** 2


def window():
    """The 11x11 gaussian window (sigma 1.5) normalised to sum 1, written from its definition."""
    k = np.arange(-5, 6)
    w = np.exp(-(k[:, None] ** 2 + k[None, :] ** 2) / (2 * 1.5 ** 2))
    return w / w.sum()


def test_ssim_of_an_image_with_itself_is_one_with_zero_gradient():
    x = np.random.default_rng(1).uniform(0, 1, (3, 23, 17))
    s, g, m = oracle.ssim(x, x)
    assert s == pytest.approx(1.0, abs=1e-14)
    assert np.abs(m - 1.0).max() < 1e-13
    assert np.abs(g).max() < 1e-15


def test_ssim_is_symmetric():
    g = np.random.default_rng(2)
    x, y = g.uniform(0, 1, (3, 19, 21)), g.uniform(0, 1, (3, 19, 21))
    assert oracle.ssim(x, y)[0] == pytest.approx(oracle.ssim(y, x)[0], abs=1e-15)


def test_constant_images_give_the_luminance_term_in_the_interior():
    """Away from the border (5 px), two constant images have zero variance and covariance, so the
    index is (2 c1 c2 + C1) / (c1^2 + c2^2 + C1) exactly (the contrast-structure factor is C2/C2)."""
    c1, c2 = 0.3, 0.7
    x = np.full((3, 30, 32), c1)
    y = np.full((3, 30, 32), c2)
    _, _, m = oracle.ssim(x, y)
    want = (2 * c1 * c2 + C1) / (c1 * c1 + c2 * c2 + C1)
    assert np.abs(m[:, 5:-5, 5:-5] - want).max() < 1e-12
    # at a corner a quarter-window of zeros lowers the means: the index differs there
    assert abs(m[0, 0, 0] - want) > 1e-3


def test_ssim_map_matches_moments_from_scipy_correlation():
    """The per-pixel index from window moments computed by scipy's correlation with zero padding
    (an implementation independent of the oracle's loops), at every pixel including the border."""
    ndimage = pytest.importorskip("scipy.ndimage")
    g = np.random.default_rng(3)
    x, y = g.uniform(0, 1, (3, 26, 29)), g.uniform(0, 1, (3, 26, 29))
    w = window()
    corr = lambda a: ndimage.correlate(a, w, mode="constant", cval=0.0)
    want = np.empty_like(x)
    for c in range(3):
        mx, my = corr(x[c]), corr(y[c])
        vx, vy, cxy = corr(x[c] * x[c]) - mx * mx, corr(y[c] * y[c]) - my * my, corr(x[c] * y[c]) - mx * my
        want[c] = (2 * mx * my + C1) * (2 * cxy + C2) / ((mx * mx + my * my + C1) * (vx + vy + C2))
    s, _, m = oracle.ssim(x, y)
    assert np.abs(m - want).max() < 1e-12
    assert s == pytest.approx(want.mean(), abs=1e-14)


def test_ssim_gradient_matches_central_differences():
    """Every pixel of a 9x8 image lies within 5 px of a border, so the zero-padded windows and the
    sum over the pixels whose window holds q are all exercised."""
    g = np.random.default_rng(4)
    x, y = g.uniform(0.1, 0.9, (3, 9, 8)), g.uniform(0.1, 0.9, (3, 9, 8))
    _, grad, _ = oracle.ssim(x, y)
    h = 1e-5
    # the difference quotient's own error (h^2 truncation, rounding of the mean over 216 values)
    # stays below 1e-9 of the largest entry; a missing or mis-weighted term is off by far more
    floor = 1e-9 * np.abs(grad).max()
    for k in g.choice(x.size, 24, replace=False):
        idx = np.unravel_index(k, x.shape)
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (oracle.ssim(xp, y)[0] - oracle.ssim(xm, y)[0]) / (2 * h)
        assert abs(fd - grad[idx]) <= 1e-7 * abs(grad[idx]) + floor, (idx, fd, grad[idx])


def test_scale_regulariser_hand_example():
    """Two gaussians, scales (1, 3, 0.5) and (2, 2, 0.25): 1/2 (|1 - 3| + 0.5 + |2 - 2| + 0.25) =
    1.375; d/d log s = s d/ds: (-1/2, 3/2, 1/4) and (0, 0, 1/8) (the first term's derivative is
    zero where the two in-plane scales are equal)."""
    ls = np.log(np.array([[1.0, 2.0], [3.0, 2.0], [0.5, 0.25]]))
    v, g = oracle.scale_reg(ls)
    assert v == pytest.approx(1.375, abs=1e-15)
    np.testing.assert_allclose(g, [[-0.5, 0.0], [1.5, 0.0], [0.25, 0.125]], atol=1e-15)


def test_scale_regulariser_gradient_matches_central_differences():
    g = np.random.default_rng(5)
    ls = g.normal(-2.0, 0.5, (3, 40))
    _, grad = oracle.scale_reg(ls)
    h = 1e-6
    for k in range(ls.size):
        idx = np.unravel_index(k, ls.shape)
        lp, lm = ls.copy(), ls.copy()
        lp[idx] += h
        lm[idx] -= h
        fd = (oracle.scale_reg(lp)[0] - oracle.scale_reg(lm)[0]) / (2 * h)
        assert abs(fd - grad[idx]) <= 1e-7 * abs(grad[idx]) + 1e-12, (idx, fd, grad[idx])
