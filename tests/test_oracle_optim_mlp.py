"""Pins of the oracle's L1 loss (Eq. 16, L1 terms), Adam, and the learned-prior MLP."""
import numpy as np
import pytest

import oracle
import synth


def test_loss_l1_closed_form():
    g = synth.rng(0)
    P = 50
    rgb, rgbt = g.uniform(size=(3, P)), g.uniform(size=(3, P))
    d, dt = g.uniform(1, 3, P), g.uniform(1, 3, P)
    dt[:10] = 0.0  # invalid targets are ignored
    rgbt[0, 0] = rgb[0, 0]  # sign(0) = 0
    L, psnr, gr, gd = oracle.loss_l1(rgb, d, rgbt, dt, 1.0, 0.1)
    exp = np.abs(rgb - rgbt).sum() / (3 * P) + 0.1 * np.abs(d - dt)[10:].sum() / 40
    assert L == pytest.approx(exp, rel=1e-14)
    assert psnr == pytest.approx(10 * np.log10(1 / np.mean((rgb - rgbt) ** 2)), rel=1e-14)
    assert gr[0, 0] == 0 and (gd[:10] == 0).all()
    # gradient = finite difference of a piecewise-linear function away from kinks
    np.testing.assert_allclose(gr, np.sign(rgb - rgbt) / (3 * P))
    np.testing.assert_allclose(gd[10:], 0.1 * np.sign(d - dt)[10:] / 40)


def test_adam_first_step_closed_form():
    """P15: the first Adam step is -lr g/(|g| + eps)."""
    g = synth.rng(1)
    n = 7
    p = g.normal(size=(14, n))
    grad = g.normal(size=(14, n)) * 10.0 ** g.integers(-9, 0, size=(14, n))
    lr = np.array([1e-3, 5e-3, 1e-3, 5e-2, 2.5e-3])
    p1, m1, v1 = oracle.adam(p, np.zeros_like(p), np.zeros_like(p), grad, 0, lr)
    rows = np.array([0, 0, 0, 1, 1, 1, 2, 2, 2, 2, 3, 4, 4, 4])
    np.testing.assert_allclose(p1, p - lr[rows][:, None] * grad / (np.abs(grad) + 1e-15), rtol=1e-12)
    np.testing.assert_allclose(m1, 0.1 * grad)
    np.testing.assert_allclose(v1, 0.001 * grad ** 2)


def test_adam_second_step():
    g = synth.rng(2)
    p = g.normal(size=(14, 3)); g1 = g.normal(size=(14, 3)); g2 = g.normal(size=(14, 3))
    lr = np.full(5, 0.01)
    p1, m1, v1 = oracle.adam(p, 0 * p, 0 * p, g1, 0, lr)
    p2, m2, v2 = oracle.adam(p1, m1, v1, g2, 1, lr)
    m = 0.9 * 0.1 * g1 + 0.1 * g2
    v = 0.999 * 0.001 * g1 ** 2 + 0.001 * g2 ** 2
    np.testing.assert_allclose(p2, p1 - 0.01 * (m / 0.19) / (np.sqrt(v / (1 - 0.999 ** 2)) + 1e-15), rtol=1e-12)


def unpack(w):
    i = 0
    out = []
    for shape in ((256, 260), (256,), (256, 256), (256,), (4, 256), (4,)):
        k = int(np.prod(shape))
        out.append(w[i:i + k].reshape(shape))
        i += k
    assert i == oracle.MLP_PARAMS
    return out


def test_mlp_zero_weights_give_bias():
    w = np.zeros(oracle.MLP_PARAMS)
    W1, b1, W2, b2, W3, b3 = unpack(w)
    b3[:] = [0.5, -1.0, 2.0, 3.25]
    x = synth.rng(3).normal(size=(5, 260))
    np.testing.assert_array_equal(oracle.mlp_fwd(x, w, bf16=False), np.tile(b3, (5, 1)))


def test_mlp_linear_regime_matches_matmul():
    """For large positive pre-activations GELU(a) = a, so the network is the affine chain
    W3 (W2 (W1 x + b1) + b2) + b3 (pins operand order and orientation)."""
    g = synth.rng(4)
    w = np.zeros(oracle.MLP_PARAMS)
    W1, b1, W2, b2, W3, b3 = unpack(w)
    W1[:] = g.uniform(0, 0.1, W1.shape); b1[:] = 40.0
    W2[:] = g.uniform(0, 0.01, W2.shape); b2[:] = 40.0
    W3[:] = g.normal(size=W3.shape); b3[:] = g.normal(size=4)
    x = g.uniform(0, 1, (6, 260))
    y = oracle.mlp_fwd(x, w, bf16=False)
    ref = ((x @ W1.T + b1) @ W2.T + b2) @ W3.T + b3
    np.testing.assert_allclose(y, ref, rtol=1e-12)


def test_mlp_bf16_round_to_nearest_even():
    """Operands are rounded to bfloat16 with ties to even: 64 (1 + 3 2^-8) -> 65, 64 (1 + 2^-8) -> 64."""
    w = np.zeros(oracle.MLP_PARAMS)
    W1, b1, W2, b2, W3, b3 = unpack(w)
    W1[0, 0] = 1.0
    W2[0, 0] = 1.0
    W3[0, 0] = 1.0
    for v, expect in ((64 * (1 + 3 / 256), 65.0), (64 * (1 + 1 / 256), 64.0), (64 * (1 + 1.5 / 256), 64.5)):
        x = np.zeros((1, 260)); x[0, 0] = v
        assert oracle.mlp_fwd(x, w, bf16=True)[0, 0] == expect
        assert oracle.mlp_fwd(x, w, bf16=False)[0, 0] == v


def test_mlp_gelu_zero():
    w = np.zeros(oracle.MLP_PARAMS)
    W1, b1, W2, b2, W3, b3 = unpack(w)
    W3[:] = 1.0
    x = np.zeros((2, 260))
    np.testing.assert_array_equal(oracle.mlp_fwd(x, w, bf16=False), 0.0)


def test_mlp_backward_matches_finite_differences():
    """P16: FP64 central differences of the MSE loss on a sample of weights (bf16 off)."""
    g = synth.rng(5)
    w = np.concatenate([g.normal(0, 0.06, 256 * 260), g.normal(0, 0.1, 256), g.normal(0, 0.06, 256 * 256),
                        g.normal(0, 0.1, 256), g.normal(0, 0.06, 4 * 256), g.normal(0, 0.1, 4)])
    x = g.normal(size=(4, 260))
    t = g.normal(size=(4, 4))
    gw, L = oracle.mlp_bwd(x, w, t, bf16=False)

    def loss(ww):
        return np.mean((oracle.mlp_fwd(x, ww, bf16=False) - t) ** 2)

    assert L == pytest.approx(loss(w), rel=1e-12)
    idx = np.concatenate([g.integers(0, 256 * 260, 12), 256 * 260 + g.integers(0, 256, 4),
                          256 * 261 + g.integers(0, 256 * 256, 12), 256 * 261 + 65536 + g.integers(0, 256, 4),
                          256 * 262 + 65536 + g.integers(0, 1028, 8)])
    h = 1e-6
    for i in idx:
        wp = w.copy(); wp[i] += h
        wm = w.copy(); wm[i] -= h
        fd = (loss(wp) - loss(wm)) / (2 * h)
        assert gw[i] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_tile_features_match_numpy_fft():
    """Tile spectrum features equal log1p |fftshift(fft2(tile luma))|; depth statistics by hand."""
    rgb, depth = synth.rgbd_frame(5, 64, 48, n_rect=6)
    f, nv = oracle.tile_features(rgb, depth, 2, 1)
    r = rgb.astype(np.float64)
    Y = (0.299 * r[0] + 0.587 * r[1] + 0.114 * r[2])[16:32, 32:48]
    ref = np.log1p(np.abs(np.fft.fftshift(np.fft.fft2(Y))))
    np.testing.assert_allclose(f[:256], ref.ravel(), rtol=1e-10, atol=1e-12)
    d = depth[16:32, 32:48].astype(np.float64)
    assert nv == 256
    np.testing.assert_allclose(f[256:], [d.mean(), d.std(), d.min(), d.max()], rtol=1e-10)
