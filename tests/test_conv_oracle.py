"""Pins of the corrector's FP64 conv oracle: library cross-check, closed-form
kernels, zero padding, central finite differences of layers and of the whole
network."""
import numpy as np
import pytest
from scipy import ndimage

import oracle


def _rand(shape, rng, s=1.0):
    return rng.normal(size=shape) * s


def test_forward_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    x = _rand((2, 7, 6, 3), rng)
    w = _rand((3, 3, 3, 4), rng)
    b = _rand(4, rng)
    y = oracle.conv3x3_fwd(x, w, b, relu=False)
    for n in range(2):
        for co in range(4):
            ref = np.full((7, 6), b[co])
            for ci in range(3):
                ref += ndimage.correlate(x[n, :, :, ci], w[:, :, ci, co], mode="constant", cval=0.0)
            assert np.allclose(y[n, :, :, co], ref, atol=1e-12)


def test_identity_shift_bias_and_relu():
    rng = np.random.default_rng(1)
    x = _rand((1, 5, 4, 2), rng)
    w = np.zeros((3, 3, 2, 2))
    w[1, 1] = np.eye(2)
    assert np.array_equal(oracle.conv3x3_fwd(x, w, np.zeros(2), False), x)
    # tap (ky=0, kx=1) reads the pixel above; the top row sees the zero padding
    w = np.zeros((3, 3, 2, 2))
    w[0, 1] = np.eye(2)
    y = oracle.conv3x3_fwd(x, w, np.zeros(2), False)
    assert np.array_equal(y[0, 1:], x[0, :-1]) and np.array_equal(y[0, 0], np.zeros((4, 2)))
    # tap (ky=1, kx=2) reads the pixel to the right
    w = np.zeros((3, 3, 2, 2))
    w[1, 2] = np.eye(2)
    y = oracle.conv3x3_fwd(x, w, np.zeros(2), False)
    assert np.array_equal(y[0, :, :-1], x[0, :, 1:]) and np.array_equal(y[0, :, -1], np.zeros((5, 2)))
    b = np.array([0.5, -0.25])
    y = oracle.conv3x3_fwd(x, np.zeros((3, 3, 2, 2)), b, True)
    assert np.array_equal(y[..., 0], np.full((1, 5, 4), 0.5)) and np.array_equal(y[..., 1], np.zeros((1, 5, 4)))


@pytest.mark.parametrize("relu", [False, True])
def test_layer_gradients_by_central_differences(relu):
    rng = np.random.default_rng(2 + relu)
    x = _rand((2, 5, 4, 3), rng)
    w = _rand((3, 3, 3, 2), rng, 0.5)
    b = _rand(2, rng, 0.1)
    r = _rand((2, 5, 4, 2), rng)       # L = sum(r * y)

    def L(x_, w_, b_):
        return float((r * oracle.conv3x3_fwd(x_, w_, b_, relu)).sum())

    y = oracle.conv3x3_fwd(x, w, b, relu)
    if relu:  # keep every pre-activation away from the kink
        z = oracle.conv3x3_fwd(x, w, b, False)
        assert np.abs(z).min() > 1e-4
    dx, dw, db = oracle.conv3x3_bwd(x, y, w, r, relu)
    h = 1e-6
    for arr, grad in ((x, dx), (w, dw), (b, db)):
        flat = arr.reshape(-1)
        for i in np.random.default_rng(9).choice(flat.size, min(flat.size, 25), replace=False):
            old = flat[i]
            flat[i] = old + h
            lp = L(x, w, b)
            flat[i] = old - h
            lm = L(x, w, b)
            flat[i] = old
            num = (lp - lm) / (2 * h)
            assert abs(num - grad.reshape(-1)[i]) <= 1e-7 * max(1.0, abs(num)), (i, num, grad.reshape(-1)[i])


def test_network_gradient_by_central_differences():
    rng = np.random.default_rng(4)
    n = oracle.corrector_num_params()
    assert n == 20835
    params = rng.normal(size=n) * 0.15
    rgb = rng.uniform(0, 1, (1, 6, 5, 3))
    x = oracle.corrector_input(rgb, rng.uniform(0, 3, (1, 6, 5)), rng.integers(0, 9, (1, 6, 5)))
    ref = rgb + rng.normal(size=rgb.shape) * 0.05
    loss, g = oracle.corrector_loss_grad(params, x, rgb, ref)
    h = 1e-6
    idx = np.concatenate([rng.choice(1472, 8, replace=False), 1472 + rng.choice(9248, 8, replace=False),
                          n - 867 + rng.choice(867, 8, replace=False)])
    for i in idx:
        p = params.copy()
        p[i] += h
        lp, _ = oracle.corrector_loss_grad(p, x, rgb, ref)
        p[i] -= 2 * h
        lm, _ = oracle.corrector_loss_grad(p, x, rgb, ref)
        num = (lp - lm) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 * max(1e-3, abs(num)) + 1e-10, (i, num, g[i])


def test_fallback_keeps_render_where_residual_is_large():
    rng = np.random.default_rng(5)
    params = rng.normal(size=oracle.corrector_num_params()) * 0.1
    rgb = rng.uniform(0, 1, (1, 8, 8, 3))
    x = oracle.corrector_input(rgb, np.ones((1, 8, 8)), np.full((1, 8, 8), 4))
    resid, _ = oracle.corrector_forward(params, x)
    out0, fb0 = oracle.corrector_apply(params, x, rgb, 0.0)
    assert fb0.all() and np.array_equal(out0, rgb)
    out1, fb1 = oracle.corrector_apply(params, x, rgb, np.inf)
    assert not fb1.any() and np.allclose(out1, rgb + resid)
    t = np.median(np.abs(resid).max(-1))
    out2, fb2 = oracle.corrector_apply(params, x, rgb, t)
    assert 0 < fb2.sum() < 64
    assert np.array_equal(out2[fb2], rgb[fb2]) and np.allclose(out2[~fb2], (rgb + resid)[~fb2])
