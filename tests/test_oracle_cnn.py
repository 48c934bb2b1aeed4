"""Pins of the restoration network's CPU definition (oracle/cnn.py).

The convolution is checked against scipy's 2D cross-correlation, the
gradients against central finite differences, and the bfloat16 rounding
against torch's float32 -> bfloat16 conversion.
"""
import numpy as np
import pytest
import torch
from scipy.signal import correlate2d

from oracle import cnn


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(3)
    v = np.concatenate([rng.normal(0, 10, 5000), rng.uniform(-1, 1, 5000),
                        [0.0, -0.0, 1.0, 1.0 + 2**-8, 1.0 + 3 * 2**-9, 1.0 + 2**-9, -2.5, 65504.0]])
    want = torch.tensor(v, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(cnn.bf16(v), want)


def test_conv_matches_scipy_cross_correlation():
    rng = np.random.default_rng(5)
    x = rng.normal(size=(2, 7, 9, 3))
    w = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    got = cnn.conv(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = sum(correlate2d(x[n, :, :, i], w[o, :, :, i], mode="same") for i in range(3)) + b[o]
            assert np.allclose(got[n, :, :, o], ref, atol=1e-12)


def test_conv_of_delta_is_the_flipped_kernel():
    x = np.zeros((1, 5, 5, 1))
    x[0, 2, 2, 0] = 1.0
    w = np.arange(9, dtype=np.float64).reshape(1, 3, 3, 1)
    y = cnn.conv(x, w)[0, 1:4, 1:4, 0]
    assert np.array_equal(y, w[0, ::-1, ::-1, 0])


def _num_grad(f, arr, eps=1e-6):
    g = np.zeros_like(arr)
    it = np.nditer(arr, flags=["multi_index"])
    for _ in it:
        i = it.multi_index
        old = arr[i]
        arr[i] = old + eps
        fp = f()
        arr[i] = old - eps
        fm = f()
        arr[i] = old
        g[i] = (fp - fm) / (2 * eps)
    return g


def test_conv_backward_matches_finite_differences():
    rng = np.random.default_rng(7)
    x = rng.normal(size=(1, 4, 5, 2))
    w = rng.normal(size=(3, 3, 3, 2))
    dy = rng.normal(size=(1, 4, 5, 3))
    dx, dw, db = cnn.conv_backward(x, w, dy)

    def f():
        return float((cnn.conv(x, w) * dy).sum())

    assert np.allclose(dx, _num_grad(f, x), atol=1e-6)
    assert np.allclose(dw, _num_grad(f, w), atol=1e-6)
    assert np.allclose(db, dy.sum(axis=(0, 1, 2)))


@pytest.mark.parametrize("seed", [11, 12])
def test_network_gradients_match_finite_differences(seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1, (1, 5, 6, 3))
    t = np.clip(x + rng.normal(0, 0.05, x.shape), 0, 1)
    params = [p.copy() for p in cnn.init_params(seed)]
    for i in range(1, 8, 2):                      # non-zero biases exercise every term
        params[i] = rng.normal(0, 0.1, params[i].shape)
    params[6] = rng.normal(0, 0.05, params[6].shape)
    loss, grads = cnn.loss_and_grads(x, t, params)

    def f():
        return cnn.loss_and_grads(x, t, params)[0]

    for k in (0, 1, 5, 6, 7):                     # first, middle and last layers
        num = _num_grad(f, params[k])
        scale = max(np.abs(num).max(), 1e-8)
        assert np.abs(grads[k] - num).max() <= 1e-5 * scale + 1e-9, k


def test_zero_last_layer_is_identity():
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 1, (1, 6, 6, 3))
    params = cnn.init_params(4)
    params[6] = np.zeros_like(params[6])
    y, z, _ = cnn.forward(x, params)
    assert np.array_equal(y, x) and not z.any()


def test_psnr_definition():
    a = np.zeros((4, 4))
    b = np.full((4, 4), 255.0)
    assert cnn.psnr(a, b) == pytest.approx(0.0)
    c = a.copy()
    c[0, 0] = 16.0                                # mse = 16
    assert cnn.psnr(a, c) == pytest.approx(10 * np.log10(255.0**2 / 16.0))
