"""Restoration network: plain float64 definition (test infrastructure only).

The network is not part of the paper: it is a learned post-filter applied to
decoded viewports, trained on (decoded, uncompressed) pairs the codec
produces.  Four 3x3 convolutions, 32 channels, ReLU after the first three,
and a residual skip:

    a1 = relu(conv(x,  W1) + b1)        3 -> 32
    a2 = relu(conv(a1, W2) + b2)       32 -> 32
    a3 = relu(conv(a2, W3) + b3)       32 -> 32
    z  = conv(a3, W4) + b4              32 -> 3
    y  = x + z

with conv the cross-correlation with zero padding ("same" size):

    conv(x, W)[n, h, w, o] = sum_{ky, kx, i} x[n, h+ky-1, w+kx-1, i] W[o, ky, kx, i]

Layout: images NHWC, weights [out][ky][kx][in].  Loss: mean squared error of y
against the target over all pixels and the three channels.

``bf16`` rounding (round to nearest, ties to even) is provided so that a test
can apply the same rounding points as a bfloat16 implementation: inputs,
weights and the activations between layers.
"""
from __future__ import annotations

import numpy as np

HIDDEN = 32
LAYERS = [(3, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, 3)]


def bf16(a):
    """Round float values to the nearest bfloat16 (ties to even); float64 result."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def conv(x, w, b=None):
    """3x3 cross-correlation, zero padding.  x [N,H,W,I], w [O,3,3,I] -> [N,H,W,O]."""
    n, h, wd, i = x.shape
    xp = np.zeros((n, h + 2, wd + 2, i), dtype=np.float64)
    xp[:, 1:-1, 1:-1] = x
    out = np.zeros((n, h, wd, w.shape[0]), dtype=np.float64)
    for ky in range(3):
        for kx in range(3):
            out += xp[:, ky:ky + h, kx:kx + wd, :] @ w[:, ky, kx, :].T
    if b is not None:
        out += b
    return out


def conv_backward(x, w, dy):
    """Gradients of sum(dy * conv(x, w)) with respect to x, w and the bias."""
    n, h, wd, i = x.shape
    xp = np.zeros((n, h + 2, wd + 2, i), dtype=np.float64)
    xp[:, 1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w, dtype=np.float64)
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + h, kx:kx + wd, :]
            dw[:, ky, kx, :] = np.einsum("nhwo,nhwi->oi", dy, patch)
            dxp[:, ky:ky + h, kx:kx + wd, :] += dy @ w[:, ky, kx, :]
    db = dy.sum(axis=(0, 1, 2))
    return dxp[:, 1:-1, 1:-1], dw, db


def init_params(seed):
    """He-normal weights, zero biases; the last layer starts at zero output."""
    rng = np.random.Generator(np.random.PCG64(seed))
    params = []
    for li, (ci, co) in enumerate(LAYERS):
        std = np.sqrt(2.0 / (9 * ci))
        w = rng.normal(0.0, std, (co, 3, 3, ci))
        if li == len(LAYERS) - 1:
            w *= 0.1
        params += [w, np.zeros(co)]
    return params


def forward(x, params, round_acts=False):
    """Returns (y, z, activations a1..a3).  With ``round_acts`` the input and the
    hidden activations are rounded to bfloat16 where a bfloat16 network stores
    them."""
    r = bf16 if round_acts else (lambda v: v)
    acts = []
    h = r(x)
    for li in range(3):
        h = r(np.maximum(conv(h, params[2 * li], params[2 * li + 1]), 0.0))
        acts.append(h)
    z = conv(h, params[6], params[7])
    return r(x) + z, z, acts


def loss_and_grads(x, t, params, round_acts=False):
    """MSE loss of y = x + z against t, and its gradients (list like params)."""
    r = bf16 if round_acts else (lambda v: v)
    y, z, acts = forward(x, params, round_acts)
    count = y.size
    diff = y - t
    loss = float((diff * diff).sum() / count)
    d = r(2.0 * diff / count)                    # dL/dz (the skip passes x through)
    grads = [None] * 8
    inputs = [r(x)] + acts
    for li in range(3, -1, -1):
        dx, dw, db = conv_backward(inputs[li], params[2 * li], d)
        grads[2 * li], grads[2 * li + 1] = dw, db
        if li > 0:
            d = r(dx * (inputs[li] > 0))          # through the ReLU of layer li
    return loss, grads


def psnr(a, b, peak=255.0):
    """Peak signal-to-noise ratio of two images in dB."""
    mse = np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2)
    return float("inf") if mse == 0 else 10.0 * np.log10(peak * peak / mse)
