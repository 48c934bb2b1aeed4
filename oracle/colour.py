"""YUV420 -> RGB, the last step of the decode.

The paper performs no colour transform (Section 5, "File Size"); the decoder
here takes YUV420 8-bit frames and converts them to RGB with the JFIF
full-range matrix

    R = Y + 1.402    (Cr - 128)
    G = Y - 0.344136 (Cb - 128) - 0.714136 (Cr - 128)
    B = Y + 1.772    (Cb - 128)

with nearest (2x2 replicate) chroma upsampling.  Integer path (5/3): Q16 fixed
point, constants round(65536 * k): 91881, 22554, 46802, 116130, and
out = ((Y << 16) + sum k_i (C_i - 128) + 32768) >> 16, clipped to 0..255.
Float path (9/7): the real formula in float64, clipped to [0, 255].
"""
from __future__ import annotations

import numpy as np

Q16 = {"r_cr": 91881, "g_cb": -22554, "g_cr": -46802, "b_cb": 116130}
REAL = {"r_cr": 1.402, "g_cb": -0.344136, "g_cr": -0.714136, "b_cb": 1.772}


def upsample2(c):
    """Nearest chroma upsampling: C[x >> 1][y >> 1] for every luma position."""
    return np.repeat(np.repeat(c, 2, axis=-2), 2, axis=-1)


def rgb_q16_samples(y, cb, cr):
    """Q16 conversion of co-sited samples (same shape arrays, int-valued)."""
    y = np.asarray(y, dtype=np.int64)
    cb = np.asarray(cb, dtype=np.int64) - 128
    cr = np.asarray(cr, dtype=np.int64) - 128
    r = ((y << 16) + Q16["r_cr"] * cr + 32768) >> 16
    g = ((y << 16) + Q16["g_cb"] * cb + Q16["g_cr"] * cr + 32768) >> 16
    b = ((y << 16) + Q16["b_cb"] * cb + 32768) >> 16
    return np.clip(np.stack([r, g, b], axis=0), 0, 255)


def rgb_real_samples(y, cb, cr):
    """Real-valued conversion of co-sited samples (float64, clipped to [0, 255])."""
    y = np.asarray(y, dtype=np.float64)
    cb = np.asarray(cb, dtype=np.float64) - 128.0
    cr = np.asarray(cr, dtype=np.float64) - 128.0
    r = y + REAL["r_cr"] * cr
    g = y + REAL["g_cb"] * cb + REAL["g_cr"] * cr
    b = y + REAL["b_cb"] * cb
    return np.clip(np.stack([r, g, b], axis=0), 0.0, 255.0)


def yuv420_to_rgb_q16(y, cb, cr):
    """Planes [..., H, W], [..., H/2, W/2] -> RGB planar [..., 3, H, W] uint8."""
    out = rgb_q16_samples(y, upsample2(cb), upsample2(cr))
    return np.moveaxis(out, 0, -3).astype(np.uint8)


def yuv420_to_rgb_real(y, cb, cr):
    """Float planes -> RGB planar [..., 3, H, W] float64."""
    out = rgb_real_samples(y, upsample2(cb), upsample2(cr))
    return np.moveaxis(out, 0, -3)
