"""Inter-frame sets: the temporal Haar transform of Section 3.2 in the
coefficient domain, and the decode of one frame of a set (int64 / float64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

An inter-frame set is n consecutive frames, n a power of two.  The frame-wise
coefficients c_0 .. c_{n-1} (Section 3.1's 2D transform of each frame) are
transformed once more along time, position by position, with the Haar
wavelet, always down to a single approximation (log2 n levels, Section 3.2).

One Haar level on consecutive pairs (a, b):   s = (a + b) / 2,  d = (a - b) / 2.
Its synthesis is a = s + d, b = s - d, one signed addition per level, so
frame t of a set is

    c_t = B_0 + sum over j = log2 n .. 1 of  sign_j(t) * B_{n / 2^j + (t >> j)}

with sign_j(t) = +1 when bit j-1 of t is 0 and -1 otherwise: log2(n) signed
additions of stored bands (Section 3.2 reconstructs a frame by iterating over
the uploaded coefficients with the high-pass sign of each level).

Readings (the paper does not fix them):
* normalisation: the averaging Haar above (analysis halves, synthesis is pure
  +/- additions), the one under which reconstruction is additions only;
* band order: B_0 the approximation, then the details of the coarsest level,
  ..., then the n/2 details of level 1, each level's details in time order;
* quantisation: every band b has its own uniform step D_b.  5/3 stores int16
  indices q_b = sign(v) floor(|v| / D_b + 1/2) of the band values v and
  decodes c_t = sum of sign * D_b * q_b exactly in integers; 9/7 stores
  float32 band values and uses them as stored;
* decode of frame t: c_t per plane, the finest dropped levels zeroed per tile
  (Section 3.7), the 2D inverse transform, rec = clip(P, 0, 255), YUV420 ->
  RGB.  No reference frame: every frame of a set is decoded on its own (the
  keyframe-free random access that Section 3.2 motivates the sets with).
"""
from __future__ import annotations

import numpy as np

from . import codec
from .wavelet import W53, fwd2d


def _log2(n):
    k = int(n).bit_length() - 1
    if n < 1 or (1 << k) != n:
        raise ValueError(f"set size {n} is not a power of two")
    return k


def haar_forward(x):
    """Full-depth averaging Haar along axis 0 of x [n, ...] (float64).
    Returns the bands [n, ...] in the order described above."""
    a = np.asarray(x, dtype=np.float64)
    _log2(a.shape[0])
    details = []
    while a.shape[0] > 1:
        even, odd = a[0::2], a[1::2]
        details.insert(0, (even - odd) / 2.0)
        a = (even + odd) / 2.0
    return np.concatenate([a] + details, axis=0)


def haar_inverse(bands):
    """All n frames from the bands: level by level, a = s + d, b = s - d."""
    b = np.asarray(bands)
    n = b.shape[0]
    _log2(n)
    a = b[0:1]
    pos = 1
    while a.shape[0] < n:
        m = a.shape[0]
        d = b[pos:pos + m]
        pos += m
        nxt = np.empty((2 * m,) + a.shape[1:], dtype=np.result_type(a, d))
        nxt[0::2] = a + d
        nxt[1::2] = a - d
        a = nxt
    return a


def frame_terms(n, t):
    """(band, sign) pairs whose sum is frame t of a set of n: the
    approximation plus one detail per level."""
    k = _log2(n)
    if not 0 <= t < n:
        raise ValueError(f"frame {t} outside a set of {n}")
    terms = [(0, 1)]
    for j in range(k, 0, -1):
        terms.append(((n >> j) + (t >> j), -1 if (t >> (j - 1)) & 1 else 1))
    return terms


def haar_frame(bands, t):
    """Frame t from the bands by iterating the terms it needs."""
    b = np.asarray(bands)
    out = np.zeros(b.shape[1:], dtype=b.dtype)
    for band, sign in frame_terms(b.shape[0], t):
        out = out + sign * b[band]
    return out


def quantise_bands(bands, steps, wavelet):
    """Per-band uniform quantisation: 5/3 -> int16 indices, 9/7 -> float32 values."""
    out = []
    for v, step in zip(bands, steps):
        q = np.sign(v) * np.floor(np.abs(v) / step + 0.5)
        if wavelet == W53:
            assert q.min() >= -32768 and q.max() <= 32767
            out.append(q.astype(np.int16))
        else:
            out.append((step * q).astype(np.float32))
    return np.stack(out)


def encode_set(frames, levels, wavelet, steps):
    """Source frames -> stored bands of a set.

    frames: list over t (n frames) of lists of planes, each plane uint8
    [n_tiles, P, P].  Returns a list over planes of bands [n, n_tiles, P, P]
    (int16 for 5/3, float32 for 9/7)."""
    n = len(frames)
    if len(steps) != n:
        raise ValueError("one step per band")
    out = []
    for p in range(len(frames[0])):
        c = np.stack([fwd2d(np.asarray(f[p]), levels, wavelet) for f in frames])
        out.append(quantise_bands(haar_forward(c), steps, wavelet))
    return out


def frame_coefficients(bands, t, steps, wavelet):
    """Dequantised frame-wise coefficients c_t of one plane from its bands
    [n, ...]: int64 for 5/3 (sum of sign * step * q), float64 for 9/7."""
    b = np.asarray(bands)
    if wavelet == W53:
        out = np.zeros(b.shape[1:], dtype=np.int64)
        for band, sign in frame_terms(b.shape[0], t):
            out += sign * int(steps[band]) * b[band].astype(np.int64)
    else:
        out = np.zeros(b.shape[1:], dtype=np.float64)
        for band, sign in frame_terms(b.shape[0], t):
            out += sign * b[band].astype(np.float64)
    return out


def decode_set_viewport(planes, t, mask, levels, wavelet, steps, level_count=None):
    """Viewport output of frame t of a set.

    planes: per plane, bands [n, n_tiles, P, P]; mask: uint8 [n_tiles];
    level_count: int or array [n_tiles] (default: all levels).
    Returns (visible tile indices, out [n_vis, C, P, P], rec planes [n_vis, P, P])."""
    vis = np.nonzero(np.asarray(mask))[0]
    coeffs = [frame_coefficients(np.asarray(b)[:, vis], t, steps, wavelet) for b in planes]
    lc = levels if level_count is None else level_count
    lc = np.broadcast_to(np.asarray(lc), (np.asarray(planes[0]).shape[1],))[vis]
    res = codec.decode_tiles([{"coeffs": coeffs, "step": 1, "intra": True, "level_count": lc}],
                             levels, wavelet)[0]
    return vis, res["out"], res["rec"]
