"""Quantiser, intra encoder and the decode definition (int64 / float64).

The decode of one GOP, for every tile independently (Section 3.1's transform
applied per tile; the paper transforms whole frames, tiles are the reading
used here so that a viewport touches a bounded set of coefficients):

  for frame t = 0 .. G-1:
    c_t   = step_t * q_t                    dequantise (inverse of the quantiser)
    c_t'  = c_t with the detail bands of the finest (L - level_count_t) levels
            set to zero                     foveated decoding, Section 3.7
    P_t   = iFWT_L(c_t')                    rows then columns per level
    rec_t = clip(P_t, 0, 255)               intra frame
    rec_t = clip(rec_{t-1} + P_t, 0, 255)   residual frame, onto the previous
                                            decoded frame (closed loop)
    out_t = YUV420 -> RGB (rec_t)           or the luma itself for grey frames

The viewport output of frame t is out_t restricted to the tiles of its mask,
in ascending tile index (Section 3.1: only the viewport is reconstructed; it
must equal the same region of a full decode).

Readings: quantiser q = sign(c) floor(|c|/step + 1/2), decoder c = step * q
(no mid-point offset); intra frames are quantised, residual frames carry their
coefficients directly (step 1).  For 9/7 the store holds float32 values that
are already multiples of the step (step * q); the chain keeps float64 planes
and clips without rounding.  The paper's own inter-frame coding (a Haar
transform in the coefficient domain) and its 8-bit min/max normalisation are
different models and are not what this chain computes.
"""
from __future__ import annotations

import numpy as np

from . import colour
from .wavelet import W53, W97, fwd2d, inv2d, zero_finest


def quantise_int(c, step):
    """Integer coefficients -> q = sign(c) * floor(|c| / step + 1/2) (exact integer form)."""
    c = np.asarray(c, dtype=np.int64)
    a = (2 * np.abs(c) + step) // (2 * step)
    return np.sign(c) * a


def quantise_float(c, step):
    """Float coefficients -> step * sign(c) * floor(|c| / step + 1/2)."""
    c = np.asarray(c, dtype=np.float64)
    return step * np.sign(c) * np.floor(np.abs(c) / step + 0.5)


def encode_intra(planes, levels, wavelet, step):
    """Source planes (uint8 [..., P, P] per plane) -> stored coefficients.

    5/3: int16 quantisation indices; 9/7: float32 dequantised values.
    """
    out = []
    for p in planes:
        c = fwd2d(np.asarray(p), levels, wavelet)
        if wavelet == W53:
            q = quantise_int(c, step)
            assert q.min() >= -32768 and q.max() <= 32767
            out.append(q.astype(np.int16))
        else:
            out.append(quantise_float(c, float(step)).astype(np.float32))
    return out


def _inverse_per_tile(c, levels, wavelet, level_count):
    """Zero dropped levels tile by tile, then the inverse transform."""
    c = np.array(c, copy=True)
    lc = np.broadcast_to(np.asarray(level_count), c.shape[:1])
    for k in np.unique(lc):
        sel = lc == k
        c[sel] = zero_finest(c[sel], levels - int(k))
    return inv2d(c, levels, wavelet)


def decode_tiles(frames, levels, wavelet=W53):
    """Decode a GOP for a set of tiles.

    frames: list of dicts with
      ``coeffs``: list of planes, each [n, P, P] (int16 for 5/3, float32 for 9/7),
      ``step``: integer dequantisation step (5/3; ignored for 9/7),
      ``intra``: bool,
      ``level_count``: int or array [n] of detail levels to apply (<= levels).
    Returns a list (per frame) of dicts ``rec`` (planes, int64 or float64)
    and ``out`` ([n, 3, P, P] RGB, or [n, 1, P, P] for a single plane).
    """
    results = []
    rec = None
    for f in frames:
        planes = []
        for pi, q in enumerate(f["coeffs"]):
            if wavelet == W53:
                c = np.asarray(q, dtype=np.int64) * int(f["step"])
            else:
                c = np.asarray(q, dtype=np.float64)
            p = _inverse_per_tile(c, levels, wavelet, f.get("level_count", levels))
            if f["intra"]:
                r = np.clip(p, 0, 255)
            else:
                assert rec is not None, "a residual frame needs a reference"
                r = np.clip(rec[pi] + p, 0, 255)
            planes.append(r)
        rec = planes
        if len(planes) == 3:
            if wavelet == W53:
                out = colour.yuv420_to_rgb_q16(*planes)
            else:
                out = colour.yuv420_to_rgb_real(*planes)
        else:
            out = planes[0][:, None].astype(np.uint8 if wavelet == W53 else np.float64)
        results.append({"rec": planes, "out": out})
    return results


def decode_viewport_gop(frames, masks, levels, wavelet=W53, tiles=None):
    """Viewport outputs of a GOP from full-frame tile-major coefficient planes.

    frames: as in ``decode_tiles`` but ``coeffs`` planes are [n_tiles, P, P]
    (flattened tile-major) and ``level_count`` is an array [n_tiles].
    masks: list of uint8 [n_tiles].  ``tiles`` restricts the work to a set of
    tile indices (default: union of all masks); since tiles are independent,
    the result for a tile does not depend on which other tiles are decoded.
    Returns per frame: (visible tile indices, out [n_vis, C, P, P], rec planes
    restricted to the visible tiles).
    """
    if tiles is None:
        tiles = np.nonzero(np.any(np.stack(masks), axis=0))[0]
    tiles = np.asarray(sorted(int(t) for t in tiles))
    sub = []
    for f in frames:
        g = dict(f)
        g["coeffs"] = [np.asarray(p)[tiles] for p in f["coeffs"]]
        lc = f.get("level_count", levels)
        g["level_count"] = np.broadcast_to(np.asarray(lc), (len(frames[0]["coeffs"][0]),))[tiles] \
            if np.ndim(lc) else lc
        sub.append(g)
    res = decode_tiles(sub, levels, wavelet)
    out = []
    pos = {t: i for i, t in enumerate(tiles.tolist())}
    for m, r in zip(masks, res):
        vis = np.nonzero(m)[0]
        idx = np.asarray([pos[int(t)] for t in vis], dtype=np.int64)
        out.append((vis, r["out"][idx], [p[idx] for p in r["rec"]]))
    return out
