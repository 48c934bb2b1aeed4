"""The paper's storage format for frame-wise coefficients (Sections 3.3, 3.4,
3.6) and its rebuild into a dense wavelet image (Section 3.5).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Encode one plane of one frame (tile-major Mallat planes [n_tiles][P][P] on the
0..255 colour scale):

1. Threshold (Eq. 2 with the level-weighted T of Eq. 3 and the pole factor of
   Section 3.6): a detail coefficient c of detail level k (1 = finest) is kept
   iff |c| / 255 > T, with
       T = alpha * ((l_max - l) / l_max)^2 + H(y),   l = k - 1,  l_max = L,
       H(y) = 1 - sin(pi * y / S_y)   (pole weighting on; else H = 0).
   Readings: l counts detail levels from 0 at the finest, so the finest
   details get the largest threshold (the paper zeroes more at high
   frequencies); coefficients compare on the 0..1 colour scale of the paper's
   float components; y is the centre row of the samples a coefficient covers,
   within its eye (S_y = eye height, frames are top-bottom stereo); the
   approximation band is never thresholded (with T = H it would vanish at the
   poles).
2. Quantise (Eq. 4): code = floor((c - c_min) / (c_max - c_min) * 255 + 1/2),
   with one (c_min, c_max) over the kept approximation coefficients of the
   plane and one over its kept detail coefficients (float64 arithmetic on the
   float32 values).  Decode: c = c_min + code * scale with
   scale = float32((c_max - c_min) / 255), each operation in float32 (the
   precision of the rebuild kernel: the product and the sum rounded once each).
3. Blocks (Section 3.4): each tile's Mallat plane is cut into B x B blocks,
   B = min(32, P).  A block's level is the level of the detail region its
   origin lies in (L + 1 for the block holding the approximation); blocks are
   ordered by level from the lowest frequency, row-major within a level.  A
   record is (code, index = y * B + x inside the block), ascending index within
   a block.  block_end[t * nb + j] is the exclusive end of the records of block
   j (in that order) of tile t, cumulative over the plane (reading: the paper's
   pointer names the last coefficient of the block; an exclusive end is the
   same information).

Rebuild of a visible tile with level count lc: zero the tile, then place every
record of the blocks whose level exceeds L - lc (the others are not read: with
level-wise order they are the tile's trailing records).  5/3 dense planes take
the nearest integer (ties to even) of the float32 value.
"""
from __future__ import annotations

import numpy as np

from . import codec
from .wavelet import W53

BLOCK = 32


def block_size(p):
    return min(BLOCK, p)


def block_level(p, levels, by, bx):
    """Level of the detail region holding block (by, bx)'s origin; levels + 1
    for the approximation region."""
    b = block_size(p)
    m = max(by, bx) * b
    for k in range(1, levels + 1):
        if m >= p >> k:
            return k
    return levels + 1


def block_order(p, levels):
    """Blocks (by, bx) of a P x P plane in storage order."""
    nb = p // block_size(p)
    blocks = [(by, bx) for by in range(nb) for bx in range(nb)]
    return sorted(blocks, key=lambda b: (-block_level(p, levels, *b), b[0], b[1]))


def coefficient_level(p, levels):
    """[P, P] detail level of every coefficient (0 = approximation)."""
    y, x = np.meshgrid(np.arange(p), np.arange(p), indexing="ij")
    m = np.maximum(y, x)
    lev = np.zeros((p, p), dtype=np.int64)
    for k in range(levels, 0, -1):
        lev[m >= (p >> k)] = k
    return lev


def coefficient_rows(p, levels):
    """[P, P] centre row (inside the tile, in samples of this plane) of the
    samples each coefficient covers."""
    y = np.arange(p)[:, None] * np.ones((1, p), dtype=np.int64)
    lev = coefficient_level(p, levels)
    rows = np.zeros((p, p), dtype=np.float64)
    for k in range(1, levels + 1):
        sel = lev == k
        half = p >> k
        band_row = np.where(y >= half, y - half, y)
        rows[sel] = ((band_row + 0.5) * (1 << k))[sel]
    sel = lev == 0
    rows[sel] = ((y + 0.5) * (1 << levels))[sel]
    return rows


def thresholds(p, levels, tiles_x, plane_height, alpha, poles):
    """[n_tiles, P, P] threshold T of every detail coefficient (Eq. 3);
    -1 for the approximation (always kept)."""
    n_tiles = (plane_height // p) * tiles_x
    lev = coefficient_level(p, levels)
    rows = coefficient_rows(p, levels)
    eye = plane_height / 2.0
    out = np.empty((n_tiles, p, p), dtype=np.float64)
    for t in range(n_tiles):
        y = (t // tiles_x) * p + rows
        h = 1.0 - np.sin(np.pi * np.mod(y, eye) / eye) if poles else np.zeros_like(y)
        lw = ((levels - (lev - 1)) / levels) ** 2
        out[t] = np.where(lev == 0, -1.0, alpha * lw + h)
    return out


def encode_plane(c, levels, tiles_x, plane_height, alpha, poles):
    """One plane (float32 [n_tiles, P, P]) -> dict with block_end (uint32),
    values (uint8), index (uint16) and the four float32 bounds."""
    c = np.asarray(c, dtype=np.float32)
    n_tiles, p, _ = c.shape
    if n_tiles != (plane_height // p) * tiles_x:
        raise ValueError("plane geometry does not match the tile count")
    b = block_size(p)
    thr = thresholds(p, levels, tiles_x, plane_height, alpha, poles)
    lev = coefficient_level(p, levels)
    approx = np.broadcast_to(lev == 0, c.shape)
    keep = approx | (np.abs(c.astype(np.float64)) / 255.0 > thr)

    def bounds(sel):
        v = c[keep & sel]
        return (np.float32(v.min()), np.float32(v.max())) if v.size else (np.float32(0), np.float32(0))

    amin, amax = bounds(approx)
    dmin, dmax = bounds(~approx)
    order = block_order(p, levels)
    block_end, values, index = [], [], []
    total = 0
    for t in range(n_tiles):
        for by, bx in order:
            blk = c[t, by * b:(by + 1) * b, bx * b:(bx + 1) * b].astype(np.float64)
            kb = keep[t, by * b:(by + 1) * b, bx * b:(bx + 1) * b]
            ab = approx[t, by * b:(by + 1) * b, bx * b:(bx + 1) * b]
            idx = np.nonzero(kb.reshape(-1))[0]
            v = blk.reshape(-1)[idx]
            is_a = ab.reshape(-1)[idx]
            lo = np.where(is_a, float(amin), float(dmin))
            hi = np.where(is_a, float(amax), float(dmax))
            span = hi - lo
            code = np.where(span > 0, np.floor((v - lo) / np.where(span > 0, span, 1.0) * 255.0 + 0.5), 0)
            values.append(code.astype(np.uint8))
            index.append(idx.astype(np.uint16))
            total += idx.size
            block_end.append(total)
    return {"block_end": np.asarray(block_end, dtype=np.uint32),
            "values": np.concatenate(values) if values else np.zeros(0, np.uint8),
            "index": np.concatenate(index) if index else np.zeros(0, np.uint16),
            "bounds": np.asarray([amin, amax, dmin, dmax], dtype=np.float32)}


def dequantise(code, lo, hi):
    """c = c_min + code * scale in float32, scale = float32((c_max - c_min) / 255)."""
    scale = np.float32((float(hi) - float(lo)) / 255.0)
    return np.float32(lo) + np.asarray(code, dtype=np.float32) * scale


def rebuild_plane(fmt, p, levels, tiles, level_count, wavelet):
    """Dense planes [len(tiles), P, P] of the given tiles (level_count: int or
    [n_tiles]): float32 (9/7) or int16 (5/3, nearest integer)."""
    b = block_size(p)
    order = block_order(p, levels)
    nb = len(order)
    amin, amax, dmin, dmax = fmt["bounds"]
    lc = np.asarray(level_count)
    out = np.zeros((len(tiles), p, p), dtype=np.float32)
    for i, t in enumerate(tiles):
        keep_levels = int(lc) if lc.ndim == 0 else int(lc[t])
        for j, (by, bx) in enumerate(order):
            if block_level(p, levels, by, bx) <= levels - keep_levels:
                continue
            g = t * nb + j
            s = int(fmt["block_end"][g - 1]) if g > 0 else 0
            e = int(fmt["block_end"][g])
            idx = fmt["index"][s:e].astype(np.int64)
            y, x = by * b + idx // b, bx * b + idx % b
            is_a = (y < (p >> levels)) & (x < (p >> levels))
            val = np.where(is_a, dequantise(fmt["values"][s:e], amin, amax),
                           dequantise(fmt["values"][s:e], dmin, dmax))
            out[i, y, x] = val
    if wavelet == W53:
        return np.clip(np.rint(out), -32768, 32767).astype(np.int16)
    return out


def decode_viewport(planes_fmt, p_edges, mask, levels, wavelet, level_count=None):
    """Viewport output of one frame stored in the format: rebuild the visible
    tiles, then the intra decode of Section 3.1.  planes_fmt: encode_plane
    results per plane; p_edges: P of each plane.
    Returns (visible tiles, out, rec planes, dense planes)."""
    vis = np.nonzero(np.asarray(mask))[0]
    n_tiles = np.asarray(mask).size
    lc = np.full(n_tiles, levels) if level_count is None else np.asarray(level_count)
    dense = [rebuild_plane(f, pe, levels, vis, lc, wavelet) for f, pe in zip(planes_fmt, p_edges)]
    res = codec.decode_tiles([{"coeffs": dense, "step": 1, "intra": True, "level_count": lc[vis]}],
                             levels, wavelet)[0]
    return vis, res["out"], res["rec"], dense
