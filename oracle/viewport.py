"""Viewport tile selection and foveation levels (float64 geometry).

Section 3.1: only the part of the panorama inside the viewport is
reconstructed, selected by a low-resolution binary mask defined on the frame.
Section 3.6: the mask is independent of the mapping; experiments use the
equirectangular projection.  Section 3.7: with gaze available, full resolution
is kept only near the fixation point and fewer wavelet levels are applied with
growing eccentricity.

Readings used here:
* frame = top-bottom stereo; each eye is an equirectangular W x H/2 image
  (longitude -180..180 left to right, latitude 90..-90 top to bottom);
* a tile is in the mask when any of ``samples`` x ``samples`` sample points
  (at (j + 0.5) * tile / samples inside the tile) lies inside a rectilinear
  frustum of fov_h x fov_v degrees around the head direction;
  ``eyes = 1`` selects the top eye only, ``eyes = 2`` both eyes (same pose);
* foveation: eccentricity = angle between the gaze (the viewport centre) and
  the tile-centre direction; drop 0 levels at <= inner, 1 at <= outer, 2 beyond.

Camera frame for yaw psi, pitch theta (degrees):
  forward = (cos t sin p, sin t, cos t cos p), right = (cos p, 0, -sin p),
  up = (-sin t sin p, cos t, -sin t cos p);
a direction d is inside when d.forward > 0 and |d.right| <= tan(fov_h/2) d.forward
and |d.up| <= tan(fov_v/2) d.forward.
"""
from __future__ import annotations

import math

import numpy as np


def _direction(x, y, eye_w, eye_h):
    """Unit direction of equirect pixel position (x, y) (continuous, in pixels)."""
    lon = (x / eye_w) * (2.0 * math.pi) - math.pi
    lat = 0.5 * math.pi - (y / eye_h) * math.pi
    cl = np.cos(lat)
    return cl * np.sin(lon), np.sin(lat), cl * np.cos(lon)


def _camera(yaw_deg, pitch_deg):
    p = yaw_deg * (math.pi / 180.0)
    t = pitch_deg * (math.pi / 180.0)
    fwd = (math.cos(t) * math.sin(p), math.sin(t), math.cos(t) * math.cos(p))
    right = (math.cos(p), 0.0, -math.sin(p))
    up = (-math.sin(t) * math.sin(p), math.cos(t), -math.sin(t) * math.cos(p))
    return fwd, right, up


def tile_mask(width, height, tile, yaw_deg, pitch_deg, fov_h_deg=110.0, fov_v_deg=110.0,
              samples=16, eyes=1):
    """uint8 [tiles_y * tiles_x] mask (row-major tile index ty * tiles_x + tx)."""
    ntx, nty = width // tile, height // tile
    eye_h = height / 2.0
    fwd, right, up = _camera(yaw_deg, pitch_deg)
    th = math.tan(fov_h_deg * (math.pi / 360.0))
    tv = math.tan(fov_v_deg * (math.pi / 360.0))
    mask = np.zeros(nty * ntx, dtype=np.uint8)
    off = (np.arange(samples, dtype=np.float64) + 0.5) * (tile / samples)
    for ty in range(nty):
        eye = 0 if (ty * tile) < eye_h else 1
        if eye >= eyes:
            continue
        for tx in range(ntx):
            xs = tx * tile + off[None, :]
            ys = ty * tile + off[:, None] - eye * eye_h
            dx, dy, dz = _direction(xs, ys, float(width), eye_h)
            zf = dx * fwd[0] + dy * fwd[1] + dz * fwd[2]
            xr = dx * right[0] + dy * right[1] + dz * right[2]
            yu = dx * up[0] + dy * up[1] + dz * up[2]
            inside = (zf > 0.0) & (np.abs(xr) <= th * zf) & (np.abs(yu) <= tv * zf)
            if inside.any():
                mask[ty * ntx + tx] = 1
    return mask


def foveation_drop(width, height, tile, yaw_deg, pitch_deg, inner_deg=20.0, outer_deg=40.0):
    """uint8 [n_tiles] number of finest detail levels to drop per tile (0, 1 or 2).

    Both eyes share the gaze; each tile's centre is mapped with its own eye.
    """
    ntx, nty = width // tile, height // tile
    eye_h = height / 2.0
    fwd, _, _ = _camera(yaw_deg, pitch_deg)
    drop = np.zeros(nty * ntx, dtype=np.uint8)
    for ty in range(nty):
        eye = 0 if (ty * tile) < eye_h else 1
        for tx in range(ntx):
            x = (tx + 0.5) * tile
            y = (ty + 0.5) * tile - eye * eye_h
            dx, dy, dz = _direction(np.float64(x), np.float64(y), float(width), eye_h)
            c = float(dx * fwd[0] + dy * fwd[1] + dz * fwd[2])
            ecc = math.degrees(math.acos(max(-1.0, min(1.0, c))))
            drop[ty * ntx + tx] = 0 if ecc <= inner_deg else (1 if ecc <= outer_deg else 2)
    return drop
