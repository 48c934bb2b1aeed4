"""Seeded GOP construction for the parity tests (inputs from wvinputs, stored
coefficients and expected values from the oracle only)."""
from __future__ import annotations

import numpy as np

import wvinputs
from oracle import codec, viewport
from oracle import wavelet as owv

W53, W97 = owv.W53, owv.W97


class Gop:
    """Full-frame tile-major coefficient planes (numpy) for a GOP, with only the
    tiles in ``tiles`` populated (tiles are independent; the rest stay zero)."""

    def __init__(self, width, height, tile, levels, wavelet, n_frames, seed, tiles=None,
                 chroma=True, intra_step=None, rects=20.0):
        self.spec = wvinputs.FrameSpec(width, height, tile, seed, chroma=chroma,
                                       rects_per_512sq=rects)
        self.levels, self.wavelet, self.n_frames = levels, wavelet, n_frames
        self.tiles = np.arange(self.spec.n_tiles) if tiles is None else np.asarray(sorted(tiles))
        if intra_step is None:
            intra_step = 4 if wavelet == W53 else 8
        self.intra_step = intra_step
        n, sp = self.spec.n_tiles, self.spec
        src = wvinputs.source_planes(sp, tiles=self.tiles)
        self.source = [s.numpy().reshape(n, *s.shape[2:]) for s in src]
        sub = [s[self.tiles] for s in self.source]
        enc = codec.encode_intra(sub, levels, wavelet, intra_step)
        frames = []
        planes = []
        for p, e in zip(self.source, enc):
            full = np.zeros(p.shape, dtype=e.dtype)
            full[self.tiles] = e
            planes.append(full)
        frames.append({"coeffs": planes, "step": intra_step, "intra": True})
        for t in range(1, n_frames):
            res = wvinputs.residual_planes(sp, t, integer=(wavelet == W53), tiles=self.tiles)
            frames.append({"coeffs": [r.numpy().reshape(n, *r.shape[2:]) for r in res],
                           "step": 1, "intra": False})
        self.frames = frames

    @property
    def nplanes(self):
        return len(self.frames[0]["coeffs"])

    def oracle(self, masks, level_counts=None):
        """Oracle viewport outputs per frame: list of (visible, out, rec)."""
        frames = []
        for t, f in enumerate(self.frames):
            g = dict(f)
            g["level_count"] = (np.full(self.spec.n_tiles, self.levels) if level_counts is None
                                else np.asarray(level_counts[t]))
            frames.append(g)
        return codec.decode_viewport_gop(frames, masks, self.levels, self.wavelet,
                                         tiles=np.unique(np.concatenate(
                                             [np.nonzero(m)[0] for m in masks])))


def pose_mask(width, height, tile, seed, gop):
    yaw, pitch = wvinputs.head_pose(seed, gop)
    return viewport.tile_mask(width, height, tile, yaw, pitch), (yaw, pitch)
