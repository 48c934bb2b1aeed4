"""Seeded synthetic inputs shared by the GPU decoder's tests/bench and the CPU oracle.

This module holds none of the codec's arithmetic: no wavelet, no quantiser,
no residual chain, no colour matrix and no viewport geometry.  It only draws
the raw material the workloads are made of, standing in for the paper's
360-degree videos (Section 4.1), which are not available:

* 8-bit source pictures: a smooth gradient, Gaussian noise and flat
  rectangles, generated tile by tile so that any subset of tiles can be
  produced on its own and agrees with the full frame;
* residual coefficient fields drawn i.i.d. from a Laplace(0, b) law;
* head poses (yaw/pitch) and head-yaw random walks with request times.

Everything is keyed by integer seeds through numpy's SeedSequence, so a tile,
a plane or a frame can be regenerated independently on any device.  Values
drawn with torch on a GPU differ from those drawn on the CPU for the same key
(different generator streams) but follow the same recipe.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch

BASE_SEED = 10859

__all__ = [
    "BASE_SEED", "FrameSpec", "derive_seed", "torch_generator", "rectangles",
    "source_tile", "source_planes", "residual_planes", "head_pose",
    "yaw_walk", "request_times",
]


def derive_seed(*keys) -> int:
    """A 63-bit seed derived from a tuple of ints/strings (SeedSequence mixing)."""
    ints = []
    for k in keys:
        if isinstance(k, str):
            ints.extend(k.encode())
        else:
            ints.append(int(k) & 0xFFFFFFFF)
    ss = np.random.SeedSequence(ints)
    return int(ss.generate_state(1, dtype=np.uint64)[0] >> np.uint64(1))


def torch_generator(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    return g


@dataclasses.dataclass(frozen=True)
class FrameSpec:
    """Geometry of one synthetic YUV420 (or grey) frame stored tile by tile.

    ``tile`` is the luma tile edge; chroma planes are half size in both
    directions (YUV420) and use tiles of ``tile // 2``.
    """
    width: int
    height: int
    tile: int
    seed: int
    chroma: bool = True
    rects_per_512sq: float = 20.0

    @property
    def tiles_x(self) -> int:
        return self.width // self.tile

    @property
    def tiles_y(self) -> int:
        return self.height // self.tile

    @property
    def n_tiles(self) -> int:
        return self.tiles_x * self.tiles_y

    def plane_tile(self, plane: int) -> int:
        return self.tile if plane == 0 else self.tile // 2

    @property
    def n_planes(self) -> int:
        return 3 if self.chroma else 1


def rectangles(spec: FrameSpec) -> dict:
    """Flat rectangles of the whole frame, in overwrite order.

    Top-left corner uniform over the frame, width/height uniform in 16..128,
    one value per plane uniform in 0..255.  The count scales with the area
    (``rects_per_512sq`` per 512x512 of luma).
    """
    count = int(round(spec.rects_per_512sq * spec.width * spec.height / (512 * 512)))
    rng = np.random.Generator(np.random.PCG64(derive_seed(spec.seed, "rect")))
    x0 = rng.integers(0, spec.width, count)
    y0 = rng.integers(0, spec.height, count)
    w = rng.integers(16, 129, count)
    h = rng.integers(16, 129, count)
    val = rng.integers(0, 256, (count, 3))
    return {"x0": x0, "y0": y0, "w": w, "h": h, "val": val}


def source_tile(spec: FrameSpec, plane: int, ty: int, tx: int, rects=None,
                device="cpu") -> torch.Tensor:
    """One tile of one plane of the 8-bit source picture (uint8, [P, P]).

    Luma: 32 + 192*(x+y)/(W+H-2) + N(0, 8^2).  Chroma (Cb, Cr): 64 + 128*x/(Wc-1)
    resp. 64 + 128*y/(Hc-1) + N(0, 4^2).  Then the frame's rectangles overwrite
    their area with a flat value, in order; round to nearest and clip to 0..255.
    """
    if rects is None:
        rects = rectangles(spec)
    p = spec.plane_tile(plane)
    sub = 1 if plane == 0 else 2
    wp, hp = spec.width // sub, spec.height // sub
    ys = torch.arange(ty * p, ty * p + p, device=device, dtype=torch.float32)
    xs = torch.arange(tx * p, tx * p + p, device=device, dtype=torch.float32)
    g = torch_generator(derive_seed(spec.seed, "noise", plane, ty, tx), device)
    noise = torch.randn((p, p), generator=g, device=device, dtype=torch.float32)
    if plane == 0:
        img = 32.0 + 192.0 * (ys[:, None] + xs[None, :]) / float(wp + hp - 2) + 8.0 * noise
    elif plane == 1:
        img = 64.0 + 128.0 * xs[None, :].expand(p, p) / float(wp - 1) + 4.0 * noise
    else:
        img = 64.0 + 128.0 * ys[:, None].expand(p, p) / float(hp - 1) + 4.0 * noise
    # rectangles intersecting this tile (in plane coordinates), in order
    rx0 = rects["x0"] // sub
    ry0 = rects["y0"] // sub
    rx1 = (rects["x0"] + rects["w"]) // sub
    ry1 = (rects["y0"] + rects["h"]) // sub
    tx0, ty0 = tx * p, ty * p
    hit = np.nonzero((rx0 < tx0 + p) & (rx1 > tx0) & (ry0 < ty0 + p) & (ry1 > ty0))[0]
    for i in hit:
        a0 = max(int(ry0[i]) - ty0, 0)
        a1 = min(int(ry1[i]) - ty0, p)
        b0 = max(int(rx0[i]) - tx0, 0)
        b1 = min(int(rx1[i]) - tx0, p)
        img[a0:a1, b0:b1] = float(rects["val"][i, plane])
    return torch.clamp(torch.round(img), 0, 255).to(torch.uint8)


def source_planes(spec: FrameSpec, tiles=None, device="cpu") -> list:
    """Source picture planes in tile-major layout: plane i is [ty, tx, P, P] uint8.

    ``tiles`` (iterable of flat tile indices) restricts generation to those
    tiles; the others are left zero.  A tile's content does not depend on
    which other tiles are generated.
    """
    rects = rectangles(spec)
    out = []
    for plane in range(spec.n_planes):
        p = spec.plane_tile(plane)
        t = torch.zeros((spec.tiles_y, spec.tiles_x, p, p), dtype=torch.uint8, device=device)
        for idx in (range(spec.n_tiles) if tiles is None else tiles):
            ty, tx = divmod(int(idx), spec.tiles_x)
            t[ty, tx] = source_tile(spec, plane, ty, tx, rects, device)
        out.append(t)
    return out


def residual_planes(spec: FrameSpec, frame: int, scale: float = 2.0, integer: bool = True,
                    tiles=None, device="cpu") -> list:
    """Residual coefficient planes of one frame, tile-major [ty, tx, P, P].

    Every coefficient position (all subbands) is an i.i.d. draw of
    Laplace(0, scale) = scale * (E1 - E2) with E1, E2 ~ Exp(1); rounded to
    int16 when ``integer``, float32 otherwise.  Seeded per (frame, plane, tile).
    """
    out = []
    for plane in range(spec.n_planes):
        p = spec.plane_tile(plane)
        dt = torch.int16 if integer else torch.float32
        t = torch.zeros((spec.tiles_y, spec.tiles_x, p, p), dtype=dt, device=device)
        for idx in (range(spec.n_tiles) if tiles is None else tiles):
            ty, tx = divmod(int(idx), spec.tiles_x)
            g = torch_generator(derive_seed(spec.seed, "resid", frame, plane, ty, tx), device)
            e1 = torch.empty((p, p), device=device, dtype=torch.float32).exponential_(generator=g)
            e2 = torch.empty((p, p), device=device, dtype=torch.float32).exponential_(generator=g)
            v = scale * (e1 - e2)
            t[ty, tx] = torch.round(v).clamp(-32768, 32767).to(dt) if integer else v
        out.append(t)
    return out


def head_pose(seed: int, gop: int) -> tuple:
    """(yaw, pitch) in degrees: yaw ~ U[-180, 180), pitch ~ U[-30, 30]."""
    rng = np.random.Generator(np.random.PCG64(derive_seed(seed, "pose", gop)))
    return float(rng.uniform(-180.0, 180.0)), float(rng.uniform(-30.0, 30.0))


def yaw_walk(seed: int, stream: int, n: int, hz: float = 90.0, sigma_deg_per_s: float = 30.0,
             pitch_range: float = 20.0) -> np.ndarray:
    """Head yaw/pitch per requested frame: yaw is a Gaussian random walk with
    standard deviation ``sigma_deg_per_s * sqrt(1/hz)`` per step; pitch fixed per
    stream, uniform in +-pitch_range.  Returns float64 [n, 2] degrees."""
    rng = np.random.Generator(np.random.PCG64(derive_seed(seed, "walk", stream)))
    yaw0 = rng.uniform(-180.0, 180.0)
    pitch = rng.uniform(-pitch_range, pitch_range)
    steps = rng.normal(0.0, sigma_deg_per_s * math.sqrt(1.0 / hz), n)
    steps[0] = 0.0
    yaw = (yaw0 + np.cumsum(steps) + 180.0) % 360.0 - 180.0
    return np.stack([yaw, np.full(n, pitch)], axis=1)


def request_times(seed: int, stream: int, n: int, hz: float = 90.0, jitter: float = 0.25) -> np.ndarray:
    """Request times (seconds) of one stream: nominal period 1/hz, each gap
    drawn as period * (1 - jitter) + Exp(period * jitter) (Poisson jitter)."""
    rng = np.random.Generator(np.random.PCG64(derive_seed(seed, "arrive", stream)))
    period = 1.0 / hz
    gaps = period * (1.0 - jitter) + rng.exponential(period * jitter, n)
    t0 = rng.uniform(0.0, period)
    return t0 + np.concatenate([[0.0], np.cumsum(gaps[:-1])])
