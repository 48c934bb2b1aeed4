"""Pins of the oracle's colour conversion and viewport geometry."""
import numpy as np
import pytest

import wvinputs
from oracle import colour, viewport


def test_q16_colour_exhaustive_within_one_lsb():
    """All 256^3 (Y, Cb, Cr): the Q16 conversion differs from round-half-up of
    the real JFIF formula (clipped) by at most 1, and is exact for R."""
    cb, cr = np.meshgrid(np.arange(256), np.arange(256), indexing="ij")
    worst = np.zeros(3)
    mism = np.zeros(3, dtype=np.int64)
    for y in range(256):
        yy = np.full_like(cb, y)
        q = colour.rgb_q16_samples(yy, cb, cr)
        real = colour.rgb_real_samples(yy, cb, cr)
        ref = np.clip(np.floor(real + 0.5), 0, 255)
        dlt = np.abs(q - ref).reshape(3, -1)
        worst = np.maximum(worst, dlt.max(axis=1))
        mism += (dlt > 0).sum(axis=1)
    assert worst.max() <= 1
    assert mism[0] == 0
    assert 0 < mism[1] < 20000 and 0 < mism[2] < 20000


def test_q16_grey_axis_identity():
    y = np.arange(256)
    out = colour.rgb_q16_samples(y, np.full(256, 128), np.full(256, 128))
    assert np.array_equal(out, np.stack([y, y, y]))
    outf = colour.rgb_real_samples(y, np.full(256, 128.0), np.full(256, 128.0))
    assert np.array_equal(outf, np.stack([y, y, y]).astype(float))


def test_upsample_is_nearest():
    c = np.arange(6).reshape(2, 3)
    u = colour.upsample2(c)
    for i in range(4):
        for j in range(6):
            assert u[i, j] == c[i >> 1, j >> 1]


W, H, T = 8192, 8192, 512


def test_viewport_fraction_matches_about_twelve_percent():
    """A one-eye 110x110 degree viewport touches about 12 % of the 256 tiles."""
    counts = []
    for gop in range(48):
        yaw, pitch = wvinputs.head_pose(wvinputs.BASE_SEED, gop)
        m = viewport.tile_mask(W, H, T, yaw, pitch)
        assert m[128:].sum() == 0          # bottom eye never in a one-eye viewport
        counts.append(int(m.sum()))
    frac = np.mean(counts) / 256
    assert 0.10 < frac < 0.17, frac
    assert min(counts) >= 24 and max(counts) <= 48


def test_viewport_contains_view_direction_and_not_its_antipode():
    for yaw, pitch in [(0.0, 0.0), (33.0, 12.0), (-150.0, -25.0), (179.0, 5.0)]:
        m = viewport.tile_mask(W, H, T, yaw, pitch)
        lon = (yaw + 180.0) / 360.0 * W
        lat = (90.0 - pitch) / 180.0 * (H / 2)
        tx, ty = int(lon // T) % 16, int(lat // T)
        assert m[ty * 16 + tx] == 1
        alon = ((yaw + 360.0) % 360.0) / 360.0 * W
        alat = (90.0 + pitch) / 180.0 * (H / 2)
        assert m[int(alat // T) * 16 + int(alon // T) % 16] == 0


def test_viewport_symmetries():
    """yaw -> -yaw mirrors tile columns; pitch -> -pitch mirrors the eye's tile
    rows; yaw + 22.5 degrees (one tile) rolls the columns by one."""
    for yaw, pitch in [(10.0, 7.0), (-63.0, 21.0), (100.0, -13.0)]:
        m = viewport.tile_mask(W, H, T, yaw, pitch).reshape(16, 16)[:8]
        mm = viewport.tile_mask(W, H, T, -yaw, pitch).reshape(16, 16)[:8]
        assert np.array_equal(m, mm[:, ::-1])
        mp = viewport.tile_mask(W, H, T, yaw, -pitch).reshape(16, 16)[:8]
        assert np.array_equal(m, mp[::-1, :])
        mr = viewport.tile_mask(W, H, T, yaw + 22.5, pitch).reshape(16, 16)[:8]
        assert np.array_equal(np.roll(m, 1, axis=1), mr)


def test_viewport_two_eyes_is_union_of_halves():
    m1 = viewport.tile_mask(W, H, T, 40.0, 10.0, eyes=1)
    m2 = viewport.tile_mask(W, H, T, 40.0, 10.0, eyes=2)
    assert np.array_equal(m2[:128], m1[:128])
    assert np.array_equal(m2[128:], m1[:128])


def test_foveation_bands_and_data_saving():
    """The tiles around the gaze keep all levels; the coefficient bytes kept by a
    4-level foveated viewport are well under a third of the full viewport, in line
    with the paper's 'up to 80 % less data' (Section 3.7)."""
    kept = []
    for gop in range(24):
        yaw, pitch = wvinputs.head_pose(wvinputs.BASE_SEED, gop)
        m = viewport.tile_mask(W, H, T, yaw, pitch).astype(bool)
        drop = viewport.foveation_drop(W, H, T, yaw, pitch)
        assert set(np.unique(drop)) <= {0, 1, 2}
        lon = (yaw + 180.0) / 360.0 * W
        lat = (90.0 - pitch) / 180.0 * (H / 2)
        assert drop[int(lat // T) * 16 + int(lon // T) % 16] == 0
        frac = (1.0 / 4.0 ** drop[m].astype(float)).sum() / m.sum()
        kept.append(frac)
    assert 0.08 < np.mean(kept) < 0.33


def test_foveation_centre_of_straight_view():
    d = viewport.foveation_drop(W, H, T, 0.0, 0.0).reshape(16, 16)
    assert d[3, 7] == d[3, 8] == d[4, 7] == d[4, 8] == 0
    assert d[4, 0] == 2 and d[0, 8] == 2
