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


# JFIF forward conversion (RGB -> YCbCr, full range), written out independently
# of the oracle's inverse so that composing the two pins the inverse's constants.
JFIF_FWD = np.array([[0.299, 0.587, 0.114],
                     [-0.168736, -0.331264, 0.5],
                     [0.5, -0.418688, -0.081312]])
JFIF_OFF = np.array([0.0, 128.0, 128.0])


def _inverse_affine(fn):
    """The affine map (matrix, offset) that ``fn`` applies to in-range
    (Y, Cb, Cr) samples, read off by unit steps around the grey point."""
    c = np.array([128.0, 128.0, 128.0])
    base = fn(*[np.array([v]) for v in c])[:, 0].astype(np.float64)
    m = np.zeros((3, 3))
    for j in range(3):
        e = c.copy()
        e[j] += 1.0
        m[:, j] = fn(*[np.array([v]) for v in e])[:, 0] - base
    return m, base - m @ c


def test_real_inverse_composed_with_jfif_forward_is_identity():
    """The oracle's inverse undoes the JFIF forward matrix: a Cb/Cr swap, a
    sign flip or a wrong constant in the inverse breaks this."""
    m, off = _inverse_affine(colour.rgb_real_samples)
    assert np.max(np.abs(m @ JFIF_FWD - np.eye(3))) < 1e-5
    assert np.max(np.abs(m @ JFIF_OFF + off)) < 1e-3
    rng = np.random.default_rng(7)
    rgb = rng.uniform(1.0, 254.0, (3, 5000))
    ycc = JFIF_FWD @ rgb + JFIF_OFF[:, None]
    back = colour.rgb_real_samples(ycc[0], ycc[1], ycc[2])
    assert np.max(np.abs(back - rgb)) < 2e-3


def test_pure_primaries_round_trip():
    """Pure red, green, blue (and black, white) through the JFIF forward
    matrix and back: exact to rounding in the real path; within 2 in the
    Q16 path after the forward values are rounded to 8-bit samples."""
    prim = np.array([[255, 0, 0], [0, 255, 0], [0, 0, 255], [0, 0, 0], [255, 255, 255],
                     [255, 255, 0], [0, 255, 255], [255, 0, 255]], np.float64).T
    ycc = JFIF_FWD @ prim + JFIF_OFF[:, None]
    back = colour.rgb_real_samples(ycc[0], ycc[1], ycc[2])
    assert np.max(np.abs(back - prim)) < 1e-2
    q = np.clip(np.floor(ycc + 0.5), 0, 255).astype(np.int64)
    backq = colour.rgb_q16_samples(q[0], q[1], q[2])
    assert np.max(np.abs(backq - prim)) <= 2
    # the dominant channel of each primary stays at the top of the range
    for k in range(3):
        assert backq[k, k] >= 253 and all(backq[j, k] <= 2 for j in range(3) if j != k)


def test_q16_inverse_composed_with_jfif_forward():
    """The Q16 constants, read as a matrix (constant / 65536), undo the JFIF
    forward matrix to within their own rounding (1 / 131072 per entry)."""
    q = colour.Q16
    m = np.array([[65536, 0, q["r_cr"]], [65536, q["g_cb"], q["g_cr"]],
                  [65536, q["b_cb"], 0]], np.float64) / 65536
    assert np.max(np.abs(m @ JFIF_FWD - np.eye(3))) < 4e-5
