"""Pins of the paper-format oracle (oracle/paperformat.py): the threshold of
Eq. 2/3 with the pole factor of Section 3.6 at closed-form points, the
level-wise block order of Section 3.4, the Eq. 4 round-trip bound, the
lossless limit, the foveated prefix property and the rebuild + decode
composition.
"""
import numpy as np
import pytest

from oracle import codec, paperformat as pf
from oracle.wavelet import W53, W97, fwd2d


def test_block_order_is_level_wise_from_the_lowest_frequency():
    p, levels = 512, 5
    order = pf.block_order(p, levels)
    assert len(order) == 256 and len(set(order)) == 256
    lev = [pf.block_level(p, levels, *b) for b in order]
    assert lev == sorted(lev, reverse=True)
    # 1 block holding the approximation (with levels 5's details), then 3, 12, 48, 192
    assert [lev.count(k) for k in (6, 4, 3, 2, 1)] == [1, 3, 12, 48, 192]
    assert order[0] == (0, 0)
    # every coefficient of a detail block belongs to that block's level
    cl = pf.coefficient_level(p, levels)
    for (by, bx), k in zip(order, lev):
        blk = cl[by * 32:(by + 1) * 32, bx * 32:(bx + 1) * 32]
        if k <= levels:
            assert np.all(blk == k)
        else:
            assert blk[0, 0] == 0 and blk.max() <= levels


def test_small_planes_are_one_block():
    assert pf.block_order(16, 2) == [(0, 0)]
    assert pf.block_size(16) == 16


def test_threshold_closed_forms():
    """Eq. 3 at the finest and coarsest detail level; H = 0 at the equator
    of each eye and close to 1 at the poles; the approximation is exempt."""
    p, levels, alpha = 64, 3, 0.25
    # a 2 x 2-tile plane: two tile rows, so plane height 128, eye height 64
    thr = pf.thresholds(p, levels, 2, 128, alpha, poles=False)
    lev = pf.coefficient_level(p, levels)
    assert np.all(thr[:, lev == 1] == alpha)
    assert np.allclose(thr[:, lev == 3], alpha / 9.0)
    assert np.allclose(thr[:, lev == 2], alpha * (2.0 / 3.0) ** 2)
    assert np.all(thr[:, lev == 0] == -1.0)
    thp = pf.thresholds(p, levels, 2, 128, alpha, poles=True)
    rows = pf.coefficient_rows(p, levels)
    # level-1 coefficient centred on eye row 32 (the equator of a 64-row eye)
    y, x = np.argwhere((lev == 1) & (rows == 33.0))[0]
    assert thp[0, y, x] == pytest.approx(alpha + 1 - np.sin(np.pi * 33 / 64))
    y0, x0 = np.argwhere((lev == 1) & (rows == 1.0))[0]
    assert thp[0, y0, x0] == pytest.approx(alpha + 1 - np.sin(np.pi / 64))
    # the second tile row is the second eye: same thresholds
    assert np.array_equal(thp[0], thp[2]) and np.array_equal(thp[1], thp[3])


def test_keep_rule_is_strictly_above_the_threshold():
    p, levels = 32, 2
    c = np.zeros((1, p, p), np.float32)
    lev = pf.coefficient_level(p, levels)
    ys, xs = np.nonzero(lev == 1)
    alpha = 0.1
    c[0, ys[0], xs[0]] = 0.1 * 255          # exactly at T: dropped
    c[0, ys[1], xs[1]] = 0.1 * 255 + 0.01   # just above: kept
    c[0, ys[2], xs[2]] = -30.0              # |c| / 255 = 0.118 > 0.1: kept
    fmt = pf.encode_plane(c, levels, 1, p, alpha, poles=False)
    n_approx = int(np.count_nonzero(lev == 0))
    assert fmt["values"].size == n_approx + 2


def test_eq4_round_trip_bound_and_lossless_limit():
    rng = np.random.default_rng(4)
    c = rng.normal(0, 20, (2, 64, 64)).astype(np.float32)
    fmt = pf.encode_plane(c, 3, 2, 64, 0.0, poles=False)     # T = 0: every non-zero kept
    assert fmt["values"].size == np.count_nonzero(c) + 0
    dense = pf.rebuild_plane(fmt, 64, 3, [0, 1], 3, W97)
    amin, amax, dmin, dmax = fmt["bounds"]
    lev = pf.coefficient_level(64, 3)
    step_a = (float(amax) - float(amin)) / 255
    step_d = (float(dmax) - float(dmin)) / 255
    err = np.abs(dense.astype(np.float64) - c)
    assert err[:, lev == 0].max() <= step_a / 2 * (1 + 1e-5) + 1e-4
    assert err[:, lev > 0].max() <= step_d / 2 * (1 + 1e-5) + 1e-4
    # a plane with two values per class is rebuilt exactly
    c2 = np.where(lev == 0, 7.0, np.where(lev % 2 == 1, -3.0, 5.0)).astype(np.float32)[None]
    f2 = pf.encode_plane(c2, 3, 1, 64, 0.0, poles=False)
    assert np.array_equal(pf.rebuild_plane(f2, 64, 3, [0], 3, W97), c2)


def test_records_are_counted_by_block_end_and_indices_in_range():
    rng = np.random.default_rng(8)
    c = rng.laplace(0, 12, (4, 64, 64)).astype(np.float32)
    fmt = pf.encode_plane(c, 4, 2, 128, 0.05, poles=True)
    be = fmt["block_end"]
    assert be.size == 4 * 4 and np.all(np.diff(be.astype(np.int64)) >= 0)
    assert int(be[-1]) == fmt["values"].size == fmt["index"].size
    assert fmt["index"].max() < 32 * 32


def test_foveated_records_are_a_prefix_of_the_tile():
    """Blocks of the dropped finest levels are the tile's trailing records, so a
    foveated read is one shorter contiguous range (Sections 3.4, 3.7)."""
    p, levels = 128, 3
    order = pf.block_order(p, levels)
    lev = [pf.block_level(p, levels, *b) for b in order]
    for drop in range(levels + 1):
        kept = [k > drop for k in lev]
        assert kept == sorted(kept, reverse=True)


def test_rebuild_and_decode_equal_the_intra_decode_of_the_rebuilt_plane():
    rng = np.random.default_rng(12)
    levels = 3
    src = rng.integers(0, 256, (4, 64, 64))
    c = fwd2d(src, levels, W97).astype(np.float32)
    fmt = pf.encode_plane(c, levels, 2, 128, 0.02, poles=True)
    mask = np.array([1, 0, 1, 1], np.uint8)
    lc = np.array([3, 3, 2, 1])
    vis, out, rec, dense = pf.decode_viewport([fmt], [64], mask, levels, W97, lc)
    want = codec.decode_tiles([{"coeffs": [dense[0]], "step": 1, "intra": True,
                                "level_count": lc[vis]}], levels, W97)[0]
    assert np.array_equal(vis, [0, 2, 3])
    assert np.array_equal(out, want["out"])
    # 5/3 dense planes are the nearest integers of the float32 values
    d53 = pf.rebuild_plane(fmt, 64, levels, vis, lc, W53)
    d97 = pf.rebuild_plane(fmt, 64, levels, vis, lc, W97)
    assert np.array_equal(d53, np.rint(d97).astype(np.int16))


def test_thresholding_shrinks_the_store_and_keeps_quality():
    """Higher alpha keeps fewer coefficients; alpha = 0.1 (the paper's HQ
    setting) on a smooth synthetic plane still decodes close to the source."""
    levels = 3
    yy, xx = np.mgrid[0:128, 0:128]
    src = (128 + 60 * np.sin(xx / 9.0) * np.cos(yy / 13.0)).reshape(1, 128, 128)
    c = fwd2d(src, levels, W97).astype(np.float32)
    sizes = [pf.encode_plane(c, levels, 1, 128, a, poles=False)["values"].size
             for a in (0.0, 0.01, 0.1, 0.25)]
    assert sizes == sorted(sizes, reverse=True) and sizes[-1] < sizes[0] / 4
    fmt = pf.encode_plane(c, levels, 1, 128, 0.1, poles=False)
    dense = pf.rebuild_plane(fmt, 128, levels, [0], levels, W97)
    rec = codec.decode_tiles([{"coeffs": [dense], "step": 1, "intra": True}], levels, W97)[0]["rec"][0]
    mse = np.mean((rec - np.clip(src, 0, 255)) ** 2)
    assert 10 * np.log10(255 ** 2 / mse) > 30
