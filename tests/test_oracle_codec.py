"""Pins of the oracle's quantiser and decode chain."""
import numpy as np
import pytest

import wvinputs
from oracle import codec, wavelet as wv


def test_quantiser_values_and_error_bound():
    c = np.array([-6, -5, -3, -2, -1, 0, 1, 2, 3, 5, 6])
    assert codec.quantise_int(c, 4).tolist() == [-2, -1, -1, -1, 0, 0, 0, 1, 1, 1, 2]
    rng = np.random.default_rng(2)
    for step in (1, 2, 3, 4, 7, 16):
        c = rng.integers(-5000, 5000, 4000)
        q = codec.quantise_int(c, step)
        assert np.all(np.abs(c - step * q) * 2 <= step)
        f = rng.normal(0, 300, 4000)
        g = codec.quantise_float(f, float(step))
        assert np.all(np.abs(f - g) <= step / 2 + 1e-9)
        assert np.allclose(g / step, np.rint(g / step))


def _small_gop(wavelet, n_frames=4, tile=32, levels=3, seed=3, clip_free=False):
    spec = wvinputs.FrameSpec(128, 128, tile, seed)
    src = [p.numpy().reshape(-1, *p.shape[2:]) for p in wvinputs.source_planes(spec)]
    if clip_free:
        src = [np.full_like(p, 128) + (p.astype(np.int64) % 17 - 8).astype(p.dtype) for p in src]
    frames = [{"coeffs": codec.encode_intra(src, levels, wavelet, 4 if wavelet == wv.W53 else 8),
               "step": 4, "intra": True, "level_count": levels}]
    for t in range(1, n_frames):
        res = wvinputs.residual_planes(spec, t, integer=(wavelet == wv.W53),
                                       scale=0.25 if clip_free else 2.0)
        frames.append({"coeffs": [r.numpy().reshape(-1, *r.shape[2:]) for r in res],
                       "step": 1, "intra": False, "level_count": levels})
    return spec, src, frames


def test_chain_closed_form_without_clipping_53():
    """With no clipping active, rec_t = P_0 + sum of the residual syntheses."""
    _, _, frames = _small_gop(wv.W53, clip_free=True)
    res = codec.decode_tiles(frames, 3, wv.W53)
    acc = None
    for f, r in zip(frames, res):
        p = [wv.inv2d(np.asarray(q, np.int64) * f["step"], 3, wv.W53) for q in f["coeffs"]]
        acc = p if acc is None else [a + b for a, b in zip(acc, p)]
        assert all(np.array_equal(a, b) for a, b in zip(acc, r["rec"]))
        assert all((a.min() > 0 and a.max() < 255) for a in acc)


def test_chain_linearity_97():
    """9/7 synthesis is linear: with no clipping active, rec_t equals the inverse
    transform of the summed coefficients of frames 0..t."""
    _, _, frames = _small_gop(wv.W97, clip_free=True)
    res = codec.decode_tiles(frames, 3, wv.W97)
    csum = None
    for f, r in zip(frames, res):
        c = [np.asarray(q, np.float64) for q in f["coeffs"]]
        csum = c if csum is None else [a + b for a, b in zip(csum, c)]
        want = [wv.inv2d(a, 3, wv.W97) for a in csum]
        assert all(a.min() > 0 and a.max() < 255 for a in want)
        assert max(np.max(np.abs(a - b)) for a, b in zip(want, r["rec"])) < 1e-9


def test_intra_lossless_at_step_one_53():
    spec, src, _ = _small_gop(wv.W53)
    coeffs = codec.encode_intra(src, 3, wv.W53, 1)
    res = codec.decode_tiles([{"coeffs": coeffs, "step": 1, "intra": True}], 3, wv.W53)
    for a, b in zip(res[0]["rec"], src):
        assert np.array_equal(a, b.astype(np.int64))


def test_intra_quantised_error_is_small_53():
    spec, src, frames = _small_gop(wv.W53)
    res = codec.decode_tiles(frames[:1], 3, wv.W53)
    err = np.abs(res[0]["rec"][0] - src[0].astype(np.int64))
    assert err.mean() < 4.0


def test_viewport_restriction_equals_full_decode_crop():
    """Decoding only the union of the masks gives, tile for tile, the full-frame
    decode restricted to each mask (tiles are independent)."""
    spec, src, frames = _small_gop(wv.W53, n_frames=5)
    n = spec.n_tiles
    rng = np.random.default_rng(9)
    masks = [(rng.random(n) < 0.4).astype(np.uint8) for _ in frames]
    for f in frames:
        f["level_count"] = rng.integers(1, 4, n)
    full = codec.decode_tiles(frames, 3, wv.W53)
    vp = codec.decode_viewport_gop(frames, masks, 3, wv.W53)
    for m, fr, (vis, out, rec) in zip(masks, full, vp):
        assert np.array_equal(vis, np.nonzero(m)[0])
        assert np.array_equal(out, fr["out"][vis])
        for a, b in zip(rec, fr["rec"]):
            assert np.array_equal(a, b[vis])


def test_foveated_decode_is_decode_of_zeroed_coefficients():
    spec, src, frames = _small_gop(wv.W97, n_frames=3)
    n = spec.n_tiles
    lc = np.array([3, 2, 1, 0] * (n // 4))
    for f in frames:
        f["level_count"] = lc
    got = codec.decode_tiles(frames, 3, wv.W97)
    zeroed = []
    for f in frames:
        planes = []
        for q in f["coeffs"]:
            q = np.array(q, dtype=np.float64)
            for i in range(n):
                q[i] = wv.zero_finest(q[i], 3 - lc[i])
            planes.append(q)
        zeroed.append(dict(f, coeffs=planes, level_count=3))
    want = codec.decode_tiles(zeroed, 3, wv.W97)
    for a, b in zip(got, want):
        assert np.max(np.abs(a["out"] - b["out"])) == 0.0
    # level_count 0 leaves only the approximation band: a tile of zero details
    assert np.all(np.isfinite(got[-1]["out"]))


def _ll_only(levels, tile, value, dtype):
    """A tile plane whose approximation band is the constant ``value`` and
    whose detail bands are zero (Mallat layout: the band sits top-left)."""
    c = np.zeros((1, tile, tile), dtype)
    n = tile >> levels
    c[0, :n, :n] = value
    return c


@pytest.mark.parametrize("wavelet", [wv.W53, wv.W97])
def test_chain_clips_the_reference_closed_loop(wavelet):
    """The residual chain clips the reference it carries forward.

    With zero details, the synthesis of a constant approximation is that
    constant (DC gain 1 of both lifting schemes).  Intra 250, then +10, then
    -10: the second frame clips to 255, and the third is 255 - 10 = 245 -- an
    open-loop chain (clip only on output, P_0 + sum of residuals carried
    unclipped) would give 250.  The same at the bottom of the range: 5, -10,
    +10 gives 0, then 10 (open loop: 5).  Every plane of a YUV420 frame
    follows its own chain."""
    L, P = 3, 32
    dt = np.int16 if wavelet == wv.W53 else np.float32
    for start, steps, want in ((250, (10, -10, -10), (255, 245, 235)),
                               (5, (-10, 10, 3), (0, 10, 13))):
        frames = [{"coeffs": [_ll_only(L, P, start, dt), _ll_only(L, P // 2, start, dt),
                              _ll_only(L, P // 2, 255 - start, dt)],
                   "step": 1, "intra": True, "level_count": L}]
        for d in steps:
            frames.append({"coeffs": [_ll_only(L, P, d, dt), _ll_only(L, P // 2, d, dt),
                                      _ll_only(L, P // 2, -d, dt)],
                           "step": 1, "intra": False, "level_count": L})
        res = codec.decode_tiles(frames, L, wavelet)
        y0, cb0, cr0 = (np.asarray(p) for p in res[0]["rec"])
        assert np.allclose(y0, start, atol=1e-9) and np.allclose(cb0, start, atol=1e-9)
        assert np.allclose(cr0, 255 - start, atol=1e-9)
        for r, w in zip(res[1:], want):
            y, cb, cr = (np.asarray(p) for p in r["rec"])
            assert np.allclose(y, w, atol=1e-9), (start, w, float(y.mean()))
            assert np.allclose(cb, w, atol=1e-9)
            assert np.allclose(cr, 255 - w, atol=1e-9)


def test_chain_clip_with_dequantisation_step():
    """The step multiplies the stored indices before the chain: intra 62 * 4
    = 248, then +3 * 4 = 260 -> 255, then -2 * 4 -> 247 (5/3, grey)."""
    L, P = 2, 16
    frames = [{"coeffs": [_ll_only(L, P, 62, np.int16)], "step": 4, "intra": True},
              {"coeffs": [_ll_only(L, P, 3, np.int16)], "step": 4, "intra": False},
              {"coeffs": [_ll_only(L, P, -2, np.int16)], "step": 4, "intra": False}]
    res = codec.decode_tiles(frames, L, wv.W53)
    assert [int(r["out"].max()) for r in res] == [248, 255, 247]
    assert [int(r["out"].min()) for r in res] == [248, 255, 247]
