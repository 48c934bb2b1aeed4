"""GPU parity: the HIP decode (through the C ABI) against the CPU oracle.

5/3 must be bit-exact (outputs and reference planes); 9/7 within max-abs 1e-3
on the 0..255 scale.  Inputs are seeded synthetic GOPs (tests/gop.py).
"""
import numpy as np
import pytest
import torch

import wvinputs
from gop import Gop, W53, W97, pose_mask
from oracle import viewport

pytestmark = pytest.mark.gpu

TOL97 = 1e-3


def _wv():
    from paper_2208_10859_amd import wv
    return wv


def _dev(planes, dtype):
    return [torch.from_numpy(np.ascontiguousarray(p)).to("cuda") for p in planes]


def _run_gop(dec, gop, masks, level_counts=None, out_every=True):
    """Decode a GOP frame by frame on the GPU; return per-frame (out, ref planes)."""
    wv = _wv()
    ref = wv.Reference(dec)
    res = []
    for t, f in enumerate(gop.frames):
        planes = _dev(f["coeffs"], dec.coef_dtype)
        nvis = int(np.count_nonzero(masks[t]))
        out = torch.full(dec.out_shape(nvis), 77, dtype=dec.sample_dtype, device="cuda") \
            if out_every else None
        lc = None if level_counts is None else level_counts[t]
        dec.decode_viewport(planes, t, f["intra"], f["step"], masks[t], ref, out, lc)
        torch.cuda.synchronize()
        res.append((None if out is None else out.cpu().numpy(),
                    [p.cpu().numpy() for p in ref.planes], ref.stamp.copy()))
    return res


def _named(name, fn, *args, **kw):
    """Run a comparison, naming the fused variant if it fails."""
    try:
        return fn(*args, **kw)
    except AssertionError as e:
        raise AssertionError(f"variant {name}: {e}") from None


def _compare(gop, res, masks, want, exact, level_counts=None):
    worst = 0.0
    for t, ((out, ref, stamp), (vis, wout, wrec)) in enumerate(zip(res, want)):
        assert np.array_equal(vis, np.nonzero(masks[t])[0])
        if exact:
            assert out.dtype == np.uint8
            assert np.array_equal(out, wout), f"frame {t}: output differs"
            for p, (r, w) in enumerate(zip(ref, wrec)):
                assert np.array_equal(r[vis], w), f"frame {t} plane {p}: reference differs"
        else:
            worst = max(worst, float(np.max(np.abs(out.astype(np.float64) - wout))))
            for r, w in zip(ref, wrec):
                worst = max(worst, float(np.max(np.abs(r[vis].astype(np.float64) - w))))
        assert np.all(stamp[vis] == t)
    return worst


# --------------------------------------------------------------- config 1
def test_config1_gray_512_three_levels_bitexact():
    """512x512 8-bit luma, 3-level 5/3, step 4, intra, full frame."""
    wv = _wv()
    gop = Gop(512, 512, 512, 3, W53, 1, seed=wvinputs.BASE_SEED + 1, chroma=False)
    masks = [np.ones(1, np.uint8)]
    want = gop.oracle(masks)
    for path in (wv.PATH_FUSED, wv.PATH_PLAIN):
        dec = wv.Decoder(512, 512, 512, 3, wv.W53, wv.GRAY8)
        dec.set_path(path)
        res = _run_gop(dec, gop, masks)
        _compare(gop, res, masks, want, exact=True)
    # every fused variant
    dec = wv.Decoder(512, 512, 512, 3, wv.W53, wv.GRAY8)
    assert dec.variants()[dec.variant].startswith("strip_")
    tried = 0
    for v, name in enumerate(dec.variants()):
        try:
            dec.variant = v
        except wv.WvError:
            continue            # compiled for another level count, or too large
        tried += 1
        res = _run_gop(dec, gop, masks)
        _named(name, _compare, gop, res, masks, want, exact=True)
    assert tried >= 8


# ------------------------------------------------- small multi-tile GOPs
@pytest.mark.parametrize("wavelet", [W53, W97])
@pytest.mark.parametrize("tile,levels", [(32, 3), (64, 5), (16, 2)])
def test_small_gop_every_variant_and_path(wavelet, tile, levels):
    wv = _wv()
    W, H = tile * 4, tile * 3
    gop = Gop(W, H, tile, levels, wavelet, 4, seed=31 + tile + levels)
    n = gop.spec.n_tiles
    rng = np.random.default_rng(tile + 7 * levels)
    masks = [np.ones(n, np.uint8)] * 4
    lcs = [rng.integers(0, levels + 1, n).astype(np.uint8) for _ in range(4)]
    want = gop.oracle(masks, lcs)
    wl = wv.W53 if wavelet == W53 else wv.W97
    dec = wv.Decoder(W, H, tile, levels, wl, wv.YUV420)
    tried = 0
    for v in range(len(dec.variants())):
        try:
            dec.variant = v
        except wv.WvError:
            continue            # variant block larger than the tile
        tried += 1
        res = _run_gop(dec, gop, masks, lcs)
        worst = _compare(gop, res, masks, want, exact=(wavelet == W53), level_counts=lcs)
        assert worst <= TOL97
    assert tried >= 1
    dec.set_path(wv.PATH_PLAIN)
    res = _run_gop(dec, gop, masks, lcs)
    assert _compare(gop, res, masks, want, exact=(wavelet == W53)) <= TOL97


def test_empty_mask_is_a_noop_and_ragged_masks():
    wv = _wv()
    gop = Gop(128, 96, 32, 3, W53, 3, seed=5)
    n = gop.spec.n_tiles
    dec = wv.Decoder(128, 96, 32, 3, wv.W53, wv.YUV420)
    ref = wv.Reference(dec)
    planes = _dev(gop.frames[0]["coeffs"], dec.coef_dtype)
    before = [p.clone() for p in ref.planes]
    dec.decode_viewport(planes, 0, True, 4, np.zeros(n, np.uint8), ref, None)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(before, ref.planes))
    assert np.all(ref.stamp == -1)
    # single tile, last tile, all tiles
    for m in ([n - 1], [0], list(range(n))):
        mask = np.zeros(n, np.uint8)
        mask[m] = 1
        masks = [mask] * 3
        res = _run_gop(dec, gop, masks)
        _compare(gop, res, masks, gop.oracle(masks), exact=True)


def test_catch_up_of_newly_visible_tiles():
    """Viewport moves during the GOP: tiles entering the view are replayed
    (out = NULL) from their last decoded frame; the result equals the full
    decode restricted to the masks."""
    wv = _wv()
    gop = Gop(256, 128, 32, 3, W53, 6, seed=8)
    n = gop.spec.n_tiles
    rng = np.random.default_rng(4)
    masks = [(rng.random(n) < 0.45).astype(np.uint8) for _ in range(6)]
    masks[0][:] = masks[0] | masks[1]
    want = gop.oracle(masks)
    dec = wv.Decoder(256, 128, 32, 3, wv.W53, wv.YUV420)
    ref = wv.Reference(dec)
    dev_frames = [_dev(f["coeffs"], dec.coef_dtype) for f in gop.frames]
    for t, f in enumerate(gop.frames):
        if not f["intra"]:
            stale = (masks[t] > 0) & (ref.stamp != t - 1)
            # replay every stale tile from the frame after its stamp (the intra
            # frame if it was never decoded), without output
            for s in range(t):
                need = stale & (ref.stamp == s - 1)
                if need.any():
                    g = gop.frames[s]
                    dec.decode_viewport(dev_frames[s], s, g["intra"], g["step"],
                                        need.astype(np.uint8), ref, None)
        nvis = int(masks[t].sum())
        out = torch.zeros(dec.out_shape(nvis), dtype=torch.uint8, device="cuda")
        dec.decode_viewport(dev_frames[t], t, f["intra"], f["step"], masks[t], ref, out)
        torch.cuda.synchronize()
        vis, wout, wrec = want[t]
        assert np.array_equal(out.cpu().numpy(), wout)


def test_errors_leave_state_untouched():
    wv = _wv()
    gop = Gop(64, 64, 32, 3, W53, 2, seed=2)
    n = gop.spec.n_tiles
    dec = wv.Decoder(64, 64, 32, 3, wv.W53, wv.YUV420)
    ref = wv.Reference(dec)
    planes = _dev(gop.frames[1]["coeffs"], dec.coef_dtype)
    mask = np.ones(n, np.uint8)
    with pytest.raises(wv.WvError) as e:
        dec.decode_viewport(planes, 1, False, 1, mask, ref, None)
    assert e.value.status == wv.ESTALE
    assert np.all(ref.stamp == -1)
    with pytest.raises(wv.WvError) as e:
        dec.decode_viewport(planes, 0, True, 0, mask, ref, None)
    assert e.value.status == wv.EINVAL
    with pytest.raises(wv.WvError) as e:
        dec.decode_viewport(planes, 0, True, 4, mask, ref, None, level_count=np.full(n, 4))
    assert e.value.status == wv.EINVAL
    need = int(n) * 3 * 32 * 32
    bad = torch.zeros(need + 16, dtype=torch.uint8, device="cuda")[1:]     # misaligned
    with pytest.raises(wv.WvError) as e:
        dec.decode_viewport(planes, 0, True, 4, mask, ref, bad)
    assert e.value.status == wv.EINVAL
    assert np.all(ref.stamp == -1)


# ----------------------------------------------- full-size configurations
def _full_gop(wavelet, levels, gop_index, foveate):
    W = H = 8192
    mask, (yaw, pitch) = pose_mask(W, H, 512, wvinputs.BASE_SEED, gop_index)
    vis = np.nonzero(mask)[0]
    gop = Gop(W, H, 512, levels, wavelet, 8, seed=wvinputs.BASE_SEED + 2 + gop_index, tiles=vis)
    lcs = None
    if foveate:
        lc = levels - viewport.foveation_drop(W, H, 512, yaw, pitch)
        lcs = [lc.astype(np.uint8)] * 8
    return gop, [mask] * 8, lcs


def test_config2_full_gop_bitexact():
    """8192x8192 YUV420, 5-level 5/3 on 512x512 tiles, GOP of 8, one-eye
    110x110 degree viewport at a seeded pose: every visible tile of every frame,
    RGB and reference planes, bit-exact; plain and fused forms agree."""
    wv = _wv()
    gop, masks, _ = _full_gop(W53, 5, 0, False)
    want = gop.oracle(masks)
    dec = wv.Decoder(8192, 8192, 512, 5, wv.W53, wv.YUV420)
    res = _run_gop(dec, gop, masks)
    _compare(gop, res, masks, want, exact=True)
    assert dec.variants()[dec.variant].startswith("strip_")
    for v, name in enumerate(dec.variants()):     # every variant that fits this geometry
        try:
            dec.variant = v
        except wv.WvError:
            continue
        _named(name, _compare, gop, _run_gop(dec, gop, masks), masks, want, exact=True)
    dec.set_path(wv.PATH_PLAIN)
    res2 = _run_gop(dec, gop, masks)
    for a, b in zip(res, res2):
        assert np.array_equal(a[0], b[0])


def test_config3_full_gop_foveated_97_within_tolerance():
    """Same frames with the 4-level CDF 9/7 in FP32, step 8, foveated decode
    (0/1/2 levels dropped at <=20, <=40, >40 degrees): max-abs <= 1e-3."""
    wv = _wv()
    gop, masks, lcs = _full_gop(W97, 4, 1, True)
    want = gop.oracle(masks, lcs)
    dec = wv.Decoder(8192, 8192, 512, 4, wv.W97, wv.YUV420)
    res = _run_gop(dec, gop, masks, lcs)
    worst = _compare(gop, res, masks, want, exact=False, level_counts=lcs)
    assert worst <= TOL97, worst
    for v, name in enumerate(dec.variants()):
        try:
            dec.variant = v
        except wv.WvError:
            continue
        w = _named(name, _compare, gop, _run_gop(dec, gop, masks, lcs), masks, want,
                   exact=False, level_counts=lcs)
        assert w <= TOL97, (name, w)
    dec.set_path(wv.PATH_PLAIN)
    res2 = _run_gop(dec, gop, masks, lcs)
    assert _compare(gop, res2, masks, want, exact=False, level_counts=lcs) <= TOL97


def _run_gop_fused(dec, gop, mask, level_counts=None):
    """The whole GOP through wv_decode_gop (one launch with a strip variant)."""
    wv = _wv()
    ref = wv.Reference(dec)
    frames = [(_dev(f["coeffs"], dec.coef_dtype), f["intra"], f["step"]) for f in gop.frames]
    nvis = int(np.count_nonzero(mask))
    outs = [torch.full(dec.out_shape(nvis), 77, dtype=dec.sample_dtype, device="cuda")
            for _ in frames]
    dec.decode_gop(frames, 0, mask, ref, outs, level_counts)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs], [p.cpu().numpy() for p in ref.planes], ref.stamp.copy()


@pytest.mark.parametrize("wavelet,levels,foveate", [(W53, 5, False), (W53, 4, True), (W97, 4, True)])
def test_gop_form_equals_oracle(wavelet, levels, foveate):
    """wv_decode_gop (every tile strip taken through all frames in one launch)
    on the full 8192^2 GOPs: 5/3 bit-exact, 9/7 foveated within 1e-3, for every
    strip variant; the last reference equals the oracle's."""
    wv = _wv()
    gop, masks, lcs = _full_gop(wavelet, levels, 0 if wavelet == W53 else 1, foveate)
    want = gop.oracle(masks, lcs)
    wl = wv.W53 if wavelet == W53 else wv.W97
    dec = wv.Decoder(8192, 8192, 512, levels, wl, wv.YUV420)
    vis = np.nonzero(masks[0])[0]
    tried = 0
    for v, name in enumerate(dec.variants()):
        if not name.startswith("strip_"):
            continue
        try:
            dec.variant = v
        except wv.WvError:
            continue
        tried += 1
        outs, ref, stamp = _run_gop_fused(dec, gop, masks[0], None if lcs is None else lcs[0])
        assert np.all(stamp[vis] == len(gop.frames) - 1)
        for t, (out, (wvis, wout, wrec)) in enumerate(zip(outs, want)):
            if wavelet == W53:
                assert np.array_equal(out, wout), f"{name}: frame {t} differs"
            else:
                assert np.max(np.abs(out.astype(np.float64) - wout)) <= TOL97, (name, t)
        for r, w in zip(ref, want[-1][2]):
            if wavelet == W53:
                assert np.array_equal(r[vis], w), name
            else:
                assert np.max(np.abs(r[vis].astype(np.float64) - w)) <= TOL97, name
    assert tried >= 3


def test_gop_form_longer_than_one_launch():
    """A 12-frame GOP in one wv_decode_gop call: the strip kernels take it in
    launches of up to 8 frames, the reference carried between them; every
    frame equals the oracle for every row-strip variant."""
    wv = _wv()
    gop = Gop(1024, 1024, 512, 3, W53, 12, seed=121)
    mask = np.array([1, 0, 1, 1], np.uint8)
    want = gop.oracle([mask] * 12)
    dec = wv.Decoder(1024, 1024, 512, 3, wv.W53, wv.YUV420)
    tried = 0
    for v, name in enumerate(dec.variants()):
        if not name.startswith("strip_"):
            continue
        try:
            dec.variant = v
        except wv.WvError:
            continue
        tried += 1
        outs, ref, stamp = _run_gop_fused(dec, gop, mask)
        assert np.all(stamp[mask == 1] == 11) and np.all(stamp[mask == 0] == -1)
        for t in range(12):
            assert np.array_equal(outs[t], want[t][1]), (name, t)
        for r, w in zip(ref, want[-1][2]):
            assert np.array_equal(r[np.nonzero(mask)[0]], w), name
    assert tried >= 3


def test_gop_form_rules():
    """The first frame obeys the stamps (nothing runs otherwise); a context
    whose variant is not a row strip decodes frame by frame, same result."""
    wv = _wv()
    gop = Gop(128, 128, 64, 3, W53, 3, seed=77)
    mask = np.ones(gop.spec.n_tiles, np.uint8)
    want = gop.oracle([mask] * 3)
    dec = wv.Decoder(128, 128, 64, 3, wv.W53, wv.YUV420)
    frames = [(_dev(f["coeffs"], dec.coef_dtype), f["intra"], f["step"]) for f in gop.frames]
    ref = wv.Reference(dec)
    with pytest.raises(wv.WvError) as e:
        dec.decode_gop(frames[1:], 1, mask, ref)        # residual frame 1 without frame 0
    assert e.value.status == wv.ESTALE and np.all(ref.stamp == -1)
    outs, _, stamp = _run_gop_fused(dec, gop, mask)      # block variant: per-frame launches
    assert np.all(stamp == 2)
    for t in range(3):
        assert np.array_equal(outs[t], want[t][1])


# ------------------------------------------------------------- batch form
def test_batch_of_streams_equals_separate_decodes():
    """Uneven tile sets of several streams (different masks and foveation) in
    one fused launch give the same result as decoding each alone."""
    wv = _wv()
    rng = np.random.default_rng(12)
    gops = [Gop(256, 256, 64, 4, W53, 3, seed=40 + i) for i in range(5)]
    n = gops[0].spec.n_tiles
    masks = [[(rng.random(n) < 0.3 + 0.1 * i).astype(np.uint8)] * 3 for i in range(5)]
    for m in masks:
        m[0][0] = 1
    lcs = [[rng.integers(1, 5, n).astype(np.uint8)] * 3 for _ in range(5)]
    decs = [wv.Decoder(256, 256, 64, 4, wv.W53, wv.YUV420) for _ in range(5)]
    refs = [wv.Reference(d) for d in decs]
    frames = [[_dev(f["coeffs"], torch.int16) for f in g.frames] for g in gops]
    for t in range(3):
        outs = [torch.zeros(decs[i].out_shape(int(masks[i][t].sum())), dtype=torch.uint8,
                            device="cuda") for i in range(5)]
        jobs = [wv.BatchJob(decs[i], frames[i][t], t, t == 0, gops[i].frames[t]["step"],
                            masks[i][t], refs[i], outs[i], lcs[i][t]) for i in range(5)]
        wv.decode_batch(jobs)
        torch.cuda.synchronize()
        for i in range(5):
            want = gops[i].oracle(masks[i], lcs[i])[t]
            assert np.array_equal(outs[i].cpu().numpy(), want[1])


def test_batch_device_table_path_many_jobs():
    """More jobs/tiles than fit in kernel arguments: the batch goes through the
    device work table, still in one launch."""
    wv = _wv()
    gop = Gop(512, 512, 32, 3, W53, 1, seed=77)
    n = gop.spec.n_tiles                                  # 256 tiles
    decs = [wv.Decoder(512, 512, 32, 3, wv.W53, wv.YUV420) for _ in range(12)]
    refs = [wv.Reference(d) for d in decs]
    planes = _dev(gop.frames[0]["coeffs"], torch.int16)
    rng = np.random.default_rng(3)
    masks = [(rng.random(n) < 0.5).astype(np.uint8) for _ in range(12)]
    outs = [torch.zeros(decs[i].out_shape(int(masks[i].sum())), dtype=torch.uint8, device="cuda")
            for i in range(12)]
    jobs = [wv.BatchJob(decs[i], planes, 0, True, 4, masks[i], refs[i], outs[i]) for i in range(12)]
    wv.decode_batch(jobs)
    torch.cuda.synchronize()
    full = gop.oracle([np.ones(n, np.uint8)])[0]
    for i in range(12):
        vis = np.nonzero(masks[i])[0]
        assert np.array_equal(outs[i].cpu().numpy(), full[1][vis])


def test_batch_device_table_strip_kernels_512_tiles():
    """The work table in device memory with 512-sample tiles: two 8192x8192
    viewports of about 190 tiles each (more items than the kernel arguments
    hold) decoded in one launch by the row-strip kernel, equal to separate
    decodes and to the oracle."""
    wv = _wv()
    rng = np.random.default_rng(wvinputs.derive_seed(5, "batch512"))
    n = 256
    masks = [(rng.random(n) < 0.75).astype(np.uint8) for _ in range(2)]
    union = np.nonzero(masks[0] | masks[1])[0]
    gop = Gop(8192, 8192, 512, 5, W53, 1, seed=wvinputs.derive_seed(6, "batch512"), tiles=union)
    assert sum(int(m.sum()) for m in masks) > 360           # beyond the argument table
    decs = [wv.Decoder(8192, 8192, 512, 5, wv.W53, wv.YUV420) for _ in range(2)]
    assert decs[0].variants()[decs[0].variant].startswith("strip_")
    planes = _dev(gop.frames[0]["coeffs"], torch.int16)
    refs = [wv.Reference(d) for d in decs]
    outs = [torch.zeros(decs[i].out_shape(int(masks[i].sum())), dtype=torch.uint8, device="cuda")
            for i in range(2)]
    jobs = [wv.BatchJob(decs[i], planes, 0, True, 4, masks[i], refs[i], outs[i]) for i in range(2)]
    wv.decode_batch(jobs)
    sep = [torch.zeros_like(o) for o in outs]
    sep_refs = [wv.Reference(d) for d in decs]
    for i in range(2):
        decs[i].decode_viewport(planes, 0, True, 4, masks[i], sep_refs[i], sep[i])
    torch.cuda.synchronize()
    full = gop.oracle([np.isin(np.arange(n), union).astype(np.uint8)])[0]
    pos = {int(t): k for k, t in enumerate(full[0])}
    for i in range(2):
        vis = np.nonzero(masks[i])[0]
        idx = [pos[int(t)] for t in vis]
        got = outs[i].cpu().numpy()
        assert np.array_equal(got, sep[i].cpu().numpy()), f"job {i}: batch != separate decode"
        assert np.array_equal(got, full[1][idx]), f"job {i}: differs from the oracle"
        for p in range(3):
            assert np.array_equal(refs[i].planes[p].cpu().numpy()[vis], full[2][p][idx])


# ----------------------------------------------------------------- encoder
@pytest.mark.parametrize("wavelet,levels", [(W53, 5), (W97, 4)])
def test_gpu_encoder_matches_oracle(wavelet, levels):
    wv = _wv()
    gop = Gop(1024, 512, 512, levels, wavelet, 1, seed=99)
    wl = wv.W53 if wavelet == W53 else wv.W97
    dec = wv.Decoder(1024, 512, 512, levels, wl, wv.YUV420)
    src = [torch.from_numpy(p).cuda() for p in gop.source]
    dst = [torch.zeros(dec.plane_shape(p), dtype=dec.coef_dtype, device="cuda") for p in range(3)]
    dec.encode_intra(src, dst, gop.intra_step)
    for p in range(3):
        got = dst[p].cpu().numpy()
        want = gop.frames[0]["coeffs"][p]
        if wavelet == W53:
            assert np.array_equal(got, want)
        else:
            # float64 forward on both sides; a rounding tie may move one step
            diff = np.abs(got.astype(np.float64) - want)
            assert np.mean(diff > 0) < 1e-4 and diff.max() <= gop.intra_step
