"""GPU parity of inter-frame-set decoding (wv_decode_set) against the oracle
(oracle/interframe.py, Section 3.2): 5/3 bit-exact, 9/7 within max-abs 1e-3
on the 0..255 scale.

Bands are seeded synthetic inputs: band 0 is an encoded synthetic frame,
the detail bands are Laplace-distributed like residual frames (tests/gop.py
builds both; expected values come from the oracle only).
"""
import numpy as np
import pytest
import torch

from gop import Gop, W53, W97
from oracle import interframe

pytestmark = pytest.mark.gpu

TOL97 = 1e-3


def _wv():
    from paper_2208_10859_amd import wv
    return wv


def _bands(wavelet, levels, n, width, height, tiles, seed):
    """Per plane, bands [n][n_tiles][P][P] (numpy) populated on `tiles`."""
    g = Gop(width, height, 512, levels, wavelet, n, seed, tiles=tiles)
    return [np.stack([g.frames[b]["coeffs"][p] for b in range(n)]) for p in range(3)], g.intra_step


def _decode(dec, bands, n, steps, t0, nf, mask, lc=None):
    dev = [torch.from_numpy(np.ascontiguousarray(b)).to("cuda") for b in bands]
    nvis = int(np.count_nonzero(mask))
    outs = [torch.full(dec.out_shape(nvis), 77, dtype=dec.sample_dtype, device="cuda") for _ in range(nf)]
    dec.decode_set(dev, n, steps, t0, mask, outs, lc)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs]


def _check(out, want, wavelet, what):
    if wavelet == W53:
        assert out.dtype == np.uint8
        assert np.array_equal(out, want), what
    else:
        err = float(np.max(np.abs(out.astype(np.float64) - want)))
        assert err <= TOL97, (what, err)


CASES = [
    # wavelet, levels, n, steps, foveate
    (W53, 5, 4, None, False),
    (W53, 4, 4, (4, 2, 1, 3), True),
    (W53, 3, 2, (3, 2), False),
    (W97, 4, 4, None, True),
    (W97, 5, 2, None, False),
]


@pytest.mark.parametrize("wavelet,levels,n,steps,foveate", CASES)
def test_set_frames_equal_oracle(wavelet, levels, n, steps, foveate):
    """A 4096 x 2048 frame (8 x 4 tiles of 512), a ragged viewport of 7 tiles,
    every frame of the set in one call and one by one, for every row-strip
    variant of the geometry."""
    wv = _wv()
    W, H = 4096, 2048
    mask = np.zeros(32, np.uint8)
    mask[[0, 5, 6, 13, 22, 30, 31]] = 1
    vis = np.nonzero(mask)[0]
    bands, step0 = _bands(wavelet, levels, n, W, H, vis, 1000 + levels * 10 + n)
    steps = tuple(steps) if steps else (step0,) + (1,) * (n - 1)
    lc = None
    if foveate:
        lc = np.full(32, levels, np.uint8)
        lc[[5, 22]] = levels - 1
        lc[[31]] = levels - 2
    wl = wv.W53 if wavelet == W53 else wv.W97
    dec = wv.Decoder(W, H, 512, levels, wl, wv.YUV420)
    want = [interframe.decode_set_viewport(bands, t, mask, levels, wavelet, steps, lc) for t in range(n)]
    for v in want:
        assert np.array_equal(v[0], vis)
    tried = 0
    for v, name in enumerate(dec.variants()):
        if not name.startswith("strip_"):
            continue
        try:
            dec.variant = v
        except wv.WvError:
            continue
        tried += 1
        outs = _decode(dec, bands, n, steps, 0, n, mask, lc)
        for t in range(n):
            _check(outs[t], want[t][1], wavelet, f"{name}: frame {t} of {n} (one call)")
        for t in range(n):
            (out,) = _decode(dec, bands, n, steps, t, 1, mask, lc)
            _check(out, want[t][1], wavelet, f"{name}: frame {t} of {n} (alone)")
    assert tried >= 2


def test_grey_set_equals_oracle():
    wv = _wv()
    W, H, levels, n = 2048, 1024, 4, 4
    mask = np.array([1, 0, 1, 1, 0, 0, 1, 0], np.uint8)
    vis = np.nonzero(mask)[0]
    g = Gop(W, H, 512, levels, W53, n, 77, tiles=vis, chroma=False)
    bands = [np.stack([g.frames[b]["coeffs"][0] for b in range(n)])]
    steps = (g.intra_step, 1, 2, 1)
    dec = wv.Decoder(W, H, 512, levels, wv.W53, wv.GRAY8)
    outs = _decode(dec, bands, n, steps, 0, n, mask)
    for t in range(n):
        _, wout, _ = interframe.decode_set_viewport(bands, t, mask, levels, W53, steps)
        _check(outs[t], wout, W53, f"grey frame {t}")


def test_zero_details_give_the_intra_decode_at_full_size():
    """8192^2, 5 levels, the bench's viewport size: with every detail band
    zero, each frame of the set equals wv_decode_viewport's intra decode of
    band 0 (a property at any size), and two tiles equal the oracle."""
    wv = _wv()
    from gop import pose_mask
    W = H = 8192
    mask, _ = pose_mask(W, H, 512, 10859, 0)
    vis = np.nonzero(mask)[0]
    g = Gop(W, H, 512, 5, W53, 1, 4242, tiles=vis)
    step0 = g.intra_step
    bands = [np.concatenate([g.frames[0]["coeffs"][p][None],
                             np.zeros((3,) + g.frames[0]["coeffs"][p].shape, np.int16)]) for p in range(3)]
    dec = wv.Decoder(W, H, 512, 5, wv.W53, wv.YUV420)
    outs = _decode(dec, bands, 4, (step0, 3, 1, 2), 0, 4, mask)
    ref = wv.Reference(dec)
    intra = torch.empty(dec.out_shape(len(vis)), dtype=torch.uint8, device="cuda")
    dec.decode_viewport([torch.from_numpy(b[0]).to("cuda") for b in bands], 0, True, step0, mask, ref, intra)
    torch.cuda.synchronize()
    intra = intra.cpu().numpy()
    for t in range(4):
        assert np.array_equal(outs[t], intra), t
    sub = np.zeros_like(mask)
    sub[vis[[0, -1]]] = 1
    _, wout, _ = interframe.decode_set_viewport(bands, 2, sub, 5, W53, (step0, 3, 1, 2))
    assert np.array_equal(outs[2][[0, -1]], wout)


def test_full_size_set_every_visible_tile_equals_oracle():
    """8192^2 set of four with Laplace details on every visible tile (the
    bench's one-eye viewport, 37 tiles), all in one launch: every tile of
    every frame equals the oracle."""
    wv = _wv()
    from gop import pose_mask
    W = H = 8192
    mask, _ = pose_mask(W, H, 512, 10859, 3)
    vis = np.nonzero(mask)[0]
    bands, step0 = _bands(W53, 5, 4, W, H, vis, 99)
    steps = (step0, 1, 1, 1)
    dec = wv.Decoder(W, H, 512, 5, wv.W53, wv.YUV420)
    outs = _decode(dec, bands, 4, steps, 0, 4, mask)
    for t in range(4):
        got_vis, wout, _ = interframe.decode_set_viewport(bands, t, mask, 5, W53, steps)
        assert np.array_equal(got_vis, vis)
        assert np.array_equal(outs[t], wout), t


def test_set_errors_and_empty_mask():
    wv = _wv()
    dec = wv.Decoder(1024, 1024, 512, 3, wv.W53, wv.YUV420)
    bands = [torch.zeros(dec.set_shape(4, p), dtype=torch.int16, device="cuda") for p in range(3)]
    mask = np.ones(4, np.uint8)
    out = torch.full(dec.out_shape(4), 5, dtype=torch.uint8, device="cuda")
    with pytest.raises(wv.WvError) as e:
        dec.decode_set(bands, 3, (1, 1, 1), 0, mask, [out])
    assert e.value.status == wv.EUNSUPPORTED
    with pytest.raises(wv.WvError) as e:
        dec.decode_set(bands, 4, (1, 1, 1, 1), 3, mask, [out, out])
    assert e.value.status == wv.EINVAL
    with pytest.raises(wv.WvError) as e:
        dec.decode_set(bands, 4, (1, 0, 1, 1), 0, mask, [out])
    assert e.value.status == wv.EINVAL
    lc = np.full(4, 4, np.uint8)
    with pytest.raises(wv.WvError) as e:
        dec.decode_set(bands, 4, (1, 1, 1, 1), 0, mask, [out], lc)
    assert e.value.status == wv.EINVAL
    dec.decode_set(bands, 4, (1, 1, 1, 1), 0, np.zeros(4, np.uint8), [out])   # nothing visible
    torch.cuda.synchronize()
    assert int(out.min()) == 5 and int(out.max()) == 5
    small = wv.Decoder(256, 256, 64, 3, wv.W53, wv.YUV420)      # no row-strip kernel for tile 64
    sb = [torch.zeros(small.set_shape(2, p), dtype=torch.int16, device="cuda") for p in range(3)]
    so = torch.empty(small.out_shape(16), dtype=torch.uint8, device="cuda")
    with pytest.raises(wv.WvError) as e:
        small.decode_set(sb, 2, (1, 1), 0, np.ones(16, np.uint8), [so])
    assert e.value.status == wv.EUNSUPPORTED
