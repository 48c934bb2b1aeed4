"""wv_decode_viewport_noalloc (no context, no allocation: its kernels' queue
counters live in the library's file-scope device array) against
wv_decode_viewport with the same persistent variant: two calls in a row on
one GPU, the second with fewer visible tiles, each compared output for output
and reference for reference (5/3 bit-exact), and with the oracle."""
import ctypes

import numpy as np
import pytest
import torch

import wvinputs
from gop import Gop, W53

pytestmark = pytest.mark.gpu


def _wv():
    from paper_2208_10859_amd import wv
    return wv


def _noalloc(wv):
    return wv.lib().wv_decode_viewport_noalloc     # prototype declared by the binding


@pytest.mark.parametrize("W,H,TILE,LEVELS", [(2048, 1024, 512, 5), (1024, 512, 64, 3)])
def test_noalloc_equals_context_entry_point(W, H, TILE, LEVELS):
    wv = _wv()
    fn = _noalloc(wv)
    n = (W // TILE) * (H // TILE)
    masks = [np.ones(n, np.uint8), np.zeros(n, np.uint8)]
    masks[1][: n // 2] = 1                                   # second call: fewer tiles
    print(f"noalloc case {W}x{H} tile {TILE} L{LEVELS}", flush=True)
    gop = Gop(W, H, TILE, LEVELS, W53, 2, seed=wvinputs.derive_seed(31, "noalloc", TILE))
    want = gop.oracle(masks)
    dec = wv.Decoder(W, H, TILE, LEVELS, wv.W53, wv.YUV420)
    pers = [v for v, name in enumerate(dec.variants()) if "persist" in name]
    for v in pers:                                           # the first that fits
        try:
            dec.variant = v
            break
        except wv.WvError:
            continue
    ref_a, ref_b = wv.Reference(dec), wv.Reference(dec)
    desc = wv.make_desc(W, H, TILE, LEVELS, wv.W53, wv.YUV420)
    stream = torch.cuda.current_stream().cuda_stream
    for t, f in enumerate(gop.frames):
        planes = [torch.from_numpy(np.ascontiguousarray(p)).cuda() for p in f["coeffs"]]
        nv = int(masks[t].sum())
        out_a = torch.full(dec.out_shape(nv), 7, dtype=torch.uint8, device="cuda")
        out_b = torch.full(dec.out_shape(nv), 9, dtype=torch.uint8, device="cuda")
        dec.decode_viewport(planes, t, f["intra"], f["step"], masks[t], ref_a, out_a)
        fr = dec.frame(planes, t, f["intra"], f["step"])
        m = np.ascontiguousarray(masks[t])
        st = fn(ctypes.byref(desc), ctypes.byref(fr), None,
                m.ctypes.data, ctypes.byref(ref_b._c),
                ctypes.c_void_p(out_b.data_ptr()), ctypes.c_void_p(stream))
        assert st == wv.OK, wv.lib().wv_last_error()
        torch.cuda.synchronize()
        a, b = out_a.cpu().numpy(), out_b.cpu().numpy()
        assert np.array_equal(a, b), f"frame {t}: no-alloc output differs"
        assert np.array_equal(b, want[t][1]), f"frame {t}: differs from the oracle"
        for p in range(3):
            assert torch.equal(ref_a.planes[p], ref_b.planes[p]), f"frame {t} plane {p}"
        assert np.array_equal(ref_a.stamp, ref_b.stamp)


def test_noalloc_errors_leave_state():
    wv = _wv()
    fn = _noalloc(wv)
    dec = wv.Decoder(1024, 512, 512, 5, wv.W53, wv.YUV420)
    ref = wv.Reference(dec)
    desc = wv.make_desc(1024, 512, 512, 5, wv.W53, wv.YUV420)
    planes = [torch.zeros(dec.plane_shape(p), dtype=torch.int16, device="cuda") for p in range(3)]
    fr = dec.frame(planes, 3, False, 1)                      # residual, stamps are -1: stale
    m = np.ones(dec.n_tiles, np.uint8)
    out = torch.zeros(dec.out_shape(dec.n_tiles), dtype=torch.uint8, device="cuda")
    st = fn(ctypes.byref(desc), ctypes.byref(fr), None, m.ctypes.data,
            ctypes.byref(ref._c), ctypes.c_void_p(out.data_ptr()), None)
    assert st == wv.ESTALE
    assert np.all(ref.stamp == -1)
    bad = wv.make_desc(1000, 512, 512, 5, wv.W53, wv.YUV420)
    st = fn(ctypes.byref(bad), ctypes.byref(fr), None, m.ctypes.data,
            ctypes.byref(ref._c), ctypes.c_void_p(out.data_ptr()), None)
    assert st == wv.EINVAL
