"""Host-side check of the format encoder in libwv (wv_sparse_encode_plane)
against the oracle's (oracle/paperformat.py): identical block ends, codes,
indices and bounds.  Host code only: no device is touched."""
import numpy as np
import pytest

import wvinputs
from oracle import paperformat as pf
from oracle.wavelet import W97, fwd2d


def _coefficients(width, height, tile, levels, plane, seed):
    """Seeded 9/7 coefficients of a synthetic frame's plane, tile-major."""
    spec = wvinputs.FrameSpec(width, height, tile, seed)
    src = wvinputs.source_planes(spec)[plane].numpy()
    src = src.reshape(src.shape[0] * src.shape[1], *src.shape[2:]) if src.ndim == 4 else src
    return fwd2d(src.astype(np.float64), levels, W97).astype(np.float32)


@pytest.mark.parametrize("plane", [0, 1])
@pytest.mark.parametrize("alpha,poles", [(0.0, False), (0.1, True), (0.25, False), (0.03, True)])
def test_library_encoder_equals_oracle(plane, alpha, poles):
    from paper_2208_10859_amd import fmt, wv
    W, H, tile, levels = 256, 256, 64, 3
    c = _coefficients(W, H, tile, levels, plane, 21 + plane)
    desc = wv.make_desc(W, H, tile, levels, wv.W97, wv.YUV420)
    got = fmt.encode_plane(desc, plane, c, alpha, poles)
    p_h = H if plane == 0 else H // 2
    want = pf.encode_plane(c, levels, W // tile, p_h, alpha, poles)
    assert np.array_equal(got["block_end"], want["block_end"])
    assert np.array_equal(got["values"], want["values"])
    assert np.array_equal(got["index"], want["index"])
    assert np.array_equal(got["bounds"], want["bounds"])
    if alpha > 0:
        assert got["values"].size < c.size


def test_laplace_details_and_512_tiles():
    from paper_2208_10859_amd import fmt, wv
    rng = np.random.default_rng(5)
    c = rng.laplace(0, 6, (2, 512, 512)).astype(np.float32)
    desc = wv.make_desc(1024, 512, 512, 5, wv.W97, wv.GRAY8)
    got = fmt.encode_plane(desc, 0, c, 0.02, True)
    want = pf.encode_plane(c, 5, 2, 512, 0.02, True)
    for k in ("block_end", "values", "index", "bounds"):
        assert np.array_equal(got[k], want[k]), k
    assert fmt.blocks_per_tile(desc, 0) == 256 and fmt.blocks_per_tile(desc, 1) == 0


def test_encoder_rejects_bad_arguments():
    from paper_2208_10859_amd import fmt, wv
    desc = wv.make_desc(256, 256, 64, 3, wv.W97, wv.GRAY8)
    c = np.zeros((16, 64, 64), np.float32)
    with pytest.raises(ValueError):                  # no plane 1 in a grey frame
        fmt.encode_plane(desc, 1, c, 0.1, False)
    for alpha in (-1.0, float("nan")):
        with pytest.raises(wv.WvError) as e:
            fmt.encode_plane(desc, 0, c, alpha, False)
        assert e.value.status == wv.EINVAL
