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


def _brute_records(enc, p, levels, mask, lc):
    """Record indices a viewport needs, block by block from the oracle's block
    order and levels (Section 3.4 block ends, Section 3.7 level drop)."""
    order = pf.block_order(p, levels)
    nb = len(order)
    be = enc["block_end"].astype(np.int64)
    need = []
    for t in np.nonzero(mask)[0]:
        for j, (by, bx) in enumerate(order):
            if pf.block_level(p, levels, by, bx) <= levels - int(lc[t]):
                continue
            g = t * nb + j
            need.extend(range(int(be[g - 1]) if g else 0, int(be[g])))
    return np.array(sorted(need), np.int64)


@pytest.mark.parametrize("plane", [0, 1])
@pytest.mark.parametrize("seed", [3, 4])
def test_visible_runs_cover_exactly_the_kept_blocks(plane, seed):
    """The merged runs hold exactly the records of the visible tiles' kept
    blocks: sorted, disjoint, not touching, none empty."""
    from paper_2208_10859_amd import fmt, wv
    W, H, tile, levels = 512, 256, 64, 3
    c = _coefficients(W, H, tile, levels, plane, 40 + seed)
    desc = wv.make_desc(W, H, tile, levels, wv.W97, wv.YUV420)
    enc = fmt.encode_plane(desc, plane, c, 0.02, True)
    rng = np.random.default_rng(seed)
    n_tiles = (W // tile) * (H // tile)
    p = tile if plane == 0 else tile // 2
    for trial in range(6):
        mask = (rng.random(n_tiles) < 0.6).astype(np.uint8)
        lc = rng.integers(0, levels + 1, n_tiles).astype(np.uint8) if trial % 2 else np.full(n_tiles, levels, np.uint8)
        b, e, tot = fmt.visible_runs(desc, plane, enc, mask, lc if trial % 2 else None)
        assert np.all(e > b) and np.all(b[1:] > e[:-1])
        got = np.concatenate([np.arange(x, y) for x, y in zip(b, e)]) if b.size else np.zeros(0, np.int64)
        want = _brute_records(enc, p, levels, mask, lc)
        assert np.array_equal(got, want)
        assert tot == want.size
    b, e, tot = fmt.visible_runs(desc, plane, enc, np.ones(n_tiles, np.uint8))
    assert list(b) == [0] and list(e) == [enc["values"].size] and tot == enc["values"].size


def test_visible_runs_errors_and_clamps():
    from paper_2208_10859_amd import fmt, wv
    desc = wv.make_desc(128, 128, 64, 2, wv.W97, wv.GRAY8)
    be = np.array([2, 3, 3, 5] + [5, 5, 9, 9] + [9] * 8, np.uint32)
    enc = {"block_end": be, "values": np.zeros(7, np.uint8)}
    # ends beyond the 7 records count as 7
    b, e, tot = fmt.visible_runs(desc, 0, enc, np.array([0, 1, 0, 0], np.uint8))
    assert list(b) == [5] and list(e) == [7] and tot == 2
    with pytest.raises(wv.WvError) as err:
        fmt.visible_runs(desc, 0, enc, np.ones(4, np.uint8), np.full(4, 3, np.uint8))
    assert err.value.status == wv.EINVAL
    bad = {"block_end": np.array([4, 3, 5, 6] + [6] * 12, np.uint32), "values": np.zeros(6, np.uint8)}
    with pytest.raises(wv.WvError):
        fmt.visible_runs(desc, 0, bad, np.array([1, 0, 0, 0], np.uint8))


def test_store_file_round_trip(tmp_path):
    """The file container (Section 3.4): frames written and read back give
    the same block ends, indices, codes and bounds; a damaged or truncated
    file is refused."""
    from paper_2208_10859_amd import fmt, wv
    W, H, tile, levels = 256, 256, 64, 3
    desc = wv.make_desc(W, H, tile, levels, wv.W97, wv.YUV420)
    frames = []
    for f in range(3):
        frames.append([fmt.encode_plane(desc, p, _coefficients(W, H, tile, levels, p, 60 + 3 * f + p),
                                        (0.0, 0.05, 0.3)[f], f == 1) for p in range(3)])
    path = tmp_path / "frames.wvf"
    fmt.write_store(path, desc, frames)
    st = fmt.Store(path, pinned=False)
    assert st.n_frames == 3 and (st.desc.width, st.desc.tile, st.desc.levels) == (W, tile, levels)
    for f in range(3):
        for p in range(3):
            got = st.arrays(f, p)
            for k in ("block_end", "index", "values", "bounds"):
                assert np.array_equal(got[k], frames[f][p][k]), (f, p, k)
    with pytest.raises(wv.WvError):
        st.frame(3)
    st.close()
    raw = bytearray(path.read_bytes())
    bad = tmp_path / "bad.wvf"
    bad.write_bytes(bytes(raw[:-40]))              # truncated: the last package is cut
    with pytest.raises(wv.WvError) as e:
        fmt.Store(bad, pinned=False)
    assert e.value.status == wv.EINVAL
    raw[0] ^= 0xff                                 # not this format
    bad.write_bytes(bytes(raw))
    with pytest.raises(wv.WvError):
        fmt.Store(bad, pinned=False)
