"""Pins of the inter-frame-set oracle (oracle/interframe.py, Section 3.2).

The temporal transform is checked against the Haar synthesis matrix built by
its textbook recursion (coarse functions stretched over pairs, finest
functions as +1/-1 pulses), against a linear solve with that matrix, and on
sequences with known transforms.  The set decode is checked against the
pinned intra decode of the frame that the matrix synthesises, and the
encoder round trip against its quantisation bound.
"""
import numpy as np
import pytest

import wvinputs
from oracle import codec, interframe
from oracle.wavelet import W53, W97, fwd2d


def haar_matrix(n):
    """Synthesis matrix A (frames = A @ bands) of the averaging Haar:
    A_1 = [1]; A_2m = [A_m kron (1, 1)^T | I_m kron (1, -1)^T]."""
    a = np.ones((1, 1))
    while a.shape[0] < n:
        m = a.shape[0]
        a = np.hstack([np.kron(a, [[1.0], [1.0]]), np.kron(np.eye(m), [[1.0], [-1.0]])])
    return a


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16])
def test_synthesis_equals_textbook_haar_matrix(n):
    a = haar_matrix(n)
    eye = np.eye(n)
    assert np.array_equal(interframe.haar_inverse(eye), a)
    for t in range(n):
        assert np.array_equal(interframe.haar_frame(eye, t), a[t])
    assert np.allclose(interframe.haar_forward(a), eye, atol=0, rtol=0)


@pytest.mark.parametrize("n", [2, 4, 8])
def test_analysis_is_the_inverse_of_the_synthesis_matrix(n):
    rng = np.random.default_rng(n)
    f = rng.normal(size=(n, 5, 3))
    want = np.linalg.solve(haar_matrix(n), f.reshape(n, -1)).reshape(f.shape)
    assert np.allclose(interframe.haar_forward(f), want, atol=1e-12)


def test_basis_is_orthogonal_with_the_averaging_gains():
    """Haar filters do not overlap: the synthesis functions are orthogonal,
    with squared norms n (approximation, coarsest detail), then n/2 ... 2."""
    a = haar_matrix(8)
    g = a.T @ a
    assert np.array_equal(g, np.diag(np.diag(g)))
    assert np.array_equal(np.diag(g), [8, 8, 4, 4, 2, 2, 2, 2])


def test_known_sequences():
    hf = interframe.haar_forward
    assert np.array_equal(hf([5.0, 5.0, 5.0, 5.0]), [5, 0, 0, 0])
    assert np.array_equal(hf([1.0, -1.0, 1.0, -1.0]), [0, 0, 1, 1])
    assert np.array_equal(hf([1.0, 1.0, -1.0, -1.0]), [0, 1, 0, 0])
    assert np.array_equal(hf([4.0, 0.0, 0.0, 0.0]), [1, 1, 2, 0])


@pytest.mark.parametrize("n", [2, 4, 8, 16])
def test_a_frame_takes_log2_n_signed_additions(n):
    a = haar_matrix(n)
    for t in range(n):
        terms = interframe.frame_terms(n, t)
        assert len(terms) == 1 + int(np.log2(n))
        assert len({b for b, _ in terms}) == len(terms)
        # exactly the bands whose synthesis function is non-zero at t, with its sign
        assert sorted(terms) == sorted((b, int(a[t, b])) for b in range(n) if a[t, b] != 0)


def test_bad_set_sizes_and_frames():
    with pytest.raises(ValueError):
        interframe.frame_terms(3, 0)
    with pytest.raises(ValueError):
        interframe.frame_terms(4, 4)


def test_perfect_reconstruction_is_exact():
    rng = np.random.default_rng(9)
    f = rng.integers(-3000, 3000, size=(8, 6, 7)).astype(np.float64)
    bands = interframe.haar_forward(f)
    assert np.array_equal(interframe.haar_inverse(bands), f)
    for t in range(8):
        assert np.array_equal(interframe.haar_frame(bands, t), f[t])


def _set_inputs(wavelet, n, levels, seed):
    """Seeded bands: the approximation from an encoded synthetic frame, the
    details Laplace-distributed like residual frames."""
    spec = wvinputs.FrameSpec(128, 128, 64, seed)
    src = [s.numpy().reshape(spec.n_tiles, *s.shape[2:]) for s in wvinputs.source_planes(spec)]
    step0 = 4 if wavelet == W53 else 8
    base = codec.encode_intra(src, levels, wavelet, step0)
    planes = []
    for p in range(3):
        bands = [base[p]]
        for b in range(1, n):
            r = wvinputs.residual_planes(spec, b, integer=(wavelet == W53))[p]
            bands.append(r.numpy().reshape(base[p].shape).astype(base[p].dtype))
        planes.append(np.stack(bands))
    steps = [step0] + [1] * (n - 1)
    return spec, planes, steps


@pytest.mark.parametrize("wavelet", [W53, W97])
@pytest.mark.parametrize("n", [2, 4])
def test_set_decode_equals_intra_decode_of_the_synthesised_frame(wavelet, n):
    levels = 3
    spec, planes, steps = _set_inputs(wavelet, n, levels, 31)
    a = haar_matrix(n)
    mask = np.zeros(spec.n_tiles, np.uint8)
    mask[[0, 2, 3]] = 1
    lc = np.array([3, 2, 1, 3])
    for t in range(n):
        vis, out, rec = interframe.decode_set_viewport(planes, t, mask, levels, wavelet, steps, lc)
        coeffs = []
        for b in planes:
            deq = b.astype(np.float64) * np.asarray(steps, np.float64)[:, None, None, None] \
                if wavelet == W53 else b.astype(np.float64)
            c = np.tensordot(a[t], deq, axes=1)
            coeffs.append(c.astype(np.int64) if wavelet == W53 else c)
        want = codec.decode_tiles([{"coeffs": [c[vis] for c in coeffs], "step": 1, "intra": True,
                                    "level_count": lc[vis]}], levels, wavelet)[0]
        assert np.array_equal(vis, [0, 2, 3])
        if wavelet == W53:
            assert np.array_equal(out, want["out"])
        else:
            assert np.allclose(out, want["out"], atol=1e-9)


def test_encoder_round_trip_within_the_quantisation_bound():
    """Each band is off by at most step/2 after quantisation, and a frame sums
    1 + log2 n bands: |c_t - decoded c_t| <= sum of their half steps."""
    n, levels = 4, 3
    spec = wvinputs.FrameSpec(128, 128, 64, 5)
    frames = []
    for t in range(n):
        sp = wvinputs.FrameSpec(128, 128, 64, wvinputs.derive_seed(5, "set", t))
        frames.append([s.numpy().reshape(spec.n_tiles, *s.shape[2:])
                       for s in wvinputs.source_planes(sp)])
    steps = [2, 3, 1, 5]
    enc = interframe.encode_set(frames, levels, W53, steps)
    for t in range(n):
        bound = sum(steps[b] / 2 for b, _ in interframe.frame_terms(n, t))
        for p in range(3):
            exact = fwd2d(frames[t][p], levels, W53)
            got = interframe.frame_coefficients(enc[p], t, steps, W53)
            assert np.max(np.abs(got - exact)) <= bound
