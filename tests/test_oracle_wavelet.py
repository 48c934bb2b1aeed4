"""Pins of the oracle's wavelet transforms against what the mathematics fixes.

None of these re-types the lifting formulas: they check perfect reconstruction,
constants, the published linear filter banks (brute-force matrices and impulse
responses) and the zero-detail special case, so that a dropped term, a wrong
sign, a wrong boundary rule or a swapped pass order fails one of them.
"""
import numpy as np
import pytest

from conftest import load_golden
from oracle import wavelet as wv


def _reflect(j, n):
    """Whole-sample symmetric extension index for a length-n signal."""
    if n == 1:
        return 0
    p = 2 * n - 2
    j %= p
    return p - j if j >= n else j


def _analysis_matrix(n, low, high):
    """Linear analysis matrix (n x n) from centre-first symmetric taps with
    whole-sample symmetric extension: rows 0..n/2-1 low band, then high band."""
    a = np.zeros((n, n))
    for i in range(n // 2):
        for k in range(-(len(low) - 1), len(low)):
            a[i, _reflect(2 * i + k, n)] += low[abs(k)]
        for k in range(-(len(high) - 1), len(high)):
            a[n // 2 + i, _reflect(2 * i + 1 + k, n)] += high[abs(k)]
    return a


def _linear_fwd2d(x, levels, low, high):
    c = np.array(x, dtype=np.float64)
    n = c.shape[-1]
    for lev in range(levels):
        m = n >> lev
        a = _analysis_matrix(m, low, high)
        c[:m, :m] = a @ c[:m, :m] @ a.T
    return c


def _linear_inv2d(c, levels, low, high):
    x = np.array(c, dtype=np.float64)
    n = x.shape[-1]
    for lev in reversed(range(levels)):
        m = n >> lev
        ai = np.linalg.inv(_analysis_matrix(m, low, high))
        x[:m, :m] = ai @ x[:m, :m] @ ai.T
    return x


# ------------------------------------------------------------------ 5/3 pins
def test_lift53_perfect_reconstruction_1d():
    rng = np.random.default_rng(1)
    for n in range(2, 130, 2):
        x = rng.integers(-300, 300, (5, n))
        s, d = wv.fwd53(x)
        assert np.array_equal(wv.inv53(s, d), x)


@pytest.mark.parametrize("n,levels", [(8, 3), (16, 4), (32, 5), (64, 2), (512, 5), (256, 5)])
def test_lift53_perfect_reconstruction_2d(n, levels):
    rng = np.random.default_rng(n + levels)
    x = rng.integers(0, 256, (3, n, n))
    c = wv.fwd2d(x, levels, wv.W53)
    assert c.dtype == np.int64
    assert np.array_equal(wv.inv2d(c, levels, wv.W53), x)


def test_lift53_constant_image():
    for val in (0, 1, 77, 255):
        c = wv.fwd2d(np.full((64, 64), val), 4, wv.W53)
        ll = 64 >> 4
        assert np.all(c[:ll, :ll] == val)
        c[:ll, :ll] = 0
        assert np.all(c == 0)


def test_lift53_matches_linear_filter_bank_8x8():
    """Integer lifting equals the textbook linear 5/3 filter bank exactly when no
    floor discards anything (inputs scaled by 2^20), and differs on raw 8-bit
    inputs (so the comparison is sharp)."""
    taps = load_golden("legall53_filters.txt")
    low, high = taps["analysis_low"], taps["analysis_high"]
    rng = np.random.default_rng(7)
    for _ in range(20):
        x = rng.integers(0, 256, (8, 8))
        xs = x * (1 << 20)
        lin = _linear_fwd2d(xs, 3, low, high)
        assert np.array_equal(wv.fwd2d(xs, 3, wv.W53), np.rint(lin).astype(np.int64))
        assert np.max(np.abs(lin - np.rint(lin))) < 1e-6
        # inverse: coefficients that are multiples of 2^20
        c = rng.integers(-200, 200, (8, 8)) * (1 << 20)
        lin_inv = _linear_inv2d(c, 3, low, high)
        assert np.max(np.abs(lin_inv - np.rint(lin_inv))) < 1e-4
        assert np.array_equal(wv.inv2d(c, 3, wv.W53), np.rint(lin_inv).astype(np.int64))
    # sharpness: raw inputs do not match the linear bank exactly
    diffs = []
    for _ in range(20):
        x = rng.integers(0, 256, (8, 8))
        diffs.append(np.max(np.abs(wv.fwd2d(x, 3, wv.W53) - _linear_fwd2d(x, 3, low, high))))
    assert max(diffs) > 0.1


def test_lift53_pass_order_is_observable():
    """Rows-first and columns-first forward levels differ for the integer 5/3,
    so the stated order (columns then rows forward) is a real convention."""
    rng = np.random.default_rng(3)
    x = rng.integers(0, 256, (16, 16))
    a = wv.fwd2d(x, 1, wv.W53)
    s, d = wv.fwd53(x)                     # rows first ...
    r = np.concatenate([s, d], axis=-1)
    s, d = wv.fwd53(r.T)                   # ... then columns
    b = np.concatenate([s, d], axis=-1).T
    assert np.count_nonzero(a != b) > 10


def _zero_detail_53(ll, levels):
    """Pure-Python synthesis with all detail bands zero: per level, every row then
    every column is upsampled as x[2i] = s[i], x[2i+1] = floor((s[i] + s[i+1]) / 2),
    with s[m] = s[m-1] (the 5/3 synthesis reduces to this when d = 0)."""
    cur = [list(map(int, r)) for r in ll]
    for _ in range(levels):
        m = len(cur)
        rows = []
        for r in cur:
            out = []
            for i in range(m):
                nxt = r[i + 1] if i + 1 < m else r[m - 1]
                out += [r[i], (r[i] + nxt) // 2]
            rows.append(out)
        cols = [[rows[i][j] for i in range(m)] for j in range(2 * m)]
        up = []
        for col in cols:
            out = []
            for i in range(m):
                nxt = col[i + 1] if i + 1 < m else col[m - 1]
                out += [col[i], (col[i] + nxt) // 2]
            up.append(out)
        cur = [[up[j][i] for j in range(2 * m)] for i in range(2 * m)]
    return np.array(cur, dtype=np.int64)


def test_lift53_zero_detail_is_interpolation():
    rng = np.random.default_rng(5)
    for levels in (1, 2, 3):
        c = rng.integers(-50, 300, (32, 32))
        z = wv.zero_finest(c, levels)
        m = 32 >> levels
        assert np.count_nonzero(z[m:, :]) == 0 and np.count_nonzero(z[:, m:]) == 0
        got = wv.inv2d(z, levels, wv.W53)
        assert np.array_equal(got, _zero_detail_53(c[:m, :m], levels))


def test_zero_finest_counts():
    c = np.ones((64, 64), dtype=np.int64)
    for k in range(0, 5):
        z = wv.zero_finest(c, k)
        assert z.sum() == (64 >> k) ** 2
        assert np.all(z[:64 >> k, :64 >> k] == 1)


# ------------------------------------------------------------------ 9/7 pins
def _impulse_rows(n, which):
    rows = []
    for j in range(n):
        x = np.zeros(n)
        x[j] = 1.0
        s, d = wv.fwd97(x)
        rows.append(s if which == "s" else d)
    return np.array(rows).T


def test_lift97_analysis_taps_match_published():
    taps = load_golden("cdf97_filters.txt")
    n = 64
    a_s = _impulse_rows(n, "s")
    a_d = _impulse_rows(n, "d")
    low = taps["analysis_low"]
    high = taps["analysis_high"]
    i = 16                       # interior low-band coefficient, centred on x[32]
    for k in range(-8, 9):
        want = low[abs(k)] if abs(k) < len(low) else 0.0
        assert abs(a_s[i, 2 * i + k] - want) < 2e-12
    for k in range(-8, 9):       # interior high-band coefficient, centred on x[33]
        want = high[abs(k)] if abs(k) < len(high) else 0.0
        assert abs(a_d[i, 2 * i + 1 + k] - want) < 2e-12


def test_lift97_synthesis_taps_match_published():
    taps = load_golden("cdf97_filters.txt")
    m = 32
    for band, name, centre in (("s", "synthesis_low", 32), ("d", "synthesis_high", 33)):
        s = np.zeros(m)
        d = np.zeros(m)
        (s if band == "s" else d)[16] = 1.0
        x = wv.inv97(s, d)
        t = taps[name]
        for k in range(-8, 9):
            want = t[abs(k)] if abs(k) < len(t) else 0.0
            assert abs(x[centre + k] - want) < 2e-12


def test_lift97_gains_and_constant():
    x = np.full(64, 3.5)
    s, d = wv.fwd97(x)
    assert np.max(np.abs(s - 3.5)) < 1e-12 and np.max(np.abs(d)) < 1e-12
    alt = np.array([(-1.0) ** k for k in range(64)])
    s, d = wv.fwd97(alt)
    assert np.max(np.abs(s)) < 1e-12
    assert np.max(np.abs(np.abs(d) - 2.0)) < 1e-9
    c = wv.fwd2d(np.full((64, 64), 200.0), 4, wv.W97)
    assert np.max(np.abs(c[:4, :4] - 200.0)) < 1e-9
    c[:4, :4] = 0
    assert np.max(np.abs(c)) < 1e-9


@pytest.mark.parametrize("n,levels", [(8, 2), (32, 4), (256, 4), (512, 4)])
def test_lift97_perfect_reconstruction(n, levels):
    rng = np.random.default_rng(n)
    x = rng.uniform(0, 255, (2, n, n))
    y = wv.inv2d(wv.fwd2d(x, levels, wv.W97), levels, wv.W97)
    assert np.max(np.abs(y - x)) < 1e-10


def test_lift97_zero_detail_is_lowpass_interpolation():
    """With zero details the 9/7 synthesis is the published synthesis low-pass
    applied to the zero-stuffed approximation (checked away from the edges)."""
    taps = load_golden("cdf97_filters.txt")["synthesis_low"]
    rng = np.random.default_rng(11)
    s = rng.uniform(-5, 5, 40)
    x = wv.inv97(s, np.zeros(40))
    up = np.zeros(80)
    up[0::2] = s
    for j in range(8, 72):
        want = sum(taps[abs(k)] * up[j - k] for k in range(-3, 4))
        assert abs(x[j] - want) < 1e-10


def test_subband_slices_partition():
    n, L = 64, 4
    cover = np.zeros((n, n), dtype=int)
    for _, _, r, c in wv.subband_slices(n, L):
        cover[r, c] += 1
    assert np.all(cover == 1)


def test_default_level_count_reading():
    """Section 3.1's default l_max = log2(N/32) - 2 gives 6 for 8k frames,
    the level count the paper reports as best for 8k."""
    assert int(np.log2(8192 / 32)) - 2 == 6
