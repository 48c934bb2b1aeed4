"""Frame-wise wavelet transforms: plain int64 / float64 definitions.

Section 3.1 of the paper: a 2D fast wavelet transform where each level halves
the approximation in both directions; the paper's own wavelet is CDF 9/7
(Cohen-Daubechies-Feauveau, the JPEG 2000 irreversible filter), and Section 2.2
names LeGall 5/3 as JPEG 2000's lossless wavelet.  Both are written here as
the JPEG 2000 Part 1 lifting factorisations:

* LeGall 5/3 reversible integer lifting (predict with floor((a+b)/2), update
  with floor((a+b+2)/4));
* CDF 9/7 irreversible lifting, steps alpha, beta, gamma, delta, then scaling
  of the low band by 1/K and the high band by K (low-pass DC gain 1, high-pass
  Nyquist gain 2).

Readings (the paper is silent on these):
* boundary: whole-sample symmetric extension, x[-1] = x[1], x[n] = x[n-2];
  in lifting form the even channel is extended by e[m] = e[m-1] at the right
  end and the odd channel by o[-1] = o[0] at the left end;
* 1D layout: low band in the first half, high band in the second half;
* 2D pass order: forward level = every column (vertical) then every row;
  inverse level = every row then every column (the exact reverse);
* multi-level layout (Mallat): level l operates on the top-left region of
  size n / 2**(l-1); after the forward level its top-left quarter is LL.
"""
from __future__ import annotations

import numpy as np

# CDF 9/7 lifting constants (JPEG 2000 Part 1 irreversible 9/7 factorisation).
ALPHA = -1.586134342059924
BETA = -0.052980118572961
GAMMA = 0.882911075530934
DELTA = 0.443506852043971
KAPPA = 1.230174104914001

W53 = "5/3"
W97 = "9/7"


def _next(v):
    """v[i+1] along the last axis, with v[m] := v[m-1] (right end of the even channel)."""
    return np.concatenate([v[..., 1:], v[..., -1:]], axis=-1)


def _prev(v):
    """v[i-1] along the last axis, with v[-1] := v[0] (left end of the odd channel)."""
    return np.concatenate([v[..., :1], v[..., :-1]], axis=-1)


def _interleave(e, o):
    x = np.empty(e.shape[:-1] + (2 * e.shape[-1],), dtype=e.dtype)
    x[..., 0::2] = e
    x[..., 1::2] = o
    return x


# ---------------------------------------------------------------- LeGall 5/3
def fwd53(x):
    """1D forward 5/3 along the last axis (int64, even length) -> (s, d)."""
    x = np.asarray(x, dtype=np.int64)
    assert x.shape[-1] % 2 == 0 and x.shape[-1] >= 2
    e = x[..., 0::2]
    o = x[..., 1::2]
    d = o - ((e + _next(e)) >> 1)           # predict: odd minus floor of the mean of its even neighbours
    s = e + ((_prev(d) + d + 2) >> 2)       # update: even plus rounded quarter of its odd neighbours
    return s, d


def inv53(s, d):
    """1D inverse 5/3: (s, d) -> x along the last axis (int64)."""
    s = np.asarray(s, dtype=np.int64)
    d = np.asarray(d, dtype=np.int64)
    e = s - ((_prev(d) + d + 2) >> 2)       # undo the update
    o = d + ((e + _next(e)) >> 1)           # undo the predict
    return _interleave(e, o)


# ------------------------------------------------------------------ CDF 9/7
def fwd97(x):
    """1D forward CDF 9/7 along the last axis (float64, even length) -> (s, d)."""
    x = np.asarray(x, dtype=np.float64)
    assert x.shape[-1] % 2 == 0 and x.shape[-1] >= 2
    e = x[..., 0::2].copy()
    o = x[..., 1::2].copy()
    o = o + ALPHA * (e + _next(e))
    e = e + BETA * (_prev(o) + o)
    o = o + GAMMA * (e + _next(e))
    e = e + DELTA * (_prev(o) + o)
    return e / KAPPA, o * KAPPA


def inv97(s, d):
    """1D inverse CDF 9/7: (s, d) -> x along the last axis (float64)."""
    e = np.asarray(s, dtype=np.float64) * KAPPA
    o = np.asarray(d, dtype=np.float64) / KAPPA
    e = e - DELTA * (_prev(o) + o)
    o = o - GAMMA * (e + _next(e))
    e = e - BETA * (_prev(o) + o)
    o = o - ALPHA * (e + _next(e))
    return _interleave(e, o)


_FWD = {W53: fwd53, W97: fwd97}
_INV = {W53: inv53, W97: inv97}


def _fwd_axis(x, axis, wavelet):
    x = np.moveaxis(x, axis, -1)
    s, d = _FWD[wavelet](x)
    return np.moveaxis(np.concatenate([s, d], axis=-1), -1, axis)


def _inv_axis(c, axis, wavelet):
    c = np.moveaxis(c, axis, -1)
    m = c.shape[-1] // 2
    x = _INV[wavelet](c[..., :m], c[..., m:])
    return np.moveaxis(x, -1, axis)


def _dtype(wavelet):
    return np.int64 if wavelet == W53 else np.float64


def fwd2d(x, levels, wavelet=W53):
    """Multi-level 2D forward transform of the last two axes (Mallat layout).

    Per level on the top-left region: columns first, then rows.
    """
    c = np.array(x, dtype=_dtype(wavelet), copy=True)
    h, w = c.shape[-2:]
    for lev in range(levels):
        hh, ww = h >> lev, w >> lev
        assert hh % 2 == 0 and ww % 2 == 0, "region must stay even at every level"
        r = c[..., :hh, :ww]
        r = _fwd_axis(r, -2, wavelet)   # vertical (every column)
        r = _fwd_axis(r, -1, wavelet)   # horizontal (every row)
        c[..., :hh, :ww] = r
    return c


def inv2d(c, levels, wavelet=W53):
    """Multi-level 2D inverse transform (Mallat layout), coarsest level first.

    Per level on the top-left region: rows first, then columns.
    """
    x = np.array(c, dtype=_dtype(wavelet), copy=True)
    h, w = x.shape[-2:]
    for lev in reversed(range(levels)):
        hh, ww = h >> lev, w >> lev
        r = x[..., :hh, :ww]
        r = _inv_axis(r, -1, wavelet)   # horizontal (every row)
        r = _inv_axis(r, -2, wavelet)   # vertical (every column)
        x[..., :hh, :ww] = r
    return x


def zero_finest(c, drop):
    """Zero the detail bands of the finest ``drop`` levels (foveation, Section 3.7).

    Level 1 is the finest: its region is the whole tile; its detail bands are
    every sample outside the top-left quarter.  Level k's region is
    n / 2**(k-1).  The approximation of the coarsest kept level is untouched.
    """
    c = np.array(c, copy=True)
    h, w = c.shape[-2:]
    for lev in range(drop):
        hh, ww = h >> lev, w >> lev
        c[..., :hh // 2, ww // 2:ww] = 0
        c[..., hh // 2:hh, :ww] = 0
    return c


def subband_slices(n, levels):
    """Index slices of every subband of an n x n Mallat layout.

    Returns a list of (name, level, rows, cols); level 1 is the finest.
    """
    out = []
    for lev in range(1, levels + 1):
        m = n >> (lev - 1)
        h = m // 2
        out.append(("HL", lev, slice(0, h), slice(h, m)))
        out.append(("LH", lev, slice(h, m), slice(0, h)))
        out.append(("HH", lev, slice(h, m), slice(h, m)))
    m = n >> levels
    out.append(("LL", levels, slice(0, m), slice(0, m)))
    return out
