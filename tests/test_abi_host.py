"""Host-only checks of the C ABI: the library loads, exports every symbol the
header declares, validates geometry before touching the device, and its
viewport selection equals the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

import wvinputs
from oracle import viewport

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols(name):
    txt = open(os.path.join(ROOT, "include", name)).read()
    return sorted(set(re.findall(r"\b(wv_[a-z_]+)\s*\(", txt)))


def test_library_exports_header_symbols():
    from paper_2208_10859_amd import cnn, fmt, wv
    lib = ctypes.CDLL(wv._LIB_PATH)
    headers = sorted(f for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h"))
    assert headers == ["wv.h", "wv_cnn.h", "wv_format.h"]
    syms = _header_symbols("wv.h")
    assert len(syms) >= 15
    for s in syms + _header_symbols("wv_cnn.h") + _header_symbols("wv_format.h"):
        assert hasattr(lib, s), s
    assert set(syms) == set(wv.EXPORTED)
    assert set(_header_symbols("wv_cnn.h")) == set(cnn.EXPORTED)
    assert set(_header_symbols("wv_format.h")) == set(fmt.EXPORTED)


def test_strerror_and_geometry_validation_without_device():
    from paper_2208_10859_amd import wv
    lib = wv.lib()
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.wv_strerror(code)
    ctx = ctypes.c_void_p()
    bad = [wv.make_desc(100, 512, 512, 3), wv.make_desc(512, 512, 48, 3),
           wv.make_desc(512, 512, 512, 0), wv.make_desc(512, 512, 512, 9, fmt=wv.YUV420),
           wv.make_desc(512, 512, 1024, 3), wv.make_desc(512, 512, 512, 3, wavelet=7)]
    for d in bad:
        assert lib.wv_create(ctypes.byref(ctx), ctypes.byref(d)) == wv.EINVAL
        assert lib.wv_last_error()
    assert lib.wv_create(None, ctypes.byref(bad[0])) == wv.EINVAL


def test_viewport_mask_and_foveation_match_oracle():
    from paper_2208_10859_amd import wv
    for g in range(40):
        yaw, pitch = wvinputs.head_pose(wvinputs.BASE_SEED, g)
        for eyes in (1, 2):
            a = wv.viewport_mask(8192, 8192, 512, yaw, pitch, eyes=eyes)
            b = viewport.tile_mask(8192, 8192, 512, yaw, pitch, eyes=eyes)
            assert np.array_equal(a, b)
        lc = wv.foveation_levels(8192, 8192, 512, 4, yaw, pitch)
        assert np.array_equal(lc, 4 - viewport.foveation_drop(8192, 8192, 512, yaw, pitch))
    # other geometry and fov
    a = wv.viewport_mask(4096, 2048, 256, 30.0, -10.0, fov_h=90.0, fov_v=100.0, samples=8)
    b = viewport.tile_mask(4096, 2048, 256, 30.0, -10.0, 90.0, 100.0, samples=8)
    assert np.array_equal(a, b)


def test_viewport_argument_errors():
    from paper_2208_10859_amd import wv
    with pytest.raises(wv.WvError):
        wv.viewport_mask(8192, 8192, 512, 0.0, 0.0, fov_h=180.0)
    with pytest.raises(wv.WvError):
        wv.viewport_mask(8192, 8192, 512, 0.0, 0.0, eyes=3)
