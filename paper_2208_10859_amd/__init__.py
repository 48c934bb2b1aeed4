"""Viewport-dependent wavelet decoding of 360-degree frames on MI355X.

The decode runs in libwv (HIP kernels for gfx950 behind the C ABI of
include/wv.h); this package is its Python binding.  Build the library with
``python -m paper_2208_10859_amd.build``.  The binding is imported on first
use, so that the build module runs where the library does not exist yet.
"""
_EXPORTS = ("W53", "W97", "GRAY8", "YUV420", "PATH_FUSED", "PATH_PLAIN", "Decoder", "Reference",
            "BatchJob", "WvError", "decode_batch", "viewport_mask", "foveation_levels", "Server",
            "ViewClass")


def __getattr__(name):
    if name in _EXPORTS:
        from . import wv
        return getattr(wv, name)
    raise AttributeError(f"module {__name__!r} has no attribute {name!r}")
