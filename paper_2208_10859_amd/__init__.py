"""Viewport-dependent wavelet decoding of 360-degree frames on MI355X.

The decode runs in libwv (HIP kernels for gfx950 behind the C ABI of
include/wv.h); this package is its Python binding.  Build the library with
``python -m paper_2208_10859_amd.build``.
"""
from .wv import (  # noqa: F401
    W53, W97, GRAY8, YUV420, PATH_FUSED, PATH_PLAIN, Decoder, Reference, BatchJob, WvError,
    decode_batch, viewport_mask, foveation_levels,
)
