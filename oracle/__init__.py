"""CPU oracle for the viewport-dependent wavelet decoder.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this package.
The product (``paper_2208_10859_amd``) never imports it, and this package never
imports the product: the two share no code.  The only shared module is
``wvinputs`` (seeded synthetic inputs, no codec arithmetic).

It is a plain, slow and obviously-correct restatement of what the decoder
computes, in int64 (LeGall 5/3) and float64 (CDF 9/7):

* ``wavelet``  -- 1D/2D lifting transforms, forward and inverse (Section 3.1);
* ``colour``   -- YUV420 -> RGB (JFIF full range, Q16 fixed point / float);
* ``viewport`` -- tile mask from a head pose, foveation level drop (Sections 3.1, 3.6, 3.7);
* ``codec``    -- quantiser, intra encoder, and the full decode definition:
  dequantise -> zero dropped levels -> inverse transform -> residual chain ->
  colour, restricted to each frame's mask;
* ``interframe`` -- the temporal Haar transform of inter-frame sets (Section
  3.2) and the decode of one frame of a set;
* ``paperformat`` -- the paper's storage format (thresholds of Eq. 2/3 with the
  pole factor, Eq. 4 8-bit quantisation, 32 x 32 blocks with block-end
  pointers) and the rebuild of dense planes from it.

Every reading the paper leaves open (boundary extension, pass order, residual
model, quantiser, colour) is stated where it is used.
"""
from . import wavelet, colour, viewport, codec, interframe, paperformat  # noqa: F401
