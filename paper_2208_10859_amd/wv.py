"""ctypes binding of libwv (include/wv.h), argument marshalling only.

Device buffers are torch tensors (torch provides device memory and streams);
every step of the decode runs in libwv's HIP kernels.  If libwv.so has not
been built, importing this module raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libwv.so")

W53, W97 = 0, 1
GRAY8, YUV420 = 0, 1
PATH_FUSED, PATH_PLAIN = 0, 1

OK, EINVAL, ESTALE, ENOMEM, EDEVICE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5


class WvError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"[{status}] {message}")
        self.status = status


class _Desc(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("levels", ctypes.c_int32), ("wavelet", ctypes.c_int32), ("format", ctypes.c_int32)]


class _Frame(ctypes.Structure):
    _fields_ = [("planes", ctypes.c_void_p * 3), ("frame_index", ctypes.c_int32),
                ("is_intra", ctypes.c_int32), ("qstep", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class _Set(ctypes.Structure):
    _fields_ = [("planes", ctypes.c_void_p * 3), ("n", ctypes.c_int32), ("qstep", ctypes.c_int32 * 4)]


class _Ref(ctypes.Structure):
    _fields_ = [("planes", ctypes.c_void_p * 3), ("tile_stamp", ctypes.POINTER(ctypes.c_int32))]


class _Job(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("coeffs", ctypes.POINTER(_Frame)),
                ("level_count", ctypes.c_void_p), ("tile_mask", ctypes.c_void_p),
                ("ref", ctypes.POINTER(_Ref)), ("out", ctypes.c_void_p)]


class ViewClass(ctypes.Structure):
    """How a client views the frame (wv_view_class)."""
    _fields_ = [("fov_h", ctypes.c_double), ("fov_v", ctypes.c_double), ("eyes", ctypes.c_int32),
                ("foveate", ctypes.c_int32), ("inner", ctypes.c_double), ("outer", ctypes.c_double)]

    def __init__(self, fov_h=110.0, fov_v=110.0, eyes=1, foveate=False, inner=20.0, outer=40.0):
        super().__init__(fov_h, fov_v, eyes, int(bool(foveate)), inner, outer)


class _StreamDesc(ctypes.Structure):
    _fields_ = [("source", ctypes.c_int32), ("n_frames", ctypes.c_int32),
                ("arrival", ctypes.c_void_p), ("yaw", ctypes.c_void_p), ("pitch", ctypes.c_void_p),
                ("view", ViewClass), ("out_frames", ctypes.c_void_p)]


class _ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("requests", "frames_decoded", "tiles_decoded",
                                               "catchup_tiles", "launches", "turns", "admitted",
                                               "max_active")] + \
               [(n, ctypes.c_double) for n in ("mpix", "wall_s", "gpu_ms", "p50_ms", "p99_ms",
                                                "max_ms", "mean_ms")]


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with `python -m paper_2208_10859_amd.build`")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i32, u8p = ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p
    sig = {
        "wv_create": (i32, [ctypes.POINTER(vp), ctypes.POINTER(_Desc)]),
        "wv_destroy": (i32, [vp]),
        "wv_strerror": (ctypes.c_char_p, [i32]),
        "wv_last_error": (ctypes.c_char_p, []),
        "wv_set_path": (i32, [vp, i32]),
        "wv_decode_viewport": (i32, [vp, ctypes.POINTER(_Frame), u8p, u8p, ctypes.POINTER(_Ref), vp, vp]),
        "wv_decode_batch": (i32, [i32, ctypes.POINTER(_Job), vp]),
        "wv_decode_viewport_noalloc": (i32, [ctypes.POINTER(_Desc), ctypes.POINTER(_Frame), u8p, u8p,
                                             ctypes.POINTER(_Ref), vp, vp]),
        "wv_decode_gop": (i32, [vp, i32, ctypes.POINTER(_Frame), u8p, u8p, ctypes.POINTER(_Ref), vp, vp]),
        "wv_decode_set": (i32, [vp, ctypes.POINTER(_Set), i32, i32, u8p, u8p, vp, vp]),
        "wv_viewport_mask": (i32, [ctypes.POINTER(_Desc), ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, i32, i32, u8p]),
        "wv_foveation_levels": (i32, [ctypes.POINTER(_Desc), ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, u8p]),
        "wv_encode_intra": (i32, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), i32, vp]),
        "wv_autotune": (i32, [vp, i32, i32, vp, ctypes.POINTER(i32)]),
        "wv_variant_count": (i32, [vp]),
        "wv_get_variant": (i32, [vp, ctypes.POINTER(i32)]),
        "wv_set_variant": (i32, [vp, i32]),
        "wv_variant_name": (ctypes.c_char_p, [vp, i32]),
        "wv_server_create": (i32, [ctypes.POINTER(vp), ctypes.POINTER(_Desc), i32, ctypes.c_int64, i32]),
        "wv_server_destroy": (i32, [vp]),
        "wv_server_slots": (i32, [vp]),
        "wv_server_add_source": (i32, [vp, i32, ctypes.POINTER(_Frame)]),
        "wv_server_add_stream": (i32, [vp, ctypes.POINTER(_StreamDesc)]),
        "wv_server_clear_streams": (i32, [vp]),
        "wv_server_run": (i32, [vp, ctypes.c_double, vp, ctypes.POINTER(_ServerStats), vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()

EXPORTED = ("wv_create", "wv_destroy", "wv_strerror", "wv_last_error", "wv_set_path",
            "wv_decode_viewport", "wv_decode_viewport_noalloc", "wv_decode_batch", "wv_decode_gop",
            "wv_decode_set",
            "wv_viewport_mask", "wv_foveation_levels",
            "wv_encode_intra", "wv_autotune", "wv_variant_count", "wv_get_variant",
            "wv_set_variant", "wv_variant_name", "wv_server_create", "wv_server_destroy",
            "wv_server_slots", "wv_server_add_source", "wv_server_add_stream",
            "wv_server_clear_streams", "wv_server_run")


def lib():
    return _lib


def _check(status: int):
    if status != OK:
        msg = _lib.wv_last_error().decode() or _lib.wv_strerror(status).decode()
        raise WvError(status, msg)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def make_desc(width, height, tile, levels, wavelet=W53, fmt=YUV420) -> _Desc:
    return _Desc(width, height, tile, levels, wavelet, fmt)


def viewport_mask(width, height, tile, yaw, pitch, fov_h=110.0, fov_v=110.0, samples=16, eyes=1):
    d = make_desc(width, height, tile, 1)
    m = np.zeros((width // tile) * (height // tile), dtype=np.uint8)
    _check(_lib.wv_viewport_mask(ctypes.byref(d), yaw, pitch, fov_h, fov_v, samples, eyes, _np_ptr(m)))
    return m


def foveation_levels(width, height, tile, levels, yaw, pitch, inner=20.0, outer=40.0):
    d = make_desc(width, height, tile, levels)
    lc = np.zeros((width // tile) * (height // tile), dtype=np.uint8)
    _check(_lib.wv_foveation_levels(ctypes.byref(d), yaw, pitch, inner, outer, _np_ptr(lc)))
    return lc


class Reference:
    """Reconstruction state of one stream: device planes + host stamps."""

    def __init__(self, decoder: "Decoder", device="cuda"):
        self.planes = [torch.zeros(decoder.plane_shape(p), dtype=decoder.sample_dtype, device=device)
                       for p in range(decoder.nplanes)]
        self.stamp = np.full(decoder.n_tiles, -1, dtype=np.int32)
        self._c = _Ref()
        self._refresh()

    def _refresh(self):
        for p in range(3):
            self._c.planes[p] = self.planes[p].data_ptr() if p < len(self.planes) else None
        self._c.tile_stamp = self.stamp.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


class Decoder:
    """One libwv context (geometry fixed at creation)."""

    def __init__(self, width, height, tile, levels, wavelet=W53, fmt=YUV420):
        self.width, self.height, self.tile, self.levels = width, height, tile, levels
        self.wavelet, self.fmt = wavelet, fmt
        self.nplanes = 3 if fmt == YUV420 else 1
        self.n_tiles = (width // tile) * (height // tile)
        self.coef_dtype = torch.int16 if wavelet == W53 else torch.float32
        self.sample_dtype = torch.uint8 if wavelet == W53 else torch.float32
        self._desc = make_desc(width, height, tile, levels, wavelet, fmt)
        self._ctx = ctypes.c_void_p()
        _check(_lib.wv_create(ctypes.byref(self._ctx), ctypes.byref(self._desc)))

    def close(self):
        if self._ctx:
            _lib.wv_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # geometry helpers
    def plane_edge(self, p):
        return self.tile if p == 0 else self.tile // 2

    def plane_shape(self, p):
        e = self.plane_edge(p)
        return (self.n_tiles, e, e)

    def out_shape(self, n_visible):
        return (n_visible, 3 if self.fmt == YUV420 else 1, self.tile, self.tile)

    def set_path(self, path):
        _check(_lib.wv_set_path(self._ctx, path))

    def _check_planes(self, planes, dtype, what):
        if len(planes) < self.nplanes:
            raise ValueError(f"{what}: need {self.nplanes} planes")
        for p in range(self.nplanes):
            t = planes[p]
            need = self.n_tiles * self.plane_edge(p) ** 2
            if (not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != dtype
                    or not t.is_contiguous() or t.numel() < need):
                raise ValueError(f"{what}[{p}]: need a contiguous {dtype} CUDA tensor with at least "
                                 f"{need} elements")

    def _check_out(self, out, n_visible):
        if out is None:
            return
        need = n_visible * (3 if self.fmt == YUV420 else 1) * self.tile * self.tile
        if (out.device.type != "cuda" or out.dtype != self.sample_dtype or not out.is_contiguous()
                or out.numel() < need):
            raise ValueError(f"out: need a contiguous {self.sample_dtype} CUDA tensor with at least "
                             f"{need} elements")

    def frame(self, planes, frame_index, is_intra, qstep=1) -> _Frame:
        self._check_planes(planes, self.coef_dtype, "coefficient planes")
        f = _Frame()
        for p in range(3):
            f.planes[p] = planes[p].data_ptr() if p < len(planes) and planes[p] is not None else None
        f.frame_index, f.is_intra, f.qstep, f.reserved = frame_index, int(bool(is_intra)), qstep, 0
        return f

    def decode_viewport(self, planes, frame_index, is_intra, qstep, mask, ref: Reference,
                        out=None, level_count=None, stream=None):
        f = self.frame(planes, frame_index, is_intra, qstep)
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        if mask.size != self.n_tiles:
            raise ValueError("mask must have one entry per tile")
        self._check_out(out, int(np.count_nonzero(mask)))
        lc = None if level_count is None else np.ascontiguousarray(level_count, dtype=np.uint8)
        if lc is not None and lc.size != self.n_tiles:
            raise ValueError("level_count must have one entry per tile")
        self._check_ref(ref)
        _check(_lib.wv_decode_viewport(self._ctx, ctypes.byref(f), _np_ptr(lc), _np_ptr(mask),
                                       ctypes.byref(ref._c), _ptr(out), _stream(stream)))

    def decode_gop(self, frames, first_index, mask, ref: Reference, outs=None, level_count=None,
                   stream=None):
        """Consecutive frames of one viewport in one call.  frames: list of
        (planes, is_intra, qstep); outs: list of output tensors (or None)."""
        n = len(frames)
        arr = (_Frame * n)()
        for i, (planes, intra, qstep) in enumerate(frames):
            arr[i] = self.frame(planes, first_index + i, intra, qstep)
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        if mask.size != self.n_tiles:
            raise ValueError("mask must have one entry per tile")
        nvis = int(np.count_nonzero(mask))
        optr = None
        if outs is not None:
            if len(outs) != n:
                raise ValueError("outs needs one entry per frame")
            for o in outs:
                self._check_out(o, nvis)
            optr = (ctypes.c_void_p * n)(*[None if o is None else o.data_ptr() for o in outs])
        lc = None if level_count is None else np.ascontiguousarray(level_count, dtype=np.uint8)
        if lc is not None and lc.size != self.n_tiles:
            raise ValueError("level_count must have one entry per tile")
        self._check_ref(ref)
        _check(_lib.wv_decode_gop(self._ctx, n, arr, _np_ptr(lc), _np_ptr(mask), ctypes.byref(ref._c),
                                  ctypes.cast(optr, ctypes.c_void_p) if optr is not None else None,
                                  _stream(stream)))

    def set_shape(self, n, p):
        """Shape of plane p's bands of an inter-frame set of n frames."""
        return (n,) + self.plane_shape(p)

    def decode_set(self, bands, n, qsteps, t0, mask, outs, level_count=None, stream=None):
        """Frames t0 .. t0 + len(outs) - 1 of an inter-frame set in one launch.
        bands: per plane a contiguous device tensor [n][n_tiles][P][P];
        qsteps: per band dequantisation steps (5/3)."""
        if len(bands) < self.nplanes:
            raise ValueError(f"bands: need {self.nplanes} planes")
        for p in range(self.nplanes):
            b = bands[p]
            if (not isinstance(b, torch.Tensor) or b.device.type != "cuda" or b.dtype != self.coef_dtype
                    or not b.is_contiguous() or b.numel() < n * self.n_tiles * self.plane_edge(p) ** 2):
                raise ValueError(f"bands[{p}]: need a contiguous {self.coef_dtype} CUDA tensor of "
                                 f"{self.set_shape(n, p)}")
        st = _Set()
        for p in range(3):
            st.planes[p] = bands[p].data_ptr() if p < self.nplanes else None
        st.n = n
        q = list(qsteps) + [1] * (4 - len(qsteps))
        for b in range(4):
            st.qstep[b] = int(q[b])
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        if mask.size != self.n_tiles:
            raise ValueError("mask must have one entry per tile")
        nvis = int(np.count_nonzero(mask))
        for o in outs:
            if o is None:
                raise ValueError("every frame needs an output")
            self._check_out(o, nvis)
        optr = (ctypes.c_void_p * max(1, len(outs)))(*[o.data_ptr() for o in outs])
        lc = None if level_count is None else np.ascontiguousarray(level_count, dtype=np.uint8)
        if lc is not None and lc.size != self.n_tiles:
            raise ValueError("level_count must have one entry per tile")
        _check(_lib.wv_decode_set(self._ctx, ctypes.byref(st), t0, len(outs), _np_ptr(lc),
                                  _np_ptr(mask), ctypes.cast(optr, ctypes.c_void_p), _stream(stream)))

    def _check_ref(self, ref):
        self._check_planes(ref.planes, self.sample_dtype, "reference planes")
        if ref.stamp.size != self.n_tiles or ref.stamp.dtype != np.int32:
            raise ValueError("reference stamps must be int32 with one entry per tile")

    def encode_intra(self, src_planes, coef_planes, qstep, stream=None):
        self._check_planes(src_planes, torch.uint8, "source planes")
        self._check_planes(coef_planes, self.coef_dtype, "coefficient planes")
        src = (ctypes.c_void_p * 3)(*[p.data_ptr() for p in src_planes], *([None] * (3 - len(src_planes))))
        dst = (ctypes.c_void_p * 3)(*[p.data_ptr() for p in coef_planes], *([None] * (3 - len(coef_planes))))
        _check(_lib.wv_encode_intra(self._ctx, src, dst, qstep, _stream(stream)))

    def autotune(self, n_visible, reps=10, stream=None):
        best = ctypes.c_int32()
        _check(_lib.wv_autotune(self._ctx, n_visible, reps, _stream(stream), ctypes.byref(best)))
        return best.value

    def variants(self):
        return [_lib.wv_variant_name(self._ctx, v).decode() for v in range(_lib.wv_variant_count(self._ctx))]

    @property
    def variant(self):
        v = ctypes.c_int32()
        _check(_lib.wv_get_variant(self._ctx, ctypes.byref(v)))
        return v.value

    @variant.setter
    def variant(self, v):
        _check(_lib.wv_set_variant(self._ctx, v))


class BatchJob:
    """One viewport decode inside decode_batch (keeps its ctypes structs alive)."""

    def __init__(self, decoder: Decoder, planes, frame_index, is_intra, qstep, mask, ref: Reference,
                 out=None, level_count=None):
        self.decoder = decoder
        self.frame = decoder.frame(planes, frame_index, is_intra, qstep)
        self.mask = np.ascontiguousarray(mask, dtype=np.uint8)
        if self.mask.size != decoder.n_tiles:
            raise ValueError("mask must have one entry per tile")
        decoder._check_out(out, int(np.count_nonzero(self.mask)))
        self.lc = None if level_count is None else np.ascontiguousarray(level_count, dtype=np.uint8)
        if self.lc is not None and self.lc.size != decoder.n_tiles:
            raise ValueError("level_count must have one entry per tile")
        decoder._check_ref(ref)
        self.ref = ref
        self.out = out


def decode_batch(jobs, stream=None):
    arr = (_Job * len(jobs))()
    for i, j in enumerate(jobs):
        arr[i].ctx = j.decoder._ctx
        arr[i].coeffs = ctypes.pointer(j.frame)
        arr[i].level_count = _np_ptr(j.lc)
        arr[i].tile_mask = _np_ptr(j.mask)
        arr[i].ref = ctypes.pointer(j.ref._c)
        arr[i].out = _ptr(j.out)
    _check(_lib.wv_decode_batch(len(jobs), arr, _stream(stream)))


class Server:
    """Continuous-batching serving loop over many head-tracked streams."""

    def __init__(self, width, height, tile, levels, wavelet=W53, fmt=YUV420, max_active=64,
                 hbm_budget=64 << 30, max_visible=None):
        self._geom = Decoder(width, height, tile, levels, wavelet, fmt)
        self.max_visible = self._geom.n_tiles if max_visible is None else int(max_visible)
        self._desc = make_desc(width, height, tile, levels, wavelet, fmt)
        h = ctypes.c_void_p()
        _check(_lib.wv_server_create(ctypes.byref(h), ctypes.byref(self._desc), max_active,
                                     int(hbm_budget), self.max_visible))
        self._srv = h
        self._sources = []   # keeps source tensors alive
        self._streams = []   # keeps output tensors alive, and the request counts
        self.n_sources = 0

    def close(self):
        if getattr(self, "_srv", None):
            _lib.wv_server_destroy(self._srv)
            self._srv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def slots(self):
        return _lib.wv_server_slots(self._srv)

    def out_shape(self):
        return self._geom.out_shape(self.max_visible)

    def add_source(self, frames):
        """frames: list of (planes, qstep), frame 0 intra.  Returns the source index."""
        arr = (_Frame * len(frames))()
        for i, (planes, qstep) in enumerate(frames):
            arr[i] = self._geom.frame(planes, i, i == 0, qstep)
        _check(_lib.wv_server_add_source(self._srv, len(frames), arr))
        self._sources.append(frames)
        self.n_sources += 1
        return self.n_sources - 1

    def add_stream(self, source, arrival, yaw, pitch, view: ViewClass = None, outs=None):
        arrival = np.ascontiguousarray(arrival, dtype=np.float64)
        yaw = np.ascontiguousarray(yaw, dtype=np.float64)
        pitch = np.ascontiguousarray(pitch, dtype=np.float64)
        n = arrival.size
        if yaw.size != n or pitch.size != n:
            raise ValueError("arrival, yaw and pitch need one entry per frame")
        d = _StreamDesc()
        d.source, d.n_frames = source, n
        d.arrival, d.yaw, d.pitch = _np_ptr(arrival), _np_ptr(yaw), _np_ptr(pitch)
        d.view = view if view is not None else ViewClass()
        keep = None
        if outs is not None:
            if len(outs) != n:
                raise ValueError("outs needs one tensor per frame")
            for o in outs:
                self._geom._check_out(o, self.max_visible)
            keep = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
            d.out_frames = ctypes.cast(keep, ctypes.c_void_p)
        _check(_lib.wv_server_add_stream(self._srv, ctypes.byref(d)))
        self._streams.append((n, outs))

    def clear_streams(self):
        _check(_lib.wv_server_clear_streams(self._srv))
        self._streams = []

    def run(self, time_scale=1.0, stream=None):
        """Play the queued streams; returns (latency_ms per request, stats dict)."""
        total = sum(n for n, _ in self._streams)
        lat = np.zeros(total, dtype=np.float64)
        st = _ServerStats()
        _check(_lib.wv_server_run(self._srv, float(time_scale), _np_ptr(lat), ctypes.byref(st),
                                  _stream(stream)))
        return lat, {n: getattr(st, n) for n, _ in _ServerStats._fields_}
