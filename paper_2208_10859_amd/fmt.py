"""ctypes binding of the sparse storage format (include/wv_format.h): argument
marshalling only; the encoder and the GPU rebuild run in libwv."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import wv as _wv

_lib = _wv.lib()
_vp, _i32, _i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64


class SparsePlane(ctypes.Structure):
    _fields_ = [("block_end", _vp), ("values", _vp), ("index", _vp), ("n_records", _i64),
                ("bounds", ctypes.c_float * 4)]


for _name, _res, _args in [
    ("wv_sparse_blocks_per_tile", _i32, [ctypes.POINTER(_wv._Desc), _i32]),
    ("wv_sparse_encode_plane", _i32, [ctypes.POINTER(_wv._Desc), _i32, _vp, ctypes.c_double, _i32,
                                      _vp, _vp, _vp, ctypes.POINTER(_i64), _vp]),
    ("wv_sparse_rebuild", _i32, [_vp, ctypes.POINTER(SparsePlane), _vp, _vp, _vp, _vp]),
    ("wv_sparse_visible_runs", _i32, [ctypes.POINTER(_wv._Desc), _i32, _vp, _i64, _vp, _vp, _vp, _vp,
                                      ctypes.POINTER(_i32), ctypes.POINTER(_i64)]),
    ("wv_prefetch_create", _i32, [_vp, _i32, _i64, ctypes.POINTER(_vp)]),
    ("wv_prefetch_destroy", _i32, [_vp]),
    ("wv_prefetch_stage", _i32, [_vp, ctypes.POINTER(SparsePlane), _i32, _vp, _vp, _i32,
                                 ctypes.POINTER(_i64)]),
    ("wv_prefetch_rebuild", _i32, [_vp, _vp, _vp]),
    ("wv_store_write", _i32, [ctypes.c_char_p, ctypes.POINTER(_wv._Desc), _i32, ctypes.POINTER(SparsePlane)]),
    ("wv_store_open", _i32, [ctypes.c_char_p, _i32, ctypes.POINTER(_vp)]),
    ("wv_store_close", _i32, [_vp]),
    ("wv_store_info", _i32, [_vp, ctypes.POINTER(_wv._Desc), ctypes.POINTER(_i32)]),
    ("wv_store_frame", _i32, [_vp, _i32, ctypes.POINTER(SparsePlane)]),
]:
    _fn = getattr(_lib, _name)
    _fn.restype, _fn.argtypes = _res, _args

EXPORTED = ("wv_sparse_blocks_per_tile", "wv_sparse_encode_plane", "wv_sparse_rebuild",
            "wv_sparse_visible_runs", "wv_prefetch_create", "wv_prefetch_destroy", "wv_prefetch_stage",
            "wv_prefetch_rebuild", "wv_store_write", "wv_store_open", "wv_store_close", "wv_store_info",
            "wv_store_frame")


def blocks_per_tile(desc, plane):
    return int(_lib.wv_sparse_blocks_per_tile(ctypes.byref(desc), plane))


def encode_plane(desc, plane, coef, alpha, poles):
    """One plane of one frame (host float32 [n_tiles, P, P]) -> dict of host
    arrays block_end (uint32), values (uint8), index (uint16), bounds (float32[4])."""
    coef = np.ascontiguousarray(coef, dtype=np.float32)
    nb = blocks_per_tile(desc, plane)
    if nb == 0:
        raise ValueError("bad geometry or plane")
    edge = desc.tile if plane == 0 else desc.tile // 2
    n_tiles = (desc.width // desc.tile) * (desc.height // desc.tile)
    if coef.shape != (n_tiles, edge, edge):
        raise ValueError(f"coef must be float32 [{n_tiles}, {edge}, {edge}]")
    block_end = np.zeros(n_tiles * nb, np.uint32)
    values = np.empty(coef.size, np.uint8)
    index = np.empty(coef.size, np.uint16)
    bounds = np.zeros(4, np.float32)
    n = _i64()
    _wv._check(_lib.wv_sparse_encode_plane(ctypes.byref(desc), plane, coef.ctypes.data, float(alpha),
                                           int(bool(poles)), block_end.ctypes.data, values.ctypes.data,
                                           index.ctypes.data, ctypes.byref(n), bounds.ctypes.data))
    return {"block_end": block_end, "values": values[:n.value].copy(),
            "index": index[:n.value].copy(), "bounds": bounds}


class DevicePlane:
    """One encoded plane moved to the device (torch tensors kept alive)."""

    def __init__(self, enc, device="cuda"):
        self.block_end = torch.from_numpy(enc["block_end"].view(np.int32)).to(device)
        n = enc["values"].size
        # at least one element so that the pointers are valid
        self.values = torch.from_numpy(enc["values"] if n else np.zeros(1, np.uint8)).to(device)
        self.index = torch.from_numpy((enc["index"] if n else np.zeros(1, np.uint16)).view(np.int16)).to(device)
        self.n_records = n
        self.bounds = [float(b) for b in enc["bounds"]]

    def nbytes(self):
        return self.block_end.numel() * 4 + self.n_records * 3

    def c(self):
        s = SparsePlane()
        s.block_end, s.values, s.index = (self.block_end.data_ptr(), self.values.data_ptr(),
                                          self.index.data_ptr())
        s.n_records = self.n_records
        for i in range(4):
            s.bounds[i] = self.bounds[i]
        return s


def rebuild(dec, planes, mask, dense, level_count=None, stream=None):
    """Rebuild the visible tiles' dense planes (device tensors shaped like the
    decoder's coefficient planes) from DevicePlane objects."""
    if len(planes) < dec.nplanes or len(dense) < dec.nplanes:
        raise ValueError(f"need {dec.nplanes} planes")
    dec._check_planes(dense, dec.coef_dtype, "dense planes")
    arr = (SparsePlane * dec.nplanes)(*[planes[p].c() for p in range(dec.nplanes)])
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    if mask.size != dec.n_tiles:
        raise ValueError("mask must have one entry per tile")
    lc = None if level_count is None else np.ascontiguousarray(level_count, dtype=np.uint8)
    if lc is not None and lc.size != dec.n_tiles:
        raise ValueError("level_count must have one entry per tile")
    dptr = (ctypes.c_void_p * 3)(*[d.data_ptr() for d in dense[:dec.nplanes]],
                                 *([None] * (3 - dec.nplanes)))
    _wv._check(_lib.wv_sparse_rebuild(dec._ctx, arr, _wv._np_ptr(lc), _wv._np_ptr(mask),
                                      ctypes.cast(dptr, ctypes.c_void_p), _wv._stream(stream)))


def visible_runs(desc, plane, enc, mask, level_count=None):
    """Merged record runs of the visible tiles of one encoded plane (host):
    (begin int64 [n], end int64 [n], records in them)."""
    be = np.ascontiguousarray(enc["block_end"], dtype=np.uint32)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    lc = None if level_count is None else np.ascontiguousarray(level_count, dtype=np.uint8)
    n_tiles = mask.size
    rb, re_ = np.zeros(n_tiles, np.int64), np.zeros(n_tiles, np.int64)
    n, tot = _i32(), _i64()
    _wv._check(_lib.wv_sparse_visible_runs(ctypes.byref(desc), plane, be.ctypes.data, int(enc["values"].size),
                                           _wv._np_ptr(lc), _wv._np_ptr(mask), rb.ctypes.data,
                                           re_.ctypes.data, ctypes.byref(n), ctypes.byref(tot)))
    return rb[:n.value].copy(), re_[:n.value].copy(), tot.value


def _pinned(a, dtype):
    """A copy of host array a in pinned (page-locked) host memory, at least
    one element long so that its pointer is valid."""
    a = np.ascontiguousarray(a, dtype=dtype)
    t = torch.empty(max(a.size, 1), dtype=getattr(torch, np.dtype(dtype).name), pin_memory=True)
    out = t.numpy()
    out[:a.size] = a
    return t, out


class HostPlane:
    """One encoded plane kept in pinned host memory: the store the prefetcher
    reads from."""

    def __init__(self, enc):
        self._be_t, self.block_end = _pinned(enc["block_end"].view(np.int32), np.int32)
        self._val_t, self.values = _pinned(enc["values"], np.uint8)
        self._idx_t, self.index = _pinned(enc["index"].view(np.int16), np.int16)
        self.n_records = int(enc["values"].size)
        self.bounds = [float(b) for b in enc["bounds"]]
        s = SparsePlane()
        s.block_end, s.values, s.index = (self.block_end.ctypes.data, self.values.ctypes.data,
                                          self.index.ctypes.data)
        s.n_records = self.n_records
        for i in range(4):
            s.bounds[i] = self.bounds[i]
        self._c = s

    def nbytes(self):
        return self.block_end.size * 4 + self.n_records * 3

    def c(self):
        return self._c


class Prefetcher:
    """Staging of the next inter-frame set from a host store while the GPU
    rebuilds and decodes the previous one (wv_prefetch_*)."""

    def __init__(self, dec, max_frames, slot_bytes):
        self.dec = dec
        self._pf = ctypes.c_void_p()
        _wv._check(_lib.wv_prefetch_create(dec._ctx, max_frames, int(slot_bytes), ctypes.byref(self._pf)))

    def close(self):
        if self._pf:
            _lib.wv_prefetch_destroy(self._pf)
            self._pf = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stage(self, frames, mask, level_count=None, direct=False):
        """frames: list over frames of lists over planes of HostPlane.
        Returns the bytes uploaded."""
        np_ = self.dec.nplanes
        flat = [f[p].c() for f in frames for p in range(np_)]
        arr = (SparsePlane * len(flat))(*flat)
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        if mask.size != self.dec.n_tiles:
            raise ValueError("mask must have one entry per tile")
        lc = None if level_count is None else np.ascontiguousarray(level_count, dtype=np.uint8)
        if lc is not None and lc.size != self.dec.n_tiles:
            raise ValueError("level_count must have one entry per tile")
        n = _i64()
        _wv._check(_lib.wv_prefetch_stage(self._pf, arr, len(frames), _wv._np_ptr(lc), _wv._np_ptr(mask),
                                          int(bool(direct)), ctypes.byref(n)))
        return n.value

    def rebuild(self, dense, stream=None):
        """dense: flat list [n_frames * nplanes] of device planes."""
        np_ = self.dec.nplanes
        for i, d in enumerate(dense):
            need = self.dec.n_tiles * self.dec.plane_edge(i % np_) ** 2
            if (not isinstance(d, torch.Tensor) or d.device.type != "cuda" or d.dtype != self.dec.coef_dtype
                    or not d.is_contiguous() or d.numel() < need):
                raise ValueError(f"dense[{i}]: need a contiguous {self.dec.coef_dtype} CUDA tensor with at "
                                 f"least {need} elements")
        ptrs = (ctypes.c_void_p * len(dense))(*[d.data_ptr() for d in dense])
        _wv._check(_lib.wv_prefetch_rebuild(self._pf, ctypes.cast(ptrs, ctypes.c_void_p), _wv._stream(stream)))


def _host_plane(enc):
    """SparsePlane over the host arrays of an encode_plane result (kept alive
    by the caller)."""
    sp = SparsePlane()
    sp.block_end = enc["block_end"].ctypes.data
    sp.values = enc["values"].ctypes.data if enc["values"].size else None
    sp.index = enc["index"].ctypes.data if enc["index"].size else None
    sp.n_records = int(enc["values"].size)
    for i in range(4):
        sp.bounds[i] = float(enc["bounds"][i])
    return sp


def write_store(path, desc, frames):
    """frames: list over frames of lists over planes of encode_plane results."""
    keep = [{k: np.ascontiguousarray(v) for k, v in e.items()} for f in frames for e in f]
    arr = (SparsePlane * len(keep))(*[_host_plane(e) for e in keep])
    _wv._check(_lib.wv_store_write(str(path).encode(), ctypes.byref(desc), len(frames), arr))


class _StorePlane:
    def __init__(self, store, sp):
        self._store, self._c = store, sp
        self.n_records = int(sp.n_records)
        self.block_end_count = 0

    def c(self):
        return self._c

    def nbytes(self):
        return self.block_end_count * 4 + self.n_records * 3


class Store:
    """A file of the format read into host memory (pinned by default), the
    store a Prefetcher stages from (wv_store_*)."""

    def __init__(self, path, pinned=True):
        self._h = ctypes.c_void_p()
        _wv._check(_lib.wv_store_open(str(path).encode(), int(bool(pinned)), ctypes.byref(self._h)))
        self.desc = _wv._Desc()
        n = _i32()
        _wv._check(_lib.wv_store_info(self._h, ctypes.byref(self.desc), ctypes.byref(n)))
        self.n_frames = n.value
        self.nplanes = 3 if self.desc.format == _wv.YUV420 else 1

    def close(self):
        if self._h:
            _lib.wv_store_close(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def frame(self, f):
        """The planes of frame f (pointing into the store) as stage() takes them."""
        arr = (SparsePlane * self.nplanes)()
        _wv._check(_lib.wv_store_frame(self._h, f, arr))
        n_tiles = (self.desc.width // self.desc.tile) * (self.desc.height // self.desc.tile)
        out = []
        for p in range(self.nplanes):
            sp = _StorePlane(self, arr[p])
            sp.block_end_count = n_tiles * blocks_per_tile(self.desc, p)
            out.append(sp)
        return out

    def arrays(self, f, p):
        """Copies of frame f, plane p's arrays (host numpy), for checks."""
        sp = self.frame(f)[p]
        c = sp.c()
        n = sp.n_records

        def view(ptr, ctype, count, dtype):
            if count == 0:
                return np.zeros(0, dtype)
            return np.ctypeslib.as_array(ctypes.cast(ptr, ctypes.POINTER(ctype)), shape=(count,)).copy()
        return {"block_end": view(c.block_end, ctypes.c_uint32, sp.block_end_count, np.uint32),
                "index": view(c.index, ctypes.c_uint16, n, np.uint16),
                "values": view(c.values, ctypes.c_uint8, n, np.uint8),
                "bounds": np.array(list(c.bounds), np.float32)}
