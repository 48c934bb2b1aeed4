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
]:
    _fn = getattr(_lib, _name)
    _fn.restype, _fn.argtypes = _res, _args

EXPORTED = ("wv_sparse_blocks_per_tile", "wv_sparse_encode_plane", "wv_sparse_rebuild")


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
