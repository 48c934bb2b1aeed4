"""ctypes binding of the restoration network (include/wv_cnn.h): argument
marshalling only; every step runs in libwv's kernels."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import wv as _wv

_lib = _wv.lib()
_vp, _i32, _i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
for _name, _res, _args in [
    ("wv_cnn_param_count", _i32, []),
    ("wv_cnn_create", _i32, [ctypes.POINTER(_vp), _i64]),
    ("wv_cnn_destroy", _i32, [_vp]),
    ("wv_cnn_set_params", _i32, [_vp, _vp, _vp]),
    ("wv_cnn_get_params", _i32, [_vp, _vp, _vp]),
    ("wv_cnn_forward", _i32, [_vp, _vp, _i32, _i32, _i32, _vp, _vp]),
    ("wv_cnn_infer", _i32, [_vp, _vp, _i32, _i32, _i32, _vp, _vp]),
    ("wv_cnn_loss_grad", _i32, [_vp, _vp, _vp, _vp]),
    ("wv_cnn_backward", _i32, [_vp, _vp, _vp]),
    ("wv_cnn_adam", _i32, [_vp, ctypes.c_float, _i32, _vp]),
    ("wv_cnn_train_step", _i32, [_vp, _vp, _vp, _i32, _i32, _i32, ctypes.c_float, _i32, _vp, _vp]),
    ("wv_cnn_gather", _i32, [_vp, _vp, _i32, _i32, _i32, _i32, _vp, _i32, _i32, _i32, _vp, _vp]),
    ("wv_cnn_restore", _i32, [_vp, _vp, _i32, _i32, _i32, ctypes.c_float, _vp,
                              ctypes.POINTER(_i32), _vp]),
]:
    _fn = getattr(_lib, _name)
    _fn.restype, _fn.argtypes = _res, _args

EXPORTED = ("wv_cnn_param_count", "wv_cnn_create", "wv_cnn_destroy", "wv_cnn_set_params",
            "wv_cnn_get_params", "wv_cnn_forward", "wv_cnn_infer", "wv_cnn_loss_grad", "wv_cnn_backward",
            "wv_cnn_adam", "wv_cnn_train_step", "wv_cnn_gather", "wv_cnn_restore")

HIDDEN = 32
LAYERS = [(3, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, 3)]


def param_count():
    return _lib.wv_cnn_param_count()


def flatten(params):
    """[W1, b1, ..., W4, b4] (W [out][3][3][in]) -> the library's fp32 vector."""
    return np.concatenate([np.asarray(p, np.float32).ravel() for p in params])


def unflatten(vec):
    out, off = [], 0
    for ci, co in LAYERS:
        n = co * 9 * ci
        out.append(np.asarray(vec[off:off + n], np.float64).reshape(co, 3, 3, ci))
        off += n
        out.append(np.asarray(vec[off:off + co], np.float64))
        off += co
    return out


def _check_dev(t, dtype, numel, what):
    if (not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != dtype
            or not t.is_contiguous() or t.numel() < numel):
        raise ValueError(f"{what}: need a contiguous {dtype} CUDA tensor with >= {numel} elements")


class Net:
    """The restoration network with its device state."""

    def __init__(self, max_pixels):
        h = ctypes.c_void_p()
        _wv._check(_lib.wv_cnn_create(ctypes.byref(h), int(max_pixels)))
        self._h = h
        self.max_pixels = int(max_pixels)
        self.loss_dev = torch.zeros(1, dtype=torch.float32, device="cuda")

    def close(self):
        if getattr(self, "_h", None):
            _lib.wv_cnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, vec, stream=None):
        vec = np.ascontiguousarray(vec, dtype=np.float32)
        if vec.size != param_count():
            raise ValueError("parameter vector has the wrong length")
        _wv._check(_lib.wv_cnn_set_params(self._h, vec.ctypes.data_as(_vp), _wv._stream(stream)))

    def get_params(self, stream=None):
        vec = np.zeros(param_count(), np.float32)
        _wv._check(_lib.wv_cnn_get_params(self._h, vec.ctypes.data_as(_vp), _wv._stream(stream)))
        return vec

    def forward(self, x, z=None, stream=None):
        n, h, w, c = x.shape
        if c != 4:
            raise ValueError("x must be NHWC with 4 channels")
        _check_dev(x, torch.bfloat16, n * h * w * 4, "x")
        if z is not None:
            _check_dev(z, torch.float32, n * h * w * 4, "z")
        _wv._check(_lib.wv_cnn_forward(self._h, _wv._ptr(x), n, h, w, _wv._ptr(z), _wv._stream(stream)))
        # the library reads x (and keeps z) in place until the backward pass
        self._x, self._z = x, z

    def infer(self, x, z, stream=None):
        """The forward pass without keeping activations (no backward may follow)."""
        n, h, w, c = x.shape
        if c != 4:
            raise ValueError("x must be NHWC with 4 channels")
        _check_dev(x, torch.bfloat16, n * h * w * 4, "x")
        _check_dev(z, torch.float32, n * h * w * 4, "z")
        _wv._check(_lib.wv_cnn_infer(self._h, _wv._ptr(x), n, h, w, _wv._ptr(z), _wv._stream(stream)))
        self._x, self._z = None, None

    def loss_grad(self, t, stream=None):
        _check_dev(t, torch.float32, 4, "t")
        _wv._check(_lib.wv_cnn_loss_grad(self._h, _wv._ptr(t), _wv._ptr(self.loss_dev), _wv._stream(stream)))
        return self.loss_dev

    def backward(self, grads=None, stream=None):
        if grads is not None:
            _check_dev(grads, torch.float32, param_count(), "grads")
        _wv._check(_lib.wv_cnn_backward(self._h, _wv._ptr(grads), _wv._stream(stream)))

    def adam(self, lr, step, stream=None):
        _wv._check(_lib.wv_cnn_adam(self._h, float(lr), int(step), _wv._stream(stream)))

    def train_step(self, x, t, lr, step, stream=None):
        n, h, w, _ = x.shape
        _check_dev(x, torch.bfloat16, n * h * w * 4, "x")
        _check_dev(t, torch.float32, n * h * w * 4, "t")
        _wv._check(_lib.wv_cnn_train_step(self._h, _wv._ptr(x), _wv._ptr(t), n, h, w, float(lr),
                                          int(step), _wv._ptr(self.loss_dev), _wv._stream(stream)))
        return self.loss_dev

    def gather(self, images, tile, tiles_x, tiles_y, crops, size, as_float, stream=None):
        """Crops (HOST int [k][3]: image, y0, x0) of tile-planar uint8 viewports."""
        crops = np.ascontiguousarray(crops, dtype=np.int32).reshape(-1, 3)
        n_img = images.shape[0]
        out = torch.empty((len(crops), size, size, 4),
                          dtype=torch.float32 if as_float else torch.bfloat16, device="cuda")
        _check_dev(images, torch.uint8, n_img * tiles_x * tiles_y * 3 * tile * tile, "images")
        _wv._check(_lib.wv_cnn_gather(self._h, _wv._ptr(images), tile, tiles_x, tiles_y, n_img,
                                      crops.ctypes.data_as(_vp), len(crops), size, int(as_float),
                                      _wv._ptr(out), _wv._stream(stream)))
        return out

    def restore(self, decoded, tile, tiles_x, tiles_y, guard, out=None, stream=None):
        """Restored viewport (same layout as `decoded`) and the fallback tile count."""
        _check_dev(decoded, torch.uint8, tiles_x * tiles_y * 3 * tile * tile, "decoded")
        if out is None:
            out = torch.empty_like(decoded)
        fell = ctypes.c_int32()
        _wv._check(_lib.wv_cnn_restore(self._h, _wv._ptr(decoded), tile, tiles_x, tiles_y,
                                       float(guard), _wv._ptr(out), ctypes.byref(fell),
                                       _wv._stream(stream)))
        return out, fell.value
