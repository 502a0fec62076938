"""ctypes binding of the warm-start network (C ABI in include/lc_nn.h).

Argument marshalling only; the network runs in the library's HIP kernels
(BF16 matrix-core convolutions).  Raises if the library or the GPU is absent.
"""
import ctypes
import os

import numpy as np

from . import lc

EXPORTS = ["lc_nn_create", "lc_nn_destroy", "lc_nn_last_error", "lc_nn_set_layer", "lc_nn_get_layer",
           "lc_nn_save", "lc_nn_load",
           "lc_nn_features", "lc_nn_predict", "lc_nn_warm_start", "lc_nn_train_step", "lc_nn_layer_forward",
           "lc_nn_layer_backward", "lc_nn_time"]
CIN = (12, 32, 32, 32)
COUT = (32, 32, 32, 5)


class Case(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_double * 3), ("a0", ctypes.c_double), ("pitch", ctypes.c_double),
                ("anchoring", ctypes.c_int), ("pad_", ctypes.c_int), ("q_amp", ctypes.c_double),
                ("q_eq", ctypes.c_double)]


def make_case(pos, a0, pitch, anchoring="normal", q_amp=0.495, q_eq=0.5):
    c = Case()
    for k in range(3):
        c.pos[k] = pos[k]
    c.a0, c.pitch = a0, pitch
    c.anchoring = lc.ANCHORING.get(anchoring, anchoring)
    c.q_amp, c.q_eq = q_amp, q_eq
    return c


_bound = False


def _lib():
    global _bound
    L = lc.load()
    if not _bound:
        vp, fp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double)
        cp = ctypes.POINTER(Case)
        L.lc_nn_create.argtypes = [ctypes.c_int, ctypes.c_ulonglong, vp, ctypes.POINTER(vp)]
        L.lc_nn_destroy.argtypes = [vp]
        L.lc_nn_destroy.restype = None
        L.lc_nn_last_error.argtypes = [vp]
        L.lc_nn_last_error.restype = ctypes.c_char_p
        L.lc_nn_set_layer.argtypes = [vp, ctypes.c_int, fp, fp]
        L.lc_nn_get_layer.argtypes = [vp, ctypes.c_int, fp, fp]
        L.lc_nn_save.argtypes = [vp, ctypes.c_char_p]
        L.lc_nn_load.argtypes = [vp, ctypes.c_char_p]
        L.lc_nn_features.argtypes = [vp, cp, fp]
        L.lc_nn_predict.argtypes = [vp, cp, dp]
        L.lc_nn_warm_start.argtypes = [vp, cp, vp, ctypes.c_int]
        L.lc_nn_train_step.argtypes = [vp, cp, dp, ctypes.POINTER(ctypes.c_ubyte), ctypes.c_float, dp]
        L.lc_nn_layer_forward.argtypes = [vp, ctypes.c_int, fp, fp]
        L.lc_nn_layer_backward.argtypes = [vp, ctypes.c_int, fp, fp, fp, fp, fp]
        L.lc_nn_time.argtypes = [vp, cp, dp, ctypes.POINTER(ctypes.c_ubyte), ctypes.c_int, dp]
        _bound = True
    return L


def _f(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _u8(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))


class Net:
    """Warm-start network for an L^3 grid on cuda:0."""

    def __init__(self, L, seed=0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the HIP library has no CPU path")
        self._L = _lib()
        self.L = L
        self.shape = (L, L, L)
        self.stream = stream if stream is not None else torch.cuda.Stream()
        h = ctypes.c_void_p()
        rc = self._L.lc_nn_create(L, seed, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc != 0:
            raise lc.LCError(rc, self._L.lc_nn_last_error(None).decode())
        self._h = h

    def _chk(self, rc):
        if rc != 0:
            raise lc.LCError(rc, self._L.lc_nn_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._L.lc_nn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_layer(self, l, W, b):
        W = np.ascontiguousarray(W, dtype=np.float32).reshape(COUT[l], CIN[l], 27)
        b = np.ascontiguousarray(b, dtype=np.float32).reshape(COUT[l])
        self._chk(self._L.lc_nn_set_layer(self._h, l, _f(W), _f(b)))

    def get_layer(self, l):
        W = np.zeros((COUT[l], CIN[l], 27), np.float32)
        b = np.zeros(COUT[l], np.float32)
        self._chk(self._L.lc_nn_get_layer(self._h, l, _f(W), _f(b)))
        return W, b

    def save(self, path):
        self._chk(self._L.lc_nn_save(self._h, os.fsencode(path)))

    def load(self, path):
        self._chk(self._L.lc_nn_load(self._h, os.fsencode(path)))

    def features(self, case):
        out = np.zeros((12,) + self.shape, np.float32)
        self._chk(self._L.lc_nn_features(self._h, ctypes.byref(case), _f(out)))
        return out

    def predict(self, case):
        out = np.zeros((5,) + self.shape)
        self._chk(self._L.lc_nn_predict(self._h, ctypes.byref(case), _d(out)))
        return out

    def warm_start(self, case, ctx, box=0):
        self._chk(self._L.lc_nn_warm_start(self._h, ctypes.byref(case), ctx._h, box))

    def train_step(self, case, Q_target, fluid, lr):
        q = np.ascontiguousarray(Q_target, dtype=np.float64)
        m = np.ascontiguousarray(fluid, dtype=np.uint8)
        loss = ctypes.c_double()
        self._chk(self._L.lc_nn_train_step(self._h, ctypes.byref(case), _d(q), _u8(m), lr, ctypes.byref(loss)))
        return loss.value

    def layer_forward(self, l, x):
        x = np.ascontiguousarray(x, dtype=np.float32)
        z = np.zeros((COUT[l],) + self.shape, np.float32)
        self._chk(self._L.lc_nn_layer_forward(self._h, l, _f(x), _f(z)))
        return z

    def layer_backward(self, l, x, dz):
        x = np.ascontiguousarray(x, dtype=np.float32)
        dz = np.ascontiguousarray(dz, dtype=np.float32)
        dW = np.zeros((COUT[l], CIN[l], 27), np.float32)
        db = np.zeros(COUT[l], np.float32)
        dx = np.zeros((CIN[l],) + self.shape, np.float32)
        self._chk(self._L.lc_nn_layer_backward(self._h, l, _f(x), _f(dz), _f(dW), _f(db), _f(dx)))
        return dW, db, dx

    def time(self, case, Q_target, fluid, n=10):
        q = np.ascontiguousarray(Q_target, dtype=np.float64)
        m = np.ascontiguousarray(fluid, dtype=np.uint8)
        out = np.zeros(2)
        self._chk(self._L.lc_nn_time(self._h, ctypes.byref(case), _d(q), _u8(m), n, _d(out)))
        return {"forward_ms": out[0], "train_step_ms": out[1]}
