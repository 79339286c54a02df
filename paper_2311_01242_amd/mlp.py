"""Warm-start MLP binding (argument marshalling over libvqe.so's vqe_mlp_*)
and the feature map of a bond-stretch geometry.

Features: x = [lambda, upper triangle of h(lambda) (row-major, diagonal
included)], standardised with the training set's mean and standard
deviation.  Targets: converged UCCSD amplitudes theta*.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _check, lib


def _fptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def features(lam, h):
    iu = np.triu_indices(h.shape[0])
    return np.concatenate([[lam], h[iu]])


class MLP:
    def __init__(self, widths):
        self.widths = [int(w) for w in widths]
        w = (C.c_int32 * len(self.widths))(*self.widths)
        out = C.c_void_p()
        _check(lib().vqe_mlp_create(len(self.widths) - 1, w, None, C.byref(out)))
        self._h = out
        n = C.c_int64()
        _check(lib().vqe_mlp_n_params(self._h, C.byref(n)))
        self.n_params = n.value

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.n_params
        _check(lib().vqe_mlp_set_params(self._h, _fptr(p)))

    def get_params(self):
        p = np.empty(self.n_params, np.float32)
        _check(lib().vqe_mlp_get_params(self._h, _fptr(p)))
        return p

    def forward(self, x):
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.empty((x.shape[0], self.widths[-1]), np.float32)
        _check(lib().vqe_mlp_forward(self._h, x.shape[0], _fptr(x), _fptr(y)))
        return y

    def loss_grad(self, x, y):
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        loss = np.empty(1, np.float32)
        g = np.empty(self.n_params, np.float32)
        _check(lib().vqe_mlp_loss_grad(self._h, x.shape[0], _fptr(x), _fptr(y), _fptr(loss), _fptr(g)))
        return float(loss[0]), g

    def train(self, x, y, steps, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        tr = np.empty(max(int(steps), 1), np.float32)
        _check(lib().vqe_mlp_train(self._h, x.shape[0], _fptr(x), _fptr(y), int(steps), float(lr),
                                   float(beta1), float(beta2), float(eps), _fptr(tr)))
        return tr[:steps]

    def close(self):
        if self._h:
            lib().vqe_mlp_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
