"""ctypes binding of librad's warm start (the C-ABI in include/rad_warmstart.h).

Argument marshalling only: POD, perceptron training and inference run in
librad's HIP kernels.  Facet-indexed tensors are facet-major (N x R,
row-major), the layout of order="tree_rmajor".
"""
from __future__ import annotations

import ctypes

import numpy as np

from .rad import RAD_BF16, RAD_F32, _check, _stream_handle, _torch, load


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _rows(t, name):
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be a 2-D facet-major tensor with unit column stride")
    return t.stride(0)


def sun_features(suns, e_lo=5.0, e_hi=30.0) -> np.ndarray:
    """(cos az, sin az, elevation mapped to [-1, 1]) per unit sun vector (FP32)."""
    s = np.asarray(suns, dtype=np.float64)
    az = np.arctan2(s[:, 1], s[:, 0])
    el = np.rad2deg(np.arcsin(np.clip(s[:, 2], -1.0, 1.0)))
    return np.column_stack([np.cos(az), np.sin(az), 2.0 * (el - e_lo) / (e_hi - e_lo) - 1.0]).astype(np.float32)


def pod_build(S, m, R=None):
    """POD modes of the first R columns of the facet-major FP32 snapshot block S.
    Returns (Phi: N x m FP32 tensor, sigma: numpy FP64)."""
    torch = _torch()
    lds = _rows(S, "S")
    N = S.shape[0]
    M = int(R if R is not None else S.shape[1])
    Phi = torch.empty((N, m), dtype=torch.float32, device=S.device)
    sigma = np.zeros(m)
    _check(load().rad_pod_build(_p(S), N, M, lds, int(m), _p(Phi), m, sigma.ctypes.data, S.device.index or 0,
                                _stream_handle()))
    return Phi, sigma


def pod_project(Phi, B, E=None, scale=None, R=None):
    """C (R x m) with C[c, j] = scale_j sum_t Phi[t, j] (B - E)[t, c]."""
    torch = _torch()
    ldb = _rows(B, "B")
    if E is not None and _rows(E, "E") != ldb:
        raise ValueError("B and E must share the leading dimension")
    R = int(R if R is not None else B.shape[1])
    N, m = Phi.shape
    C = torch.empty((R, m), dtype=torch.float32, device=B.device)
    _check(load().rad_pod_project(_p(Phi), N, m, _rows(Phi, "Phi"), _p(B), _p(E), R, ldb, _p(scale), _p(C),
                                  _stream_handle()))
    return C


def pod_expand(Phi, C, scale=None, E=None, out=None, R=None):
    """B[t, c] = E[t, c] + sum_j Phi[t, j] scale_j C[c, j] (facet-major, R columns)."""
    torch = _torch()
    N, m = Phi.shape
    R = int(R if R is not None else C.shape[0])
    if out is None:
        out = torch.empty((N, R), dtype=torch.float32, device=Phi.device)
    ldb = _rows(out, "out")
    if E is not None and _rows(E, "E") != ldb:
        raise ValueError("out and E must share the leading dimension")
    _check(load().rad_pod_expand(_p(Phi), N, m, _rows(Phi, "Phi"), _p(C.contiguous()), _p(scale), _p(E), R, ldb,
                                 _p(out), _stream_handle()))
    return out


class MLP:
    """tanh perceptron trained and evaluated by librad's kernels."""

    def __init__(self, sizes, params, compute="f32", max_batch=4096, device=0):
        L = load()
        sz = np.ascontiguousarray(sizes, dtype=np.int32)
        p = np.ascontiguousarray(params, dtype=np.float32)
        h = ctypes.c_void_p()
        cmp = {"f32": RAD_F32, "bf16": RAD_BF16}[compute]
        _check(L.rad_mlp_create(sz.ctypes.data, len(sz), p.ctypes.data, cmp, int(max_batch), int(device),
                                ctypes.byref(h)))
        self._h = h
        self.sizes = [int(x) for x in sizes]
        self.P = int(L.rad_mlp_param_count(h))
        if self.P != p.size:
            self.close()
            raise ValueError(f"parameter vector has {p.size} entries, the network needs {self.P}")

    def params(self) -> np.ndarray:
        out = np.empty(self.P, dtype=np.float32)
        _check(load().rad_mlp_get_params(self._h, out.ctypes.data))
        return out

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        _check(load().rad_mlp_set_params(self._h, p.ctypes.data))

    def forward(self, X, out=None):
        torch = _torch()
        X = X.contiguous()
        if out is None:
            out = torch.empty((X.shape[0], self.sizes[-1]), dtype=torch.float32, device=X.device)
        _check(load().rad_mlp_forward(self._h, _p(X), X.shape[0], _p(out), _stream_handle()))
        return out

    def loss_grad(self, X, T, w):
        loss = ctypes.c_double()
        g = np.empty(self.P, dtype=np.float32)
        _check(load().rad_mlp_loss_grad(self._h, _p(X.contiguous()), _p(T.contiguous()), _p(w.contiguous()),
                                        X.shape[0], ctypes.byref(loss), g.ctypes.data, _stream_handle()))
        return loss.value, g

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        _check(load().rad_mlp_adam_step(self._h, lr, beta1, beta2, eps, _stream_handle()))

    def train(self, X, T, w, steps, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        hist = np.zeros(int(steps))
        _check(load().rad_mlp_train(self._h, _p(X.contiguous()), _p(T.contiguous()), _p(w.contiguous()), X.shape[0],
                                    int(steps), lr, beta1, beta2, eps, hist.ctypes.data, _stream_handle()))
        return hist

    def close(self):
        if getattr(self, "_h", None):
            load().rad_mlp_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
