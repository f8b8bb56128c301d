"""ctypes binding of librad's time stepper (the C-ABI in include/rad_timestep.h).

Argument marshalling only: the flux products, the absorbed-flux update and
the Crank-Nicolson column steps of Algorithm 6 run in librad's HIP kernels.
Tensors use the caller's facet order by default: a block of R scenarios is
an (R, N) contiguous tensor (column-major N x R with ld = N), the column
temperatures (M + 1, R, N), a run of direct-insolation levels (n_steps, R, N).
With order="tree_rmajor" they use the library's internal layout instead
(rows in tree order, scenarios contiguous, ld = ldr_of(R)): blocks (N, ldr),
temperatures (M + 1, N, ldr), levels (n_steps, N, ldr), as rad_insolation
writes them with the same order.
"""
from __future__ import annotations

import ctypes

import numpy as np

from .rad import _check, _stream_handle, _torch, ldr_of, load

_ORDERS = {"original": 0, "tree_rmajor": 2}

RAD_TS_T, RAD_TS_QABS, RAD_TS_QREFL, RAD_TS_QIR, RAD_TS_QRAD = range(5)
_FIELDS = {"T": RAD_TS_T, "Q_abs": RAD_TS_QABS, "Q_refl": RAD_TS_QREFL, "Q_ir": RAD_TS_QIR, "Q_rad": RAD_TS_QRAD}


class TsParams(ctypes.Structure):
    _fields_ = [("n_layers", ctypes.c_int32), ("z", ctypes.c_void_p), ("conductivity", ctypes.c_double),
                ("heat_capacity", ctypes.c_double), ("dt", ctypes.c_double), ("albedo", ctypes.c_double),
                ("emissivity", ctypes.c_double), ("bottom_flux", ctypes.c_double), ("surface", ctypes.c_int32),
                ("newton", ctypes.c_int32)]

SURFACE = {"half_layer": 0, "balanced": 1}


_bound = False


def _lib():
    global _bound
    L = load()
    if not _bound:
        vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.rad_ts_create.argtypes = [vp, ctypes.POINTER(TsParams), i64, ctypes.POINTER(vp)]
        L.rad_ts_init.argtypes = [vp, vp, i64, vp, i64, dbl, i32, vp]
        L.rad_ts_step.argtypes = [vp, i64, vp, i64, i64, i32, vp]
        L.rad_ts_read.argtypes = [vp, i32, vp, i64, i32, vp]
        for name in ("rad_ts_create", "rad_ts_init", "rad_ts_step", "rad_ts_read"):
            getattr(L, name).restype = ctypes.c_int
        L.rad_ts_time_column.argtypes = [vp, i32, vp, ctypes.POINTER(dbl)]
        L.rad_ts_time_column.restype = ctypes.c_int
        L.rad_ts_level.argtypes = [vp]
        L.rad_ts_level.restype = i64
        L.rad_ts_free.argtypes = [vp]
        L.rad_ts_free.restype = None
        _bound = True
    return L


def _block(t, shape, dtype, name):
    if tuple(t.shape) != tuple(shape) or t.dtype != dtype or not t.is_contiguous() or not t.is_cuda:
        raise ValueError(f"{name} must be a contiguous {dtype} device tensor of shape {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


class TimeStepper:
    """R scenarios of Algorithm 6 on the facets of an HMatrix (needs max_rhs >= 2 R)."""

    def __init__(self, H, z, conductivity, heat_capacity, dt, albedo, emissivity, bottom_flux=0.0, R=1,
                 surface="half_layer", newton=3):
        self.H = H
        self._z = np.ascontiguousarray(z, dtype=np.float64)
        self.M = len(self._z) - 1
        self.R = int(R)
        self.N = H.N
        p = TsParams(self.M, self._z.ctypes.data, float(conductivity), float(heat_capacity), float(dt),
                     float(albedo), float(emissivity), float(bottom_flux), SURFACE[surface], int(newton))
        h = ctypes.c_void_p()
        _check(_lib().rad_ts_create(H._h, ctypes.byref(p), self.R, ctypes.byref(h)))
        self._h = h

    def _flux_dtype(self):
        return self.H.torch_dtype

    def _layout(self, order):
        """(C-ABI order, block shape, leading dimension) of one N x R block."""
        if order not in _ORDERS:
            raise ValueError(f"order must be one of {sorted(_ORDERS)}")
        if order == "tree_rmajor":
            ld = ldr_of(self.R)
            return _ORDERS[order], (self.N, ld), ld
        return _ORDERS[order], (self.R, self.N), self.N

    def init(self, T0, Qdir0, H0=0.0, order="original"):
        torch = _torch()
        o, blk, ld = self._layout(order)
        pt = _block(T0, (self.M + 1,) + blk, torch.float64, "T0")
        pq = _block(Qdir0, blk, self._flux_dtype(), "Qdir0")
        _check(_lib().rad_ts_init(self._h, pt, ld, pq, ld, float(H0), o, _stream_handle()))

    def step(self, Qdir, order="original"):
        """Advance len(Qdir) levels; Qdir is (n_steps,) + one block, in the matrix precision."""
        o, blk, ld = self._layout(order)
        n = int(Qdir.shape[0])
        pq = _block(Qdir, (n,) + blk, self._flux_dtype(), "Qdir")
        _check(_lib().rad_ts_step(self._h, n, pq, ld, blk[0] * blk[1], o, _stream_handle()))

    def read(self, field, order="original"):
        """FP64 copy of one field: M + 1 blocks for "T", else one block."""
        torch = _torch()
        o, blk, ld = self._layout(order)
        shape = (self.M + 1,) + blk if field == "T" else blk
        out = torch.empty(shape, dtype=torch.float64, device=f"cuda:{self.H.device}")
        _check(_lib().rad_ts_read(self._h, _FIELDS[field], ctypes.c_void_p(out.data_ptr()), ld, o,
                                  _stream_handle()))
        return out

    def time_column(self, nrep=20):
        """Average ms per launch of the column kernel alone (diagnostic; the
        state is overwritten: call init again afterwards)."""
        ms = ctypes.c_double()
        _check(_lib().rad_ts_time_column(self._h, int(nrep), _stream_handle(), ctypes.byref(ms)))
        return ms.value

    @property
    def level(self):
        return int(_lib().rad_ts_level(self._h))

    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib().rad_ts_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
