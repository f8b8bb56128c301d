"""CPU-side checks of the C-ABI library: it loads, exports every symbol that
include/*.h declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    inc = os.path.join(ROOT, "include")
    text = "".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc)) if f.endswith(".h"))
    return sorted(set(re.findall(r"\b(rad_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_core_entry_points():
    syms = _declared_symbols()
    for name in ["rad_hmat_build", "rad_hmat_matvec", "rad_solve", "rad_hmat_free", "rad_last_error"]:
        assert name in syms


def test_library_exports_every_declared_symbol():
    from paper_2209_07632_amd import rad
    L = rad.load()
    for name in _declared_symbols():
        assert hasattr(L, name), name
    assert set(rad.EXPORTS) <= set(_declared_symbols())


def test_build_rejects_bad_arguments():
    from paper_2209_07632_amd import rad
    L = rad.load()
    o = rad.BuildOpts()
    L.rad_build_opts_default(ctypes.byref(o))
    assert abs(o.tol - 1e-3) < 1e-15 and o.leaf_size == 64
    h = ctypes.c_void_p()
    verts = np.zeros((3, 3))
    faces = np.array([[0, 1, 5]], dtype=np.int32)
    # null mesh
    st = L.rad_hmat_build(None, 3, None, 1, ctypes.byref(o), ctypes.byref(h))
    assert st == rad.RAD_EINVAL and not h.value
    # bad tolerance
    o.tol = -1.0
    st = L.rad_hmat_build(verts.ctypes.data, 3, faces.ctypes.data, 1, ctypes.byref(o), ctypes.byref(h))
    assert st == rad.RAD_EINVAL and b"tol" in L.rad_last_error()
    o.tol = 1e-3
    # vertex index out of range
    st = L.rad_hmat_build(verts.ctypes.data, 3, faces.ctypes.data, 1, ctypes.byref(o), ctypes.byref(h))
    assert st == rad.RAD_EINVAL and b"outside" in L.rad_last_error()
    # zero-area face
    faces2 = np.array([[0, 1, 2]], dtype=np.int32)
    st = L.rad_hmat_build(verts.ctypes.data, 3, faces2.ctypes.data, 1, ctypes.byref(o), ctypes.byref(h))
    assert st == rad.RAD_EINVAL and b"zero area" in L.rad_last_error()
    # non-finite coordinate
    v3 = np.array([[0, 0, 0], [1, 0, 0], [0, np.nan, 0]], dtype=np.float64)
    st = L.rad_hmat_build(v3.ctypes.data, 3, faces2.ctypes.data, 1, ctypes.byref(o), ctypes.byref(h))
    assert st == rad.RAD_EINVAL and b"non-finite" in L.rad_last_error()


def test_calls_on_null_handle_fail_cleanly():
    from paper_2209_07632_amd import rad
    L = rad.load()
    st = L.rad_hmat_matvec(None, 1, 0, None, 1, None, 1, 0, None)
    assert st == rad.RAD_EINVAL
    s = rad.Stats()
    assert L.rad_hmat_info(None, ctypes.byref(s)) == rad.RAD_EINVAL
    assert L.rad_hmat_n(None) == -1
    L.rad_hmat_free(None)


def test_time_stepper_rejects_null_arguments():
    from paper_2209_07632_amd import rad
    from paper_2209_07632_amd.timestep import TsParams, _lib
    L = _lib()
    h = ctypes.c_void_p()
    z = np.array([0.0, 0.1])
    p = TsParams(1, z.ctypes.data, 0.01, 1e6, 100.0, 0.1, 0.9, 0.0)
    assert L.rad_ts_create(None, ctypes.byref(p), 1, ctypes.byref(h)) == rad.RAD_EINVAL and not h.value
    assert L.rad_ts_step(None, 1, None, 1, 1, 0, None) == rad.RAD_EINVAL
    assert L.rad_ts_init(None, None, 1, None, 1, 0.0, 0, None) == rad.RAD_EINVAL
    assert L.rad_ts_read(None, 0, None, 1, 0, None) == rad.RAD_EINVAL
    assert L.rad_ts_level(None) == -1
    L.rad_ts_free(None)


def test_build_tree_rejects_bad_tree_dims():
    from paper_2209_07632_amd import rad
    L = rad.load()
    o = rad.BuildOpts()
    L.rad_build_opts_default(ctypes.byref(o))
    h = ctypes.c_void_p()
    verts = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], dtype=np.float64)
    faces = np.array([[0, 1, 2]], dtype=np.int32)
    st = L.rad_hmat_build_tree(verts.ctypes.data, 3, faces.ctypes.data, 1, ctypes.byref(o), 4, ctypes.byref(h))
    assert st == rad.RAD_EINVAL and b"tree_dims" in L.rad_last_error() and not h.value
