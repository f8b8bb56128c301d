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


def test_build_facets_rejects_bad_geometry():
    from paper_2209_07632_amd import rad
    L = rad.load()
    o = rad.BuildOpts()
    L.rad_build_opts_default(ctypes.byref(o))
    assert not o.allocator
    h = ctypes.c_void_p()
    x = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    n = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, 1.0]])
    a = np.array([1.0, 1.0])
    st = L.rad_hmat_build_facets(None, n.ctypes.data, a.ctypes.data, 2, None, ctypes.byref(o), 2, ctypes.byref(h))
    assert st == rad.RAD_EINVAL and not h.value
    n2 = n.copy()
    n2[1, 2] = 0.5   # not a unit normal
    st = L.rad_hmat_build_facets(x.ctypes.data, n2.ctypes.data, a.ctypes.data, 2, None, ctypes.byref(o), 2,
                                 ctypes.byref(h))
    assert st == rad.RAD_EINVAL and b"unit" in L.rad_last_error() and not h.value
    a2 = np.array([1.0, 0.0])
    st = L.rad_hmat_build_facets(x.ctypes.data, n.ctypes.data, a2.ctypes.data, 2, None, ctypes.byref(o), 2,
                                 ctypes.byref(h))
    assert st == rad.RAD_EINVAL and b"area" in L.rad_last_error()
    o.visibility = 1   # ray casting needs the triangles
    st = L.rad_hmat_build_facets(x.ctypes.data, n.ctypes.data, a.ctypes.data, 2, None, ctypes.byref(o), 2,
                                 ctypes.byref(h))
    assert st == rad.RAD_EINVAL and b"tri_verts" in L.rad_last_error()


def test_files_reject_bad_input(tmp_path):
    from paper_2209_07632_amd import rad
    L = rad.load()
    h = ctypes.c_void_p()
    assert L.rad_hmat_export(None, b"x") == rad.RAD_EINVAL
    assert L.rad_hmat_save(None, b"x") == rad.RAD_EINVAL
    missing = str(tmp_path / "missing.bin").encode()
    assert L.rad_hmat_load(missing, 0, 0, None, ctypes.byref(h)) == rad.RAD_EDEVICE and not h.value
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"NOTAHMAT" + bytes(64))
    st = L.rad_hmat_load(str(bad).encode(), 0, 0, None, ctypes.byref(h))
    assert st == rad.RAD_EINVAL and b"not a saved" in L.rad_last_error() and not h.value
    assert L.rad_hmat_lowp(None) == -1 and L.rad_hmat_max_rhs(None) == -1


def test_block_export_reader(tmp_path):
    """The test-side reader of rad_hmat_export files on a hand-made file: one
    dense, one CSR and one rank-one block of a 4-facet matrix."""
    import struct
    from hmat_blocks import densify, read_export
    perm = np.array([2, 0, 3, 1], dtype=np.int32)
    out = [b"RADHBLKS", struct.pack("<Ii", 1, 0), struct.pack("<qq", 4, 3), perm.tobytes()]
    A = np.array([[0.0, 1.0], [2.0, 0.0]])
    out += [struct.pack("<6iq", 1, 0, 2, 0, 2, 0, 2), A.T.tobytes()]
    out += [struct.pack("<6iq", 2, 2, 2, 2, 2, 0, 2), np.array([0, 1, 2], np.int32).tobytes(),
            np.array([1, 0], np.int32).tobytes(), np.array([5.0, 7.0]).tobytes()]
    U, V = np.array([[1.0], [2.0]]), np.array([[3.0], [4.0]])
    out += [struct.pack("<6iq", 3, 0, 2, 2, 2, 1, 4), U.T.tobytes(), V.T.tobytes()]
    path = tmp_path / "b.bin"
    path.write_bytes(b"".join(out))
    ex = read_export(path)
    Ft = densify(ex, original_order=False)
    expect = np.array([[0, 1, 3, 4], [2, 0, 6, 8], [0, 0, 0, 5], [0, 0, 7, 0]], dtype=float)
    np.testing.assert_array_equal(Ft, expect)
    F = densify(ex)
    np.testing.assert_array_equal(F[np.ix_(perm, perm)], expect)
