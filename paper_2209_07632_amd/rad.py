"""ctypes binding of librad (the C-ABI in include/rad.h).

Argument marshalling only: every step of the computation runs in librad's
HIP kernels.  Device tensors are torch CUDA tensors; the binding passes their
data pointers and the current torch stream.  There is no fallback: if
librad.so is missing or the device is not available, calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "librad.so")

RAD_OK, RAD_EINVAL, RAD_ENOMEM, RAD_EDEVICE, RAD_ENOCONV, RAD_EUNSUP = range(6)
RAD_F64, RAD_F32, RAD_F16, RAD_BF16 = range(4)
NEARFIELD = {"auto": 0, "dense": 1, "csr": 2}
VISIBILITY = {"backface": 0, "raycast": 1}
ORDER = {"original": 0, "tree": 1, "tree_rmajor": 2}
DTYPES = {"f64": RAD_F64, "f32": RAD_F32}


class RadError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"librad status {status}: {msg}")
        self.status = status


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32)


class Allocator(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN)]


class BuildOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("leaf_size", ctypes.c_int32), ("max_depth", ctypes.c_int32),
                ("nearfield", ctypes.c_int32), ("visibility", ctypes.c_int32), ("storage", ctypes.c_int32),
                ("oversample", ctypes.c_int32), ("power_iters", ctypes.c_int32), ("max_rhs", ctypes.c_int32),
                ("device", ctypes.c_int32), ("seed", ctypes.c_uint64), ("verbose", ctypes.c_int32),
                ("max_rank", ctypes.c_int32), ("lowp", ctypes.c_int32),
                ("allocator", ctypes.POINTER(Allocator))]


class TorchAllocator:
    """rad_allocator hook backed by torch's caching allocator, so that torch
    owns the device memory of the matrices built with it.  The object (and its
    callbacks) must outlive those matrices; HMatrix keeps a reference."""

    def __init__(self):
        import torch

        def _alloc(ctx, nbytes, device):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), int(device))
            except Exception:
                return None

        def _free(ctx, ptr, nbytes, device):
            torch.cuda.caching_allocator_delete(int(ptr))

        self._alloc_fn = ALLOC_FN(_alloc)
        self._free_fn = FREE_FN(_free)
        self.struct = Allocator(None, self._alloc_fn, self._free_fn)


class SolveOpts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("order", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("refine", ctypes.c_int32),
                ("inner_iters", ctypes.c_int32), ("warm", ctypes.c_int32), ("method", ctypes.c_int32),
                ("lam_lo", ctypes.c_double), ("lam_hi", ctypes.c_double), ("restart", ctypes.c_int32)]


METHODS = {"jacobi": 0, "chebyshev": 1, "gmres": 2}


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.POINTER(ctypes.c_int32)), ("rel_change", ctypes.POINTER(ctypes.c_double)),
                ("total_iters", ctypes.c_int32), ("inner_iters", ctypes.c_int32),
                ("warm_columns", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_leaves", ctypes.c_int64), ("depth", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("n_dense", ctypes.c_int64), ("n_csr", ctypes.c_int64),
                ("n_lowrank", ctypes.c_int64), ("n_zero", ctypes.c_int64), ("bytes_dense", ctypes.c_int64),
                ("bytes_csr", ctypes.c_int64), ("bytes_lowrank", ctypes.c_int64), ("bytes_total", ctypes.c_int64),
                ("nnz_near", ctypes.c_int64), ("sum_rank", ctypes.c_int64), ("lowrank_elems", ctypes.c_int64),
                ("max_rank", ctypes.c_int32), ("build_seconds", ctypes.c_double), ("flops_per_rhs", ctypes.c_double),
                ("lowrank_row_elems", ctypes.c_int64), ("lowrank_col_elems", ctypes.c_int64),
                ("max_panel_cols", ctypes.c_int64), ("bytes_csr_panels", ctypes.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


EXPORTS = ["rad_build_opts_default", "rad_hmat_build", "rad_hmat_build_tree", "rad_hmat_build_facets",
           "rad_hmat_export", "rad_hmat_save", "rad_hmat_load", "rad_hmat_convert", "rad_hmat_matvec",
           "rad_hmat_matvec_noalloc", "rad_noalloc_scratch_bytes", "rad_solve_opts_default", "rad_solve",
           "rad_insolation", "rad_equilibrium", "rad_hmat_time_phases", "rad_hmat_info", "rad_hmat_n", "rad_hmat_dtype", "rad_hmat_lowp",
           "rad_hmat_max_rhs", "rad_hmat_perm", "rad_hmat_free",
           "rad_last_error", "rad_pod_build", "rad_pod_project", "rad_pod_expand", "rad_mlp_create",
           "rad_mlp_param_count", "rad_mlp_get_params", "rad_mlp_set_params", "rad_mlp_forward", "rad_mlp_loss_grad",
           "rad_mlp_adam_step", "rad_mlp_train", "rad_mlp_free", "rad_hmat_group", "rad_hmat_instances",
           "rad_hmat_group_layout", "rad_hmat_autotune", "rad_hmat_set_config", "rad_hmat_get_config"]

_lib = None


def load(path: str = LIB_PATH):
    """Load librad.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2209_07632_amd.build_lib.build()")
    # torch's HIP runtime must be loaded before librad's dependency on it is
    # resolved, or torch later finds no device
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    L.rad_build_opts_default.argtypes = [ctypes.POINTER(BuildOpts)]
    L.rad_build_opts_default.restype = None
    L.rad_solve_opts_default.argtypes = [ctypes.POINTER(SolveOpts)]
    L.rad_solve_opts_default.restype = None
    L.rad_hmat_build.argtypes = [vp, ctypes.c_int64, vp, ctypes.c_int64, ctypes.POINTER(BuildOpts),
                                 ctypes.POINTER(vp)]
    L.rad_hmat_build.restype = ctypes.c_int
    L.rad_hmat_build_tree.argtypes = [vp, ctypes.c_int64, vp, ctypes.c_int64, ctypes.POINTER(BuildOpts),
                                      ctypes.c_int32, ctypes.POINTER(vp)]
    L.rad_hmat_build_tree.restype = ctypes.c_int
    L.rad_hmat_build_facets.argtypes = [vp, vp, vp, ctypes.c_int64, vp, ctypes.POINTER(BuildOpts), ctypes.c_int32,
                                        ctypes.POINTER(vp)]
    L.rad_hmat_build_facets.restype = ctypes.c_int
    L.rad_hmat_convert.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(vp)]
    L.rad_hmat_convert.restype = ctypes.c_int
    L.rad_hmat_export.argtypes = [vp, ctypes.c_char_p]
    L.rad_hmat_export.restype = ctypes.c_int
    L.rad_hmat_save.argtypes = [vp, ctypes.c_char_p]
    L.rad_hmat_save.restype = ctypes.c_int
    L.rad_hmat_load.argtypes = [ctypes.c_char_p, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Allocator),
                                ctypes.POINTER(vp)]
    L.rad_hmat_load.restype = ctypes.c_int
    L.rad_hmat_matvec.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, vp, ctypes.c_int64, vp, ctypes.c_int64,
                                  ctypes.c_int32, vp]
    L.rad_hmat_matvec.restype = ctypes.c_int
    L.rad_hmat_matvec_noalloc.argtypes = L.rad_hmat_matvec.argtypes
    L.rad_hmat_matvec_noalloc.restype = ctypes.c_int
    L.rad_noalloc_scratch_bytes.argtypes = []
    L.rad_noalloc_scratch_bytes.restype = ctypes.c_size_t
    L.rad_solve.argtypes = [vp, vp, ctypes.c_double, ctypes.c_int64, ctypes.c_int32, vp, ctypes.c_int64, vp,
                            ctypes.c_int64, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), vp]
    L.rad_solve.restype = ctypes.c_int
    L.rad_insolation.argtypes = [vp, ctypes.c_int64, vp, ctypes.c_double, ctypes.c_int32, vp, ctypes.c_int64,
                                 ctypes.c_int32, vp]
    L.rad_insolation.restype = ctypes.c_int
    L.rad_equilibrium.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, vp, ctypes.c_int64, ctypes.c_double,
                                  ctypes.c_double, vp, vp, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo),
                                  ctypes.POINTER(SolveInfo), vp]
    L.rad_equilibrium.restype = ctypes.c_int
    L.rad_hmat_time_phases.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, vp,
                                       ctypes.POINTER(ctypes.c_double)]
    L.rad_hmat_time_phases.restype = ctypes.c_int
    L.rad_hmat_info.argtypes = [vp, ctypes.POINTER(Stats)]
    L.rad_hmat_info.restype = ctypes.c_int
    L.rad_hmat_n.argtypes = [vp]
    L.rad_hmat_n.restype = ctypes.c_int64
    L.rad_hmat_dtype.argtypes = [vp]
    L.rad_hmat_dtype.restype = ctypes.c_int32
    L.rad_hmat_lowp.argtypes = [vp]
    L.rad_hmat_lowp.restype = ctypes.c_int32
    L.rad_hmat_max_rhs.argtypes = [vp]
    L.rad_hmat_max_rhs.restype = ctypes.c_int32
    L.rad_hmat_perm.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.rad_hmat_perm.restype = ctypes.c_int
    L.rad_hmat_free.argtypes = [vp]
    L.rad_hmat_free.restype = None
    L.rad_last_error.argtypes = []
    L.rad_last_error.restype = ctypes.c_char_p
    i64, i32, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    sigs = {
        "rad_pod_build": [vp, i64, i64, i64, i32, vp, i64, vp, i32, vp],
        "rad_pod_project": [vp, i64, i32, i64, vp, vp, i64, i64, vp, vp, vp],
        "rad_pod_expand": [vp, i64, i32, i64, vp, vp, vp, i64, i64, vp, vp],
        "rad_mlp_create": [vp, i32, vp, i32, i32, i32, ctypes.POINTER(vp)],
        "rad_mlp_get_params": [vp, vp],
        "rad_mlp_set_params": [vp, vp],
        "rad_mlp_forward": [vp, vp, i64, vp, vp],
        "rad_mlp_loss_grad": [vp, vp, vp, vp, i64, vp, vp, vp],
        "rad_mlp_adam_step": [vp, dbl, dbl, dbl, dbl, vp],
        "rad_mlp_train": [vp, vp, vp, vp, i64, i32, dbl, dbl, dbl, dbl, vp, vp],
    }
    for name, args in sigs.items():
        getattr(L, name).argtypes = args
        getattr(L, name).restype = ctypes.c_int
    L.rad_hmat_group.argtypes = [vp, i32, i32, ctypes.POINTER(vp)]
    L.rad_hmat_group.restype = ctypes.c_int
    L.rad_hmat_instances.argtypes = [vp]
    L.rad_hmat_instances.restype = i32
    L.rad_hmat_group_layout.argtypes = [vp, vp, vp]
    L.rad_hmat_group_layout.restype = ctypes.c_int
    L.rad_hmat_autotune.argtypes = [vp, i64, i32, ctypes.c_char_p, vp, vp, vp]
    L.rad_hmat_autotune.restype = ctypes.c_int
    L.rad_hmat_set_config.argtypes = [vp, i64, vp]
    L.rad_hmat_set_config.restype = ctypes.c_int
    L.rad_hmat_get_config.argtypes = [vp, i64, vp]
    L.rad_hmat_get_config.restype = ctypes.c_int
    L.rad_mlp_param_count.argtypes = [vp]
    L.rad_mlp_param_count.restype = i64
    L.rad_mlp_free.argtypes = [vp]
    L.rad_mlp_free.restype = None
    _lib = L
    return L


def _check(status):
    if status != RAD_OK:
        raise RadError(status, load().rad_last_error().decode())


def _torch():
    import torch
    return torch


def _stream_handle():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def ldr_of(R: int) -> int:
    """Leading dimension of the internal R-major layout for R right-hand sides."""
    return (int(R) + 3) // 4 * 4


def _rmajor(t, N, R):
    """Check a (N, ldr_of(R)) row-major device tensor for RAD_ORDER_TREE_RMAJOR."""
    ldr = ldr_of(R)
    if t.dim() != 2 or t.shape[0] != N or t.shape[1] != ldr or not t.is_contiguous():
        raise ValueError(f"tree_rmajor tensors must be contiguous with shape ({N}, {ldr})")
    return t, ldr


def _colmajor(t, N):
    """View a (N,) or (N,R) device tensor as column-major with leading dimension >= N."""
    if t.dim() == 1:
        t = t.reshape(N, 1)
    if t.stride(0) != 1 or (t.shape[1] > 1 and t.stride(1) < N):
        t = t.t().contiguous().t()
    ld = t.stride(1) if t.shape[1] > 1 else N
    return t, ld


def _build_opts(tol, leaf_size, max_depth, nearfield, visibility, storage, oversample, power_iters, max_rhs, device,
                seed, verbose, max_rank, lowp, allocator):
    o = BuildOpts()
    load().rad_build_opts_default(ctypes.byref(o))
    o.tol = float(tol)
    o.leaf_size = int(leaf_size)
    o.max_depth = int(max_depth)
    o.nearfield = NEARFIELD[nearfield]
    o.visibility = VISIBILITY[visibility]
    o.storage = DTYPES[storage]
    o.oversample = int(oversample)
    o.power_iters = int(power_iters)
    o.max_rhs = int(max_rhs)
    o.device = int(device)
    o.seed = int(seed)
    o.verbose = int(bool(verbose))
    o.max_rank = int(max_rank)
    o.lowp = {None: 0, "f16": RAD_F16, "bf16": RAD_BF16}[lowp]
    if allocator is not None:
        o.allocator = ctypes.pointer(allocator.struct)
    return o


def _allocator(allocator):
    if allocator is None or isinstance(allocator, TorchAllocator):
        return allocator
    if allocator == "torch":
        return TorchAllocator()
    raise ValueError("allocator must be None, 'torch' or a TorchAllocator")


class HMatrix:
    """Compressed view-factor matrix F-hat resident on one GPU.
    allocator="torch" places all of its device memory in torch's caching
    allocator (rad_allocator hook)."""

    def __init__(self, verts, faces, tol=1e-3, leaf_size=64, max_depth=0, nearfield="auto",
                 visibility="backface", storage="f64", oversample=8, power_iters=1, max_rhs=1, device=0,
                 seed=0x5EED, verbose=False, max_rank=0, lowp=None, tree="quad", allocator=None):
        L = load()
        alloc = _allocator(allocator)
        o = _build_opts(tol, leaf_size, max_depth, nearfield, visibility, storage, oversample, power_iters, max_rhs,
                        device, seed, verbose, max_rank, lowp, alloc)
        v = np.ascontiguousarray(verts, dtype=np.float64)
        f = np.ascontiguousarray(faces, dtype=np.int32)
        h = ctypes.c_void_p()
        if tree not in ("quad", "oct"):
            raise ValueError("tree must be 'quad' (on x, y) or 'oct' (on x, y, z)")
        if tree == "quad":
            _check(L.rad_hmat_build(v.ctypes.data, v.shape[0], f.ctypes.data, f.shape[0], ctypes.byref(o),
                                    ctypes.byref(h)))
        else:
            _check(L.rad_hmat_build_tree(v.ctypes.data, v.shape[0], f.ctypes.data, f.shape[0], ctypes.byref(o), 3,
                                         ctypes.byref(h)))
        self._adopt(h, int(o.lowp), int(max_rhs), int(device), alloc)

    def _adopt(self, h, lowp, max_rhs, device, alloc):
        L = load()
        self._alloc = alloc      # keeps the allocator's callbacks alive as long as the matrix
        self._h = h
        self.N = int(L.rad_hmat_n(h))
        self.rad_dtype = int(L.rad_hmat_dtype(h))
        self.lowp = int(lowp)
        self.max_rhs = int(max_rhs)
        self.device = int(device)
        self.n_inst = int(L.rad_hmat_instances(h))

    @classmethod
    def from_facets(cls, x, n, area, tri=None, tol=1e-3, leaf_size=64, max_depth=0, nearfield="auto",
                    visibility="backface", storage="f64", oversample=8, power_iters=1, max_rhs=1, device=0,
                    seed=0x5EED, verbose=False, max_rank=0, lowp=None, tree="quad", allocator=None):
        """Build from centroids x (N, 3), unit normals n (N, 3) and areas (N,);
        tri (N, 3, 3) the facets' triangles for ray casting and shadows, or None."""
        L = load()
        alloc = _allocator(allocator)
        o = _build_opts(tol, leaf_size, max_depth, nearfield, visibility, storage, oversample, power_iters, max_rhs,
                        device, seed, verbose, max_rank, lowp, alloc)
        xa = np.ascontiguousarray(x, dtype=np.float64)
        na = np.ascontiguousarray(n, dtype=np.float64)
        aa = np.ascontiguousarray(area, dtype=np.float64)
        N = aa.shape[0]
        if xa.shape != (N, 3) or na.shape != (N, 3):
            raise ValueError("x and n must have shape (N, 3)")
        ta = None if tri is None else np.ascontiguousarray(np.reshape(tri, (N, 9)), dtype=np.float64)
        if tree not in ("quad", "oct"):
            raise ValueError("tree must be 'quad' (on x, y) or 'oct' (on x, y, z)")
        h = ctypes.c_void_p()
        _check(L.rad_hmat_build_facets(xa.ctypes.data, na.ctypes.data, aa.ctypes.data, N,
                                       None if ta is None else ta.ctypes.data, ctypes.byref(o),
                                       2 if tree == "quad" else 3, ctypes.byref(h)))
        self = object.__new__(cls)
        self._adopt(h, int(o.lowp), int(max_rhs), int(device), alloc)
        return self

    @classmethod
    def load(cls, path, device=0, max_rhs=0, allocator=None):
        """Read a matrix written by save(); workspace for max_rhs columns
        (0: the saved matrix's)."""
        L = load()
        alloc = _allocator(allocator)
        h = ctypes.c_void_p()
        _check(L.rad_hmat_load(str(path).encode(), int(device), int(max_rhs),
                               None if alloc is None else ctypes.pointer(alloc.struct), ctypes.byref(h)))
        self = object.__new__(cls)
        self._adopt(h, int(L.rad_hmat_lowp(h)), int(L.rad_hmat_max_rhs(h)), int(device), alloc)
        if self.n_inst > 1:
            self.offsets = np.zeros(self.n_inst, dtype=np.int64)
            self.sizes = np.zeros(self.n_inst, dtype=np.int64)
            _check(L.rad_hmat_group_layout(h, self.offsets.ctypes.data, self.sizes.ctypes.data))
        return self

    def convert(self, storage, max_rhs=0):
        """The same compressed operator stored in another precision ("f64" or
        "f32"), as a new matrix (rad_hmat_convert)."""
        L = load()
        h = ctypes.c_void_p()
        _check(L.rad_hmat_convert(self._h, DTYPES[storage], int(max_rhs), ctypes.byref(h)))
        G = object.__new__(type(self))
        G._adopt(h, 0, int(L.rad_hmat_max_rhs(h)), self.device, getattr(self, "_alloc", None))
        return G

    def save(self, path):
        """Write the whole compressed operator to a file (rad_hmat_save)."""
        _check(load().rad_hmat_save(self._h, str(path).encode()))

    def export(self, path):
        """Write the blocks of F-hat, FP64, to a file (rad_hmat_export)."""
        _check(load().rad_hmat_export(self._h, str(path).encode()))

    @classmethod
    def group(cls, parts, max_rhs):
        """Block-diagonal group of built matrices (one launch per kernel for all
        instances).  Its layout is tree_rmajor with instance k at rows
        offsets[k] .. offsets[k] + sizes[k]; padding rows between instances stay zero."""
        L = load()
        arr = (ctypes.c_void_p * len(parts))(*[p._h.value for p in parts])
        h = ctypes.c_void_p()
        _check(L.rad_hmat_group(arr, len(parts), int(max_rhs), ctypes.byref(h)))
        self = object.__new__(cls)
        self._alloc = getattr(parts[0], "_alloc", None)   # the group allocates through the parts' hook
        self._h = h
        self.N = int(L.rad_hmat_n(h))
        self.rad_dtype = int(L.rad_hmat_dtype(h))
        self.lowp = parts[0].lowp
        self.max_rhs = int(max_rhs)
        self.device = parts[0].device
        self.n_inst = int(L.rad_hmat_instances(h))
        self.offsets = np.zeros(self.n_inst, dtype=np.int64)
        self.sizes = np.zeros(self.n_inst, dtype=np.int64)
        _check(L.rad_hmat_group_layout(h, self.offsets.ctypes.data, self.sizes.ctypes.data))
        return self

    @property
    def torch_dtype(self):
        torch = _torch()
        return torch.float64 if self.rad_dtype == RAD_F64 else torch.float32

    def autotune(self, R, nrep=5, cache=None):
        """Pick the fastest multi-RHS launch configuration for R columns
        (timed on this matrix, or read from the JSON cache file)."""
        cfg = np.zeros(3, dtype=np.int32)
        ms = ctypes.c_double()
        path = None if cache is None else str(cache).encode()
        _check(load().rad_hmat_autotune(self._h, int(R), int(nrep), path, cfg.ctypes.data, ctypes.byref(ms),
                                        _stream_handle()))
        return {"tn": int(cfg[0]), "persistent": int(cfg[1]), "blocks_per_cu": int(cfg[2]), "ms": ms.value}

    def set_config(self, R, tn, persistent=0, blocks_per_cu=2):
        cfg = np.array([tn, persistent, blocks_per_cu], dtype=np.int32)
        _check(load().rad_hmat_set_config(self._h, int(R), cfg.ctypes.data))

    def get_config(self, R):
        cfg = np.zeros(3, dtype=np.int32)
        _check(load().rad_hmat_get_config(self._h, int(R), cfg.ctypes.data))
        return {"tn": int(cfg[0]), "persistent": int(cfg[1]), "blocks_per_cu": int(cfg[2])}

    def stats(self) -> dict:
        s = Stats()
        _check(load().rad_hmat_info(self._h, ctypes.byref(s)))
        return s.as_dict()

    def perm(self) -> np.ndarray:
        p = np.empty(self.N, dtype=np.int32)
        _check(load().rad_hmat_perm(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return p

    def matvec(self, X, out=None, order="original", R=None, lowp=False):
        """Y = F-hat X.  Column-major orders take X of shape (N,) or (N, R);
        order="tree_rmajor" takes the internal layout, shape (N, ldr_of(R)).
        lowp=True applies the 16-bit copy of the operator (FP32 X and Y)."""
        torch = _torch()
        dt = self.lowp if lowp else self.rad_dtype
        if order == "tree_rmajor":
            R = int(R if R is not None else X.shape[1])
            Xc, ldx = _rmajor(X, self.N, R)
            if out is None:
                out = torch.zeros_like(X)
            Yc, ldy = _rmajor(out, self.N, R)
            _check(load().rad_hmat_matvec(self._h, R, dt, ctypes.c_void_p(Xc.data_ptr()), ldx,
                                          ctypes.c_void_p(Yc.data_ptr()), ldy, ORDER[order], _stream_handle()))
            return out
        squeeze = X.dim() == 1
        Xc, ldx = _colmajor(X, self.N)
        R = Xc.shape[1]
        if out is None:
            out = torch.empty((R, self.N), dtype=X.dtype, device=X.device).t()
        Yc, ldy = _colmajor(out, self.N)
        _check(load().rad_hmat_matvec(self._h, R, dt, ctypes.c_void_p(Xc.data_ptr()), ldx,
                                      ctypes.c_void_p(Yc.data_ptr()), ldy, ORDER[order], _stream_handle()))
        if Yc.data_ptr() != out.data_ptr():
            out.copy_(Yc)
        return out.reshape(-1) if squeeze else out

    def matvec_noalloc(self, X, out, order="original", R=None):
        """Y = F-hat X through rad_hmat_matvec_noalloc (1 <= R <= 15): the
        library allocates nothing; `out` is the caller's preallocated Y in the
        layout `order` names (for column-major orders it must already be
        column-major with leading dimension >= N)."""
        if order == "tree_rmajor":
            R = int(R if R is not None else X.shape[1])
            Xc, ldx = _rmajor(X, self.N, R)
            Yc, ldy = _rmajor(out, self.N, R)
        else:
            Xc, ldx = _colmajor(X, self.N)
            R = Xc.shape[1]
            Yc, ldy = _colmajor(out, self.N)
            if Yc.data_ptr() != out.data_ptr():
                raise ValueError("out must be column-major with leading dimension >= N")
        _check(load().rad_hmat_matvec_noalloc(self._h, R, self.rad_dtype, ctypes.c_void_p(Xc.data_ptr()), ldx,
                                              ctypes.c_void_p(Yc.data_ptr()), ldy, ORDER[order], _stream_handle()))
        return out

    def solve(self, E, rho=0.3, rtol=1e-3, max_iter=100, order="original", check_every=1, out=None,
              raise_on_noconv=True, use_graph=True, R=None, refine=False, inner_iters=3, warm=None,
              method="jacobi", lam=None, restart=30):
        """Solve of (I - diag(rho) F-hat) B = E; returns (B, info dict).
        method: "jacobi" (the paper's), "chebyshev" (scalar rho; lam = (lo, hi)
        an interval holding F-hat's spectrum, default from the largest row sum)
        or "gmres" (restart = Arnoldi steps per cycle).
        warm: optional starting guess in the layout of B (judged per column
        against the cold start); it may be `out` itself (Jacobi only)."""
        torch = _torch()
        L = load()
        squeeze = False
        if order == "tree_rmajor":
            R = int(R if R is not None else E.shape[1])
            Ec, lde = _rmajor(E, self.N, R)
            if out is None:
                out = torch.zeros_like(E)
            Bc, ldb = _rmajor(out, self.N, R)
        else:
            squeeze = E.dim() == 1
            Ec, lde = _colmajor(E, self.N)
            R = Ec.shape[1]
            if out is None:
                out = torch.empty((R, self.N), dtype=E.dtype, device=E.device).t()
            Bc, ldb = _colmajor(out, self.N)
        if warm is not None:
            if warm.shape[0] != self.N or warm.dtype != Bc.dtype:
                raise ValueError("warm must match B in shape and dtype")
            if warm.data_ptr() != Bc.data_ptr():
                Bc.copy_(warm if order == "tree_rmajor" else warm.reshape(Bc.shape))
        rho_ptr = ctypes.c_void_p(0)
        rho_s = 0.0
        if isinstance(rho, (float, int)):
            rho_s = float(rho)
        else:
            rho_t = rho.contiguous()
            rho_ptr = ctypes.c_void_p(rho_t.data_ptr())
        o = SolveOpts()
        L.rad_solve_opts_default(ctypes.byref(o))
        o.rtol = float(rtol)
        o.max_iter = int(max_iter)
        o.order = ORDER[order]
        o.check_every = int(check_every)
        o.use_graph = int(bool(use_graph))
        o.refine = int(bool(refine))
        o.inner_iters = int(inner_iters)
        o.warm = int(warm is not None)
        o.method = METHODS[method]
        if lam is not None:
            o.lam_lo, o.lam_hi = float(lam[0]), float(lam[1])
        o.restart = int(restart)
        iters = np.zeros(R * self.n_inst, dtype=np.int32)
        rel = np.zeros(R * self.n_inst, dtype=np.float64)
        info = SolveInfo(iters.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                         rel.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 0, 0, 0)
        st = L.rad_solve(self._h, rho_ptr, rho_s, R, self.rad_dtype, ctypes.c_void_p(Ec.data_ptr()), lde,
                         ctypes.c_void_p(Bc.data_ptr()), ldb, ctypes.byref(o), ctypes.byref(info),
                         _stream_handle())
        if st != RAD_OK and not (st == RAD_ENOCONV and not raise_on_noconv):
            _check(st)
        if Bc.data_ptr() != out.data_ptr():
            out.copy_(Bc)
        res = {"iters": iters, "rel_change": rel, "total_iters": int(info.total_iters),
               "inner_iters": int(info.inner_iters), "warm_columns": int(info.warm_columns),
               "converged": st == RAD_OK}
        return (out.reshape(-1) if squeeze else out), res

    def insolation(self, suns, flux=1365.0, order="original", out=None):
        """Q_dir on the device for sun unit vectors suns (R, 3): shape (N, R)
        column-major, or (N, ldr_of(R)) for order="tree_rmajor"."""
        torch = _torch()
        s = np.ascontiguousarray(np.atleast_2d(suns), dtype=np.float64)
        R = s.shape[0]
        dev = f"cuda:{self.device}"
        if order == "tree_rmajor":
            if out is None:
                out = torch.zeros((self.N, ldr_of(R)), dtype=self.torch_dtype, device=dev)
            Qc, ldq = _rmajor(out, self.N, R)
        else:
            if out is None:
                out = torch.empty((R, self.N), dtype=self.torch_dtype, device=dev).t()
            Qc, ldq = _colmajor(out, self.N)
        _check(load().rad_insolation(self._h, R, s.ctypes.data, float(flux), self.rad_dtype,
                                     ctypes.c_void_p(Qc.data_ptr()), ldq, ORDER[order], _stream_handle()))
        if Qc.data_ptr() != out.data_ptr():
            out.copy_(Qc)
        return out

    def equilibrium(self, Qdir, albedo=0.3, emissivity=0.99, rtol=1e-8, max_iter=200, order="original", R=None,
                    use_graph=True):
        """Two-band equilibrium temperature; returns (T, Q_vis, Q_IR, info)."""
        torch = _torch()
        L = load()
        if order == "tree_rmajor":
            R = int(R if R is not None else Qdir.shape[1])
            Qc, ld = _rmajor(Qdir, self.N, R)
            mk = lambda: torch.zeros_like(Qc)
        else:
            Q2 = Qdir.reshape(self.N, -1)
            Qc = Q2.t().contiguous().t()
            R, ld = Qc.shape[1], self.N
            mk = lambda: torch.empty((R, self.N), dtype=Qc.dtype, device=Qc.device).t()
        T, Qv, Qi = mk(), mk(), mk()
        o = SolveOpts()
        L.rad_solve_opts_default(ctypes.byref(o))
        o.rtol, o.max_iter, o.order, o.use_graph = float(rtol), int(max_iter), ORDER[order], int(bool(use_graph))
        its = [np.zeros(R, dtype=np.int32) for _ in range(2)]
        infos = [SolveInfo(x.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), None, 0, 0, 0) for x in its]
        p = lambda t: ctypes.c_void_p(t.data_ptr())
        _check(L.rad_equilibrium(self._h, R, self.rad_dtype, p(Qc), ld, float(albedo), float(emissivity), p(T),
                                 p(Qv), p(Qi), ctypes.byref(o), ctypes.byref(infos[0]), ctypes.byref(infos[1]),
                                 _stream_handle()))
        return T, Qv, Qi, {"iters_sw": its[0], "iters_ir": its[1]}

    def time_phases(self, R, nrep=20, lowp=False):
        """Average ms per launch of (projections, split-K sum, expansion + Jacobi update);
        lowp=True times the 16-bit kernels."""
        ms = (ctypes.c_double * 3)()
        dt = self.lowp if lowp else self.rad_dtype
        _check(load().rad_hmat_time_phases(self._h, int(R), dt, int(nrep), _stream_handle(), ms))
        return list(ms)

    def close(self):
        if getattr(self, "_h", None):
            load().rad_hmat_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
