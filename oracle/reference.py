"""Plain FP64 CPU reference for the radiosity model (TEST INFRASTRUCTURE ONLY).

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark import this module.  The product library never does; the two share
no code.  Heavy O(N^2)/O(N^3) loops live in ``vf_oracle.c`` (plain C, FP64);
this module wraps them with ctypes and adds the small numpy pieces.

Paper passages followed (Potter et al., arXiv 2209.07632):
  * geometry and eq. FF-def ........................ section 3
  * visibility V_ij .................................. section 3.2
  * insolation, eq. insolation ....................... section 2 / 5.1
  * radiosity system B = E + diag(rho) F B ........... eq. radiosity-system
  * Jacobi relaxation ................................ section 3 / 5.1
  * Chebyshev acceleration (not in the paper) ........ Saad, section 12.1
  * GMRES (a Krylov solve for the same systems) ...... Saad, section 6.5
  * two-band equilibrium, eqs. Qvis, QIR, 3d-equilbr . sections 2 and 5.1
  * closed-form bowl-crater temperature .............. section 7.1
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build_oracle

SIGMA_SB = 5.670374419e-8  # Stefan-Boltzmann constant, W m^-2 K^-4

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = build_oracle.LIB
        if not os.path.exists(path):
            build_oracle.build(force=True)
        L = ctypes.CDLL(path)
        d = ctypes.POINTER(ctypes.c_double)
        u8 = ctypes.POINTER(ctypes.c_uint8)
        i32 = ctypes.POINTER(ctypes.c_int32)
        i64 = ctypes.POINTER(ctypes.c_int64)
        L.orc_geometry.argtypes = [d, ctypes.c_int64, i32, ctypes.c_int64, d, d, d]
        L.orc_geometry.restype = ctypes.c_int64
        L.orc_pair_visibility.argtypes = [ctypes.c_int64, d, d, ctypes.c_int64, d, ctypes.c_int, u8]
        L.orc_F_dense.argtypes = [ctypes.c_int64, d, d, d, u8, d]
        L.orc_F_rows.argtypes = [ctypes.c_int64, d, d, d, ctypes.c_int64, d, ctypes.c_int,
                                 ctypes.c_int64, i64, d]
        L.orc_directed_visibility.argtypes = [ctypes.c_int64, d, d, ctypes.c_int64, d, u8]
        L.orc_matvec_free.argtypes = [ctypes.c_int64, d, d, d, u8, ctypes.c_int64, d,
                                      ctypes.c_int64, d, ctypes.c_int64]
        L.orc_sun_visibility.argtypes = [ctypes.c_int64, d, ctypes.c_int64, d, ctypes.c_int64,
                                         d, u8]
        L.orc_ray_hits_triangle.argtypes = [d, d, ctypes.c_double, ctypes.c_double, d]
        L.orc_ray_hits_triangle.restype = ctypes.c_int
        L.orc_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a, ct=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def num_threads() -> int:
    return int(lib().orc_num_threads())


# --------------------------------------------------------------------------
# Geometry and the view-factor matrix (section 3)
# --------------------------------------------------------------------------
class Facets:
    """Centroids x (N,3), unit normals n (N,3), areas A (N,) and the mesh triangles."""

    def __init__(self, verts, faces):
        verts = np.ascontiguousarray(verts, dtype=np.float64)
        faces = np.ascontiguousarray(faces, dtype=np.int32)
        N = faces.shape[0]
        self.x = np.empty((N, 3))
        self.n = np.empty((N, 3))
        self.A = np.empty(N)
        bad = lib().orc_geometry(_p(verts), verts.shape[0], _p(faces, ctypes.c_int32), N,
                                 _p(self.x), _p(self.n), _p(self.A))
        if bad:
            raise ValueError(f"{bad} degenerate faces")
        self.tri = np.ascontiguousarray(verts[faces].reshape(N, 9))
        self.N = N

    @classmethod
    def from_arrays(cls, x, n, A, tri=None):
        """Facets given directly by centroid, unit normal and area (no mesh)."""
        self = cls.__new__(cls)
        self.x = np.ascontiguousarray(x, dtype=np.float64)
        self.n = np.ascontiguousarray(n, dtype=np.float64)
        self.A = np.ascontiguousarray(A, dtype=np.float64)
        self.N = self.x.shape[0]
        self.tri = (np.zeros((self.N, 9)) if tri is None
                    else np.ascontiguousarray(tri, dtype=np.float64).reshape(self.N, 9))
        return self


def pair_visibility(fac: Facets, mode: str = "raycast") -> np.ndarray:
    """V (N,N) uint8: back-face test then (mode 'raycast') a brute-force segment test."""
    m = {"backface": 0, "raycast": 1}[mode]
    vis = np.empty((fac.N, fac.N), dtype=np.uint8)
    lib().orc_pair_visibility(fac.N, _p(fac.x), _p(fac.n), fac.N, _p(fac.tri), m,
                              _p(vis, ctypes.c_uint8))
    return vis


def directed_visibility(fac: Facets) -> np.ndarray:
    """Segment test cast from the row facet for every ordered facing pair (not
    symmetrised); test use only: it exposes the pairs whose two directions
    disagree, which the once-per-pair cast of ``pair_visibility`` settles."""
    vis = np.empty((fac.N, fac.N), dtype=np.uint8)
    lib().orc_directed_visibility(fac.N, _p(fac.x), _p(fac.n), fac.N, _p(fac.tri), _p(vis, ctypes.c_uint8))
    return vis


def view_factor_matrix(fac: Facets, vis: np.ndarray | None = None) -> np.ndarray:
    """Dense F (eq. FF-def); ``vis=None`` means back-face visibility only."""
    F = np.empty((fac.N, fac.N))
    vp = None if vis is None else _p(np.ascontiguousarray(vis, dtype=np.uint8), ctypes.c_uint8)
    lib().orc_F_dense(fac.N, _p(fac.x), _p(fac.n), _p(fac.A), vp, _p(F))
    return F


def view_factor_rows(fac: Facets, rows, mode: str = "backface") -> np.ndarray:
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty((rows.size, fac.N))
    m = {"backface": 0, "raycast": 1}[mode]
    lib().orc_F_rows(fac.N, _p(fac.x), _p(fac.n), _p(fac.A), fac.N, _p(fac.tri), m,
                     rows.size, _p(rows, ctypes.c_int64), _p(out))
    return out


def matvec_free(fac: Facets, X: np.ndarray, vis: np.ndarray | None = None) -> np.ndarray:
    """Y = F X with rows of F computed on the fly (no N x N storage)."""
    X2 = np.asfortranarray(X.reshape(fac.N, -1), dtype=np.float64)
    R = X2.shape[1]
    Y = np.empty((fac.N, R), order="F")
    vp = None if vis is None else _p(np.ascontiguousarray(vis, dtype=np.uint8), ctypes.c_uint8)
    lib().orc_matvec_free(fac.N, _p(fac.x), _p(fac.n), _p(fac.A), vp, R, _p(X2), fac.N,
                          _p(Y), fac.N)
    return Y.reshape(X.shape)


# --------------------------------------------------------------------------
# Insolation (eq. insolation; point sun, distance in AU)
# --------------------------------------------------------------------------
def sun_visibility(fac: Facets, suns: np.ndarray) -> np.ndarray:
    suns = np.ascontiguousarray(np.atleast_2d(suns), dtype=np.float64)
    R = suns.shape[0]
    out = np.empty((R, fac.N), dtype=np.uint8)  # column-major N x R == row-major R x N
    lib().orc_sun_visibility(fac.N, _p(fac.x), fac.N, _p(fac.tri), R, _p(suns),
                             _p(out, ctypes.c_uint8))
    return out.T


def insolation(fac: Facets, suns: np.ndarray, S: float = 1365.0, dist_au: float = 1.0,
               sunvis: np.ndarray | None = None) -> np.ndarray:
    """Q_dir (N,R) = S / d^2 * sin(e_local) * V_sun with sin(e_local) = max(0, n.s)."""
    suns = np.atleast_2d(suns)
    if sunvis is None:
        sunvis = sun_visibility(fac, suns)
    cos_inc = np.maximum(fac.n @ suns.T, 0.0)
    return (S / dist_au ** 2) * cos_inc * sunvis


# --------------------------------------------------------------------------
# Radiosity solves (eq. radiosity-system)
# --------------------------------------------------------------------------
def jacobi(matvec, rho, E, tol: float = 1e-13, max_iter: int = 500):
    """Relaxation B^{k+1} = E + rho * (F B^k), B^0 = E (F_ii = 0, so this is Jacobi).

    Stops when every column has ||B^{k+1}-B^k||_2 <= tol ||E||_2.  Returns
    (B, iters) with iters[c] the first k at which column c met the test.
    Raises RuntimeError after ``max_iter`` iterations.
    """
    E2 = E.reshape(E.shape[0], -1)
    rho = np.asarray(rho, dtype=np.float64)
    rho2 = rho.reshape(-1, 1) if rho.ndim else rho
    enorm = np.linalg.norm(E2, axis=0)
    B = E2.copy()
    iters = np.full(E2.shape[1], -1, dtype=np.int64)
    for k in range(1, max_iter + 1):
        Bn = E2 + rho2 * matvec(B)
        d = np.linalg.norm(Bn - B, axis=0)
        B = Bn
        done = d <= tol * np.where(enorm > 0, enorm, 1.0)
        iters[(iters < 0) & done] = k
        if np.all(iters >= 0):
            return B.reshape(E.shape), iters
    raise RuntimeError("Jacobi did not converge")


def chebyshev(matvec, rho: float, E, lam_lo: float, lam_hi: float, tol: float = 1e-13, max_iter: int = 500,
              strict: bool = True):
    """Chebyshev acceleration of B = E + rho F B (not in the paper: a faster
    iteration for systems whose F has a spectral radius near one).

    Reciprocity (A_i F_ij = A_j F_ji, eq. FF-def with symmetric visibility)
    makes F self-adjoint in the area-weighted inner product, so its spectrum
    is real.  Given [lam_lo, lam_hi] containing it, M = I - rho F has its
    spectrum in [1 - rho lam_hi, 1 - rho lam_lo] (rho > 0), and the
    three-term Chebyshev iteration for M B = E (Saad, Iterative Methods for
    Sparse Linear Systems, 2nd ed., section 12.1) is run from B^0 = E with one
    product per iteration: its error in the area-weighted norm is at most
    the initial error over T_k(theta / delta), theta and delta the centre and
    half-width of that interval.  Stops when every column's recurrence
    residual is <= tol ||E||.  Returns (B, iters); after max_iter iterations
    it raises, or with strict=False returns that iterate.
    """
    E2 = E.reshape(E.shape[0], -1)
    lo, hi = 1.0 - rho * lam_hi, 1.0 - rho * lam_lo
    if not 0.0 < lo <= hi:
        raise ValueError("need 0 < 1 - rho lam_hi <= 1 - rho lam_lo")
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    enorm = np.linalg.norm(E2, axis=0)
    thr = tol * np.where(enorm > 0, enorm, 1.0)
    B = E2.copy()
    r = E2 - (B - rho * matvec(B))
    iters = np.full(E2.shape[1], -1, dtype=np.int64)
    iters[np.linalg.norm(r, axis=0) <= thr] = 0
    if delta == 0.0:      # a single point: one scaled step is exact
        return (B + r / theta).reshape(E.shape), np.maximum(iters, 1)
    sigma = theta / delta
    rk = 1.0 / sigma
    d = r / theta
    for k in range(1, max_iter + 1):
        B = B + d
        r = r - (d - rho * matvec(d))
        iters[(iters < 0) & (np.linalg.norm(r, axis=0) <= thr)] = k
        if np.all(iters >= 0):
            return B.reshape(E.shape), iters
        rk1 = 1.0 / (2.0 * sigma - rk)
        d = rk1 * rk * d + (2.0 * rk1 / delta) * r
        rk = rk1
    if strict:
        raise RuntimeError("Chebyshev iteration did not converge")
    return B.reshape(E.shape), iters


def gmres(matvec, rho, E, tol: float = 1e-13, restart: int = 50, max_iter: int = 500):
    """GMRES for (I - diag(rho) F) B = E, one column at a time, from B = 0
    (Saad, Iterative Methods for Sparse Linear Systems, 2nd ed., section 6.5:
    Arnoldi with modified Gram-Schmidt, Givens rotations on the Hessenberg
    matrix, restarted every ``restart`` steps).  Stops a column when its
    residual norm is <= tol ||E_c||.  Returns (B, iters, history) with iters[c]
    the number of Arnoldi steps (products) taken and history[c] the residual
    norms after 0, 1, 2, ... steps.
    """
    E2 = E.reshape(E.shape[0], -1)
    n, R = E2.shape
    rho = np.broadcast_to(np.asarray(rho, dtype=np.float64), (n,))

    def A(v):
        return v - rho * matvec(v[:, None])[:, 0]

    B = np.zeros_like(E2, dtype=np.float64)
    iters = np.zeros(R, dtype=np.int64)
    history = []
    for c in range(R):
        b = E2[:, c].astype(np.float64)
        thr = tol * (np.linalg.norm(b) if np.linalg.norm(b) > 0 else 1.0)
        x = np.zeros(n)
        r = b.copy()
        beta = np.linalg.norm(r)
        hist = [beta]
        steps = 0
        while beta > thr and steps < max_iter:
            m = min(restart, max_iter - steps)
            V = np.zeros((m + 1, n))
            Hm = np.zeros((m + 1, m))
            cs, sn = np.zeros(m), np.zeros(m)
            g = np.zeros(m + 1)
            g[0] = beta
            V[0] = r / beta
            j_done = 0
            for j in range(m):
                w = A(V[j])
                for i in range(j + 1):            # modified Gram-Schmidt
                    Hm[i, j] = w @ V[i]
                    w = w - Hm[i, j] * V[i]
                Hm[j + 1, j] = np.linalg.norm(w)
                if Hm[j + 1, j] > 0:
                    V[j + 1] = w / Hm[j + 1, j]
                for i in range(j):                # earlier rotations on the new column
                    t = cs[i] * Hm[i, j] + sn[i] * Hm[i + 1, j]
                    Hm[i + 1, j] = -sn[i] * Hm[i, j] + cs[i] * Hm[i + 1, j]
                    Hm[i, j] = t
                d = np.hypot(Hm[j, j], Hm[j + 1, j])
                cs[j], sn[j] = Hm[j, j] / d, Hm[j + 1, j] / d
                Hm[j, j], Hm[j + 1, j] = d, 0.0
                g[j + 1] = -sn[j] * g[j]
                g[j] = cs[j] * g[j]
                j_done = j + 1
                steps += 1
                hist.append(abs(g[j + 1]))
                if abs(g[j + 1]) <= thr or Hm[j, j] == 0.0:
                    break
            y = np.linalg.solve(np.triu(Hm[:j_done, :j_done]), g[:j_done])
            x = x + V[:j_done].T @ y
            r = b - A(x)
            beta = np.linalg.norm(r)
        if beta > thr:
            raise RuntimeError("GMRES did not converge")
        B[:, c] = x
        iters[c] = steps
        history.append(np.array(hist))
    return B.reshape(E.shape), iters, history


def solve_direct(F: np.ndarray, rho, E: np.ndarray) -> np.ndarray:
    """LAPACK solve of (I - diag(rho) F) B = E."""
    rho = np.broadcast_to(np.asarray(rho, dtype=np.float64), (F.shape[0],))
    M = np.eye(F.shape[0]) - rho[:, None] * F
    return np.linalg.solve(M, E)


def equilibrium_temperature(matvec, Qdir, albedo: float, emiss: float, H=0.0,
                            tol: float = 1e-13):
    """Two-band equilibrium (section 5.1 with eqs. Qvis, QIR, 3d-equilbr).

    Short wave: B_s = albedo * (Q_dir + Q_refl) solves (I - albedo F) B_s = albedo Q_dir;
    Q_refl = F B_s.  Long wave: B_IR = (1-albedo) Q_vis + H + Q_IR solves
    (I - F) B_IR = (1-albedo) Q_vis + H; Q_IR = F B_IR.  Then
    emiss sigma T^4 = (1-albedo) Q_vis + emiss Q_IR (negative flux clamped to 0).
    """
    Bs, it_s = jacobi(matvec, albedo, albedo * Qdir, tol=tol)
    Qrefl = matvec(Bs)
    Qvis = Qdir + Qrefl
    Bir, it_ir = jacobi(matvec, 1.0, (1.0 - albedo) * Qvis + H, tol=tol)
    Qir = matvec(Bir)
    absorbed = np.maximum((1.0 - albedo) * Qvis + emiss * Qir, 0.0)
    T = (absorbed / (emiss * SIGMA_SB)) ** 0.25
    return dict(B_s=Bs, Q_refl=Qrefl, Q_vis=Qvis, B_ir=Bir, Q_ir=Qir, T=T,
                iters_s=it_s, iters_ir=it_ir)


# --------------------------------------------------------------------------
# Closed form for the spherical-cap crater (section 7.1)
# --------------------------------------------------------------------------
def crater_f(diameter_over_depth: float) -> float:
    """1/f = 1 + (D/d)^2 / 4."""
    return 1.0 / (1.0 + 0.25 * diameter_over_depth ** 2)


def crater_b(f: float, albedo: float, emiss: float) -> float:
    """b = f (emiss + albedo (1-f)) / (1 - albedo f)."""
    return f * (emiss + albedo * (1.0 - f)) / (1.0 - albedo * f)


def crater_temperature(S: float, sin_e_sun: float, sin_e_local, shadowed, albedo: float,
                       emiss: float, f: float):
    """Equilibrium T inside the bowl: emiss sigma T^4 = (1-albedo) S (sin e_loc + b sin e_sun)
    on sunlit facets and (1-albedo) S b sin e_sun on shadowed facets."""
    b = crater_b(f, albedo, emiss)
    direct = np.where(shadowed, 0.0, np.maximum(sin_e_local, 0.0))
    flux = (1.0 - albedo) * S * (direct + b * sin_e_sun)
    return (flux / (emiss * SIGMA_SB)) ** 0.25


def crater_shadow_temperature(S: float, e_sun_deg: float, albedo: float, emiss: float,
                              f: float) -> float:
    """sigma T^4 = S sin e f (1-albedo)/(1-albedo f) * [1 + albedo (1-f)/emiss]."""
    s = np.sin(np.deg2rad(e_sun_deg))
    val = S * s * f * (1.0 - albedo) / (1.0 - albedo * f) * (1.0 + albedo * (1.0 - f) / emiss)
    return (val / SIGMA_SB) ** 0.25
