"""Time-dependent simulation with subsurface heat storage, plain FP64
(TEST INFRASTRUCTURE ONLY: imported by the tests, never by the product).

Paper passages followed (Potter et al., arXiv 2209.07632):
  * heat equation and radiation boundary condition ...... section 2
    (eqs. heat-equation, radiation-boundary-condition)
  * one 1-D column of M layers under each facet centroid,
    flux-conservative, Crank-Nicolson, linearised upper
    boundary, fixed flux at the bottom .................. section 5.2
  * flux recursions of the time stepper ................. Algorithm 6

The paper leaves the column discretisation to its reference; the one used
here is written out in ``cn_step``.  Every column is independent; they are
advanced together with a tridiagonal (Thomas) solve vectorised over columns.
"""
from __future__ import annotations

import numpy as np

from .reference import SIGMA_SB


def layer_depths(M: int, z_max: float, growth: float = 1.0) -> np.ndarray:
    """Node depths z_0 = 0 < z_1 < ... < z_M = z_max (m); layer thickness
    grows geometrically by ``growth`` from the surface down."""
    w = growth ** np.arange(M, dtype=np.float64)
    dz = z_max * w / w.sum()
    return np.concatenate([[0.0], np.cumsum(dz)])


def thomas(lower: np.ndarray, diag: np.ndarray, upper: np.ndarray, rhs: np.ndarray) -> np.ndarray:
    """Solves tridiagonal systems, one per row of the (C, n) arrays:
    lower[:, i] x[i-1] + diag[:, i] x[i] + upper[:, i] x[i+1] = rhs[:, i]
    (lower[:, 0] and upper[:, n-1] are ignored).  Forward elimination and
    back substitution without pivoting (the column systems are diagonally
    dominant)."""
    n = diag.shape[1]
    c = np.empty_like(diag)
    d = np.empty_like(rhs)
    c[:, 0] = upper[:, 0] / diag[:, 0]
    d[:, 0] = rhs[:, 0] / diag[:, 0]
    for i in range(1, n):
        m = diag[:, i] - lower[:, i] * c[:, i - 1]
        c[:, i] = upper[:, i] / m if i < n - 1 else 0.0
        d[:, i] = (rhs[:, i] - lower[:, i] * d[:, i - 1]) / m
    x = np.empty_like(rhs)
    x[:, -1] = d[:, -1]
    for i in range(n - 2, -1, -1):
        x[:, i] = d[:, i] - c[:, i] * x[:, i + 1]
    return x


def cell_volumes(z: np.ndarray) -> np.ndarray:
    """Thickness of the control volume of each node: half the layers on
    either side (half a layer at the surface and at the bottom)."""
    dz = np.diff(z)
    V = np.empty(len(z))
    V[0] = 0.5 * dz[0]
    V[-1] = 0.5 * dz[-1]
    V[1:-1] = 0.5 * (dz[:-1] + dz[1:])
    return V


def cn_step(T: np.ndarray, qabs_old: np.ndarray, qabs_new: np.ndarray, dt: float, z: np.ndarray, k: float,
            rhoc: float, emiss, H_bottom) -> np.ndarray:
    """One Crank-Nicolson step of every column (T: (N, M+1), T[:, 0] the
    surface).  Finite volumes around the nodes z_j (``cell_volumes``):

      rhoc V_j dT_j/dt = q_{j-1/2} - q_{j+1/2},  q_{j+1/2} = -k (T_{j+1} - T_j) / (z_{j+1} - z_j)

    (q positive downward); the surface volume receives the net radiative
    input Qabs - emiss sigma T_0^4 from above, the bottom volume the fixed
    upward flux H_bottom from below.  Conduction and Qabs are averaged over
    the old and new time levels; the emission is averaged with its new value
    linearised about T_0^old:  emiss sigma [T^4 + 2 T^3 (T_0^new - T_0^old)]."""
    N, n = T.shape
    V = cell_volumes(z)
    g = k / np.diff(z)                      # conductance of each layer, W m^-2 K^-1
    cap = rhoc * V / dt                     # rhoc V_j / dt
    emiss = np.broadcast_to(np.asarray(emiss, dtype=np.float64), (N,))
    Hb = np.broadcast_to(np.asarray(H_bottom, dtype=np.float64), (N,))
    # conduction operator L T: (L T)_j = g_{j} (T_{j-1} - T_j) + g_{j+1} (T_{j+1} - T_j)
    LT = np.zeros_like(T)
    LT[:, 1:] += g * (T[:, :-1] - T[:, 1:])
    LT[:, :-1] += g * (T[:, 1:] - T[:, :-1])
    lower = np.zeros((N, n))
    upper = np.zeros((N, n))
    diag = np.broadcast_to(cap, (N, n)).copy()
    lower[:, 1:] = -0.5 * g
    upper[:, :-1] = -0.5 * g
    diag[:, 1:] += 0.5 * g
    diag[:, :-1] += 0.5 * g
    rhs = cap * T + 0.5 * LT
    T0 = T[:, 0]
    rad = emiss * SIGMA_SB * T0 ** 4
    drad = 2.0 * emiss * SIGMA_SB * T0 ** 3   # half the derivative of the emission
    diag[:, 0] += drad
    rhs[:, 0] += 0.5 * (qabs_old + qabs_new) - rad + drad * T0
    rhs[:, -1] += Hb
    return thomas(lower, diag, upper, rhs)


def cn_step_balanced(T: np.ndarray, qabs_old: np.ndarray, qabs_new: np.ndarray, dt: float, z: np.ndarray,
                     k: float, rhoc: float, emiss, H_bottom, newton: int = 3) -> np.ndarray:
    """A second reading of the column step: the surface node holds no heat and
    satisfies the radiation boundary condition of section 2 at the new level,

      Qabs' + k (T_1' - T_0') / z_1 = emiss sigma T_0'^4.

    Nodes 1..M take the Crank-Nicolson average of conduction (half a layer at
    the bottom, which receives H_bottom); node 1 exchanges with the surface at
    both levels, the old surface temperature having met the balance with Qabs
    at its own level.  Given the new surface temperature u the rows of nodes
    1..M are linear, so T_1' = a + s u (a, s from two solves with the surface
    held at 0 and at 1), and the condition becomes one quartic per column,

      f(u) = emiss sigma u^4 + c u - b = 0,   c = k (1 - s) / z_1,  b = Qabs' + k a / z_1.

    f is increasing and convex for u > 0 (c > 0): a Newton step from any point
    lands at or above the root, and from above the root Newton's method
    descends to it without overshoot.  The first step is taken from the old
    surface temperature T_0^n and capped by the smaller of two bounds above the
    root, (b / emiss sigma)^(1/4) and b / c (the cap matters after a jump in
    Qabs, when a step from far below the root would overshoot far above it);
    ``newton`` more steps follow.  Then the column is solved with the surface
    at u.
    ``qabs_old`` is not needed by this form (it is carried by T_0^n) and is
    accepted for a common signature."""
    N, n = T.shape
    V = cell_volumes(z)
    V[0] = 0.0
    g = k / np.diff(z)
    cap = rhoc * V / dt
    emiss = np.broadcast_to(np.asarray(emiss, dtype=np.float64), (N,))
    Hb = np.broadcast_to(np.asarray(H_bottom, dtype=np.float64), (N,))
    LT = np.zeros_like(T)
    LT[:, 1:] += g * (T[:, :-1] - T[:, 1:])
    LT[:, :-1] += g * (T[:, 1:] - T[:, :-1])
    lower = np.zeros((N, n))
    upper = np.zeros((N, n))
    diag = np.broadcast_to(cap, (N, n)).copy()
    lower[:, 1:] = -0.5 * g
    diag[:, 1:] += 0.5 * g
    diag[:, 1:-1] += 0.5 * g[1:]
    upper[:, 1:-1] = -0.5 * g[1:]
    rhs = cap * T
    rhs[:, 1:] += 0.5 * LT[:, 1:]
    rhs[:, -1] += Hb
    # the surface row holds T_0' = u
    diag[:, 0] = 1.0
    upper[:, 0] = 0.0

    def with_surface(u):
        r = rhs.copy()
        r[:, 0] = u
        return thomas(lower, diag, upper, r)

    a = with_surface(np.zeros(N))[:, 1]
    s = with_surface(np.ones(N))[:, 1] - a
    es = emiss * SIGMA_SB
    c = g[0] * (1.0 - s)
    b = qabs_new + g[0] * a
    bound = np.minimum((np.maximum(b, 0.0) / es) ** 0.25, np.maximum(b, 0.0) / c)
    t0 = T[:, 0]
    u = np.minimum(t0 - (es * t0 ** 4 + c * t0 - b) / (4.0 * es * t0 ** 3 + c), bound)
    for _ in range(newton):
        u = u - (es * u ** 4 + c * u - b) / (4.0 * es * u ** 3 + c)
    return with_surface(u)


def column_energy(T: np.ndarray, z: np.ndarray, rhoc: float) -> np.ndarray:
    """Heat content per unit area of each column, rhoc sum_j V_j T_j (J m^-2)."""
    return rhoc * (T * cell_volumes(z)).sum(axis=1)


def simulate(matvec, qdir_steps: np.ndarray, albedo, emiss, T_init: np.ndarray, z: np.ndarray, k: float,
             rhoc: float, dt: float, H_bottom=0.0, H0=0.0, step=cn_step):
    """Algorithm 6.  qdir_steps: (n_steps + 1, N) direct insolation at the
    time levels 0..n_steps; T_init: (N, M+1) initial column temperatures.

    Level 0: Qabs = (1 - albedo) Qdir + H0, Qrefl = QIR = 0, Qrad = Qabs.
    Each step:  Qrefl' = F diag(albedo) (Qdir' + Qrefl)
                QIR'   = F (Qrad + (1 - emiss) QIR)
                Qabs'  = (1 - albedo) (Qdir' + Qrefl') + emiss QIR'
    then every column steps with Qabs and Qabs' (``step``: ``cn_step``, or
    ``cn_step_balanced``) and
    Qrad' = emiss sigma T_0'^4.  Returns the final state and the surface
    temperature of every level, shape (n_steps + 1, N)."""
    N = qdir_steps.shape[1]
    a = np.broadcast_to(np.asarray(albedo, dtype=np.float64), (N,))
    e = np.broadcast_to(np.asarray(emiss, dtype=np.float64), (N,))
    qabs = (1.0 - a) * qdir_steps[0] + H0
    qrefl = np.zeros(N)
    qir = np.zeros(N)
    qrad = qabs.copy()
    T = np.array(T_init, dtype=np.float64, copy=True)
    surface = [T[:, 0].copy()]
    for n in range(qdir_steps.shape[0] - 1):
        qdir = qdir_steps[n + 1]
        qrefl_new = matvec(a * (qdir + qrefl))
        qir_new = matvec(qrad + (1.0 - e) * qir)
        qabs_new = (1.0 - a) * (qdir + qrefl_new) + e * qir_new
        T = step(T, qabs, qabs_new, dt, z, k, rhoc, e, H_bottom)
        qrad = e * SIGMA_SB * T[:, 0] ** 4
        qrefl, qir, qabs = qrefl_new, qir_new, qabs_new
        surface.append(T[:, 0].copy())
    return dict(T=T, Q_abs=qabs, Q_refl=qrefl, Q_ir=qir, Q_rad=qrad, surface=np.array(surface))
