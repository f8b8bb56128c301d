"""Pins of the time-stepping reference (Algorithm 6 with a Crank-Nicolson
column under every facet, section 5.2) against closed forms, invariants and
brute force.  CPU only.

A slip in the column scheme (a wrong end volume, a missing half in the
Crank-Nicolson weights, an emission linearised about the wrong level, a flux
with the wrong sign) or in the flux recursions of Algorithm 6 (a lag on the
wrong term, a dropped albedo or emissivity factor) fails at least one test.
"""
import numpy as np
import pytest

from oracle import reference as ref
from oracle import timestep as ts
from synth import CapSpec, cap_mesh


# ------------------------------------------------------------ tridiagonal solve
def test_thomas_matches_dense_solve():
    rng = np.random.default_rng(0)
    C, n = 7, 13
    lo = rng.uniform(-1.0, 0.0, (C, n))
    up = rng.uniform(-1.0, 0.0, (C, n))
    dg = 2.5 + rng.uniform(0.0, 1.0, (C, n))
    b = rng.standard_normal((C, n))
    x = ts.thomas(lo, dg, up, b)
    for c in range(C):
        A = np.diag(dg[c]) + np.diag(lo[c, 1:], -1) + np.diag(up[c, :-1], 1)
        assert np.allclose(A @ x[c], b[c], rtol=0, atol=1e-13)


# ------------------------------------------------------------ column scheme
@pytest.mark.parametrize("m", [1, 3, 7])
def test_insulated_cosine_mode_decays_by_cn_factor(m):
    """With no emission, no absorbed flux and no bottom flux the uniform column
    is the reflecting second difference, whose eigenvectors are cos(pi m j / M)
    with eigenvalue 2 kappa (1 - cos(pi m / M)) / dz^2; Crank-Nicolson scales
    such a mode by (1 - lam dt / 2) / (1 + lam dt / 2) each step."""
    M, L, k, rhoc, dt = 20, 0.5, 0.7, 2.0e3, 30.0
    z = ts.layer_depths(M, L)
    kappa, dz = k / rhoc, L / M
    mode = np.cos(np.pi * m * np.arange(M + 1) / M)
    T = 100.0 + mode[None, :]
    lam = 2.0 * kappa * (1.0 - np.cos(np.pi * m / M)) / dz ** 2
    g = (1.0 - 0.5 * lam * dt) / (1.0 + 0.5 * lam * dt)
    zero = np.zeros(1)
    for n in range(1, 6):
        T = ts.cn_step(T, zero, zero, dt, z, k, rhoc, 0.0, 0.0)
        assert np.max(np.abs(T[0] - (100.0 + g ** n * mode))) < 1e-12


def test_cosine_mode_follows_heat_equation():
    """Fine grid and short steps: the slowest insulated mode decays as
    exp(-kappa pi^2 t / L^2), the solution of the heat equation of section 2."""
    M, L, k, rhoc = 200, 1.0, 1.3, 1.0e3
    kappa = k / rhoc
    z = ts.layer_depths(M, L)
    t_end = 0.1 * L * L / kappa
    steps = 400
    dt = t_end / steps
    T = np.cos(np.pi * z / L)[None, :]
    zero = np.zeros(1)
    for _ in range(steps):
        T = ts.cn_step(T, zero, zero, dt, z, k, rhoc, 0.0, 0.0)
    exact = np.exp(-kappa * np.pi ** 2 * t_end / L ** 2) * np.cos(np.pi * z / L)
    assert np.max(np.abs(T[0] - exact)) < 2e-5


def _linear_profile(z, qabs, H, k, emiss):
    """Steady column under constant absorbed flux and bottom flux H (upward):
    T(z) = T_s + H z / k with emiss sigma T_s^4 = qabs + H."""
    Ts = ((qabs + H) / (emiss * ref.SIGMA_SB)) ** 0.25
    return Ts[:, None] + H * z[None, :] / k


def test_steady_linear_profile_is_fixed_point():
    """On a graded grid the steady conduction profile with the radiative top is
    returned unchanged by a step (the flux-conservative scheme is exact for it)."""
    z = ts.layer_depths(25, 2.5, 1.15)
    k, rhoc, emiss, H = 0.005, 1.1e6, 0.95, 0.03
    qabs = np.array([0.0, 2.0, 45.0, 400.0])
    T = _linear_profile(z, qabs, H, k, emiss)
    T1 = ts.cn_step(T, qabs, qabs, 3600.0, z, k, rhoc, emiss, H)
    assert np.max(np.abs(T1 - T) / T) < 1e-12


def test_relaxes_to_steady_linear_profile():
    """From a uniform start under constant flux the column settles on the same
    profile (the sign of the emission and of both boundary fluxes matter)."""
    z = ts.layer_depths(8, 0.1, 1.15)
    k, rhoc, emiss, H = 0.02, 1.0e5, 0.9, 0.5
    qabs = np.array([20.0, 100.0, 300.0])
    T = np.full((3, 9), 200.0)
    for _ in range(900):
        T = ts.cn_step(T, qabs, qabs, 1000.0, z, k, rhoc, emiss, H)
    exact = _linear_profile(z, qabs, H, k, emiss)
    assert np.max(np.abs(T - exact) / exact) < 1e-11


def test_energy_budget_without_emission():
    """Flux-conservative: the heat content changes by exactly dt times the
    time-averaged absorbed flux plus the bottom flux."""
    rng = np.random.default_rng(3)
    z = ts.layer_depths(30, 1.0, 1.08)
    k, rhoc, dt = 0.04, 9.0e5, 7200.0
    T = rng.uniform(80.0, 300.0, (5, 31))
    qa_old = rng.uniform(0.0, 400.0, 5)
    qa_new = rng.uniform(0.0, 400.0, 5)
    H = rng.uniform(-0.1, 0.1, 5)
    E0 = ts.column_energy(T, z, rhoc)
    T1 = ts.cn_step(T, qa_old, qa_new, dt, z, k, rhoc, 0.0, H)
    E1 = ts.column_energy(T1, z, rhoc)
    budget = dt * (0.5 * (qa_old + qa_new) + H)
    assert np.max(np.abs((E1 - E0) - budget) / np.abs(budget)) < 1e-9


def _radiating_day(dt, M=12, day=86400.0, growth=1.1, step=ts.cn_step):
    """Column temperatures after one day of a sinusoidally varying absorbed flux."""
    z = ts.layer_depths(M, 0.3, growth)
    k, rhoc, emiss = 0.01, 1.2e6, 0.95
    n = int(round(day / dt))
    t = np.arange(n + 1) * dt
    qa = 400.0 * (1.0 + 0.5 * np.sin(2.0 * np.pi * t / day))
    T = np.full((1, M + 1), (qa[0] / (emiss * ref.SIGMA_SB)) ** 0.25)
    for i in range(n):
        T = step(T, qa[i:i + 1], qa[i + 1:i + 2], dt, z, k, rhoc, emiss, 0.0)
    return T[0]


def test_second_order_in_time_with_emission():
    """Crank-Nicolson with the emission averaged over both levels is second
    order in dt: halving the step quarters the error (an emission taken at
    one level only, or only the new absorbed flux, would halve it)."""
    fine = _radiating_day(86400.0 / 4096)
    errs = [np.max(np.abs(_radiating_day(86400.0 / n) - fine)) for n in (64, 128, 256)]
    ratios = [errs[0] / errs[1], errs[1] / errs[2]]
    assert all(3.6 < r < 4.4 for r in ratios), ratios


# ------------------------------------------------------------ Algorithm 6
@pytest.fixture(scope="module")
def bowl():
    v, f = cap_mesh(CapSpec(h=120.0, seed=3))
    fac = ref.Facets(v, f)
    F = ref.view_factor_matrix(fac)
    e = np.deg2rad(15.0)
    sun = np.array([[np.cos(e), 0.0, np.sin(e)]])
    Q = ref.insolation(fac, sun, S=1365.0)[:, 0]
    return F, Q


@pytest.mark.parametrize("n_steps", [1, 2, 5])
def test_reflected_flux_is_neumann_partial_sum(bowl, n_steps):
    """Under a constant sun Algorithm 6 gives Q_refl after n steps as the first
    n terms of the scattering series sum_k (F diag(albedo))^k Q_dir."""
    F, Q = bowl
    N = F.shape[0]
    albedo = np.linspace(0.1, 0.4, N)
    z = ts.layer_depths(6, 0.1)
    qd = np.tile(Q, (n_steps + 1, 1))
    out = ts.simulate(lambda x: F @ x, qd, albedo, 0.95, np.full((N, 7), 200.0), z, 0.02, 1.0e5, 600.0)
    FA = F * albedo[None, :]
    expect = np.zeros(N)
    term = Q.copy()
    for _ in range(n_steps):
        term = FA @ term
        expect += term
    assert np.max(np.abs(out["Q_refl"] - expect)) < 1e-12 * np.max(np.abs(expect))


def test_no_exchange_gives_independent_columns():
    """F = 0 (a flat plane): terrain fluxes stay zero and every facet evolves as a
    lone column driven by (1 - albedo) Q_dir."""
    rng = np.random.default_rng(5)
    N, steps = 9, 40
    z = ts.layer_depths(10, 0.5, 1.1)
    k, rhoc, dt, emiss, H = 0.01, 1.0e6, 1800.0, 0.95, 0.005
    albedo = rng.uniform(0.05, 0.4, N)
    qd = rng.uniform(0.0, 600.0, (steps + 1, N))
    T0 = rng.uniform(150.0, 250.0, (N, 11))
    out = ts.simulate(lambda x: 0.0 * x, qd, albedo, emiss, T0, z, k, rhoc, dt, H_bottom=H)
    assert not out["Q_refl"].any() and not out["Q_ir"].any()
    for i in range(N):
        T = T0[i:i + 1]
        qa = (1.0 - albedo[i]) * qd[:, i]
        for n in range(steps):
            T = ts.cn_step(T, qa[n:n + 1], qa[n + 1:n + 2], dt, z, k, rhoc, emiss, H)
        assert np.array_equal(T[0], out["T"][i])


@pytest.mark.parametrize("step", [ts.cn_step, ts.cn_step_balanced])
@pytest.mark.parametrize("H", [0.0, 0.5])
def test_constant_sun_reaches_two_band_equilibrium(bowl, H, step):
    """Held under one sun, the lagged one-multiply-per-step recursions settle on
    the solution of the two equilibrium systems of section 5.1 (eqs. Qvis and
    QIR, solved here by Jacobi to 1e-13), with the surface balance
    emiss sigma T^4 = (1 - albedo) Q_vis + emiss Q_IR + H and the linear
    conduction profile below."""
    F, Q = bowl
    N = F.shape[0]
    albedo, emiss = 0.3, 0.95
    z = ts.layer_depths(8, 0.1, 1.15)
    k, rhoc, dt, steps = 0.02, 1.0e5, 1000.0, 900
    qd = np.tile(Q, (steps + 1, 1))
    out = ts.simulate(lambda x: F @ x, qd, albedo, emiss, np.full((N, 9), 250.0), z, k, rhoc, dt,
                      H_bottom=H, step=step)
    eq = ref.equilibrium_temperature(lambda X: F @ X, Q[:, None], albedo, emiss, H=H)
    Qvis, Qir = eq["Q_vis"][:, 0], eq["Q_ir"][:, 0]
    Ts = (((1.0 - albedo) * Qvis + emiss * Qir + H) / (emiss * ref.SIGMA_SB)) ** 0.25
    assert np.max(np.abs(out["Q_refl"] - eq["Q_refl"][:, 0])) < 1e-10 * Q.max()
    assert np.max(np.abs(out["Q_ir"] - Qir)) < 1e-9 * Qir.max()
    assert np.max(np.abs(out["surface"][-1] - Ts) / Ts) < 1e-11
    assert np.max(np.abs(out["T"] - (Ts[:, None] + H * z[None, :] / k)) / Ts[:, None]) < 1e-11
    if H == 0.0:
        assert np.max(np.abs(Ts - eq["T"][:, 0]) / Ts) < 1e-12


# ------------------------------------------------------------ surface held by its balance
def test_balanced_steady_profile_is_fixed_point():
    z = ts.layer_depths(25, 2.5, 1.15)
    k, rhoc, emiss, H = 0.005, 1.1e6, 0.95, 0.03
    qabs = np.array([0.0, 2.0, 45.0, 400.0])
    T = _linear_profile(z, qabs, H, k, emiss)
    T1 = ts.cn_step_balanced(T, qabs, qabs, 3600.0, z, k, rhoc, emiss, H)
    assert np.max(np.abs(T1 - T) / T) < 1e-12


def test_balanced_surface_meets_radiation_condition():
    """After the step the surface satisfies Qabs' + k (T_1 - T_0) / z_1 =
    emiss sigma T_0^4 (the radiation boundary condition of section 2) to
    Newton's convergence, from any start."""
    rng = np.random.default_rng(0)
    z = ts.layer_depths(25, 2.5, 1.15)
    k, emiss = 0.005, 0.95
    T = rng.uniform(150.0, 300.0, (4, 26))
    qn = np.array([0.0, 10.0, 200.0, 600.0])
    x = ts.cn_step_balanced(T, qn, qn, 3600.0, z, k, 1.1e6, emiss, 0.03, newton=8)
    emit = emiss * ref.SIGMA_SB * x[:, 0] ** 4
    res = qn + k / z[1] * (x[:, 1] - x[:, 0]) - emit
    assert np.max(np.abs(res)) <= 1e-10 * np.max(emit)


def test_balanced_surface_after_a_jump_in_sunlight():
    """Columns at 150 K stepped 0.3 day into shadow and into sunlight of 750
    and 1,200 W m^-2, with 20 layers to 1 m of low-conductivity regolith:
    with many repeats the surface meets the radiation condition of section 2
    to rounding; with the default three it is within 1e-6 (relative) of that
    solution;
    and the sunlit surfaces stay below the temperature at which emission alone
    would carry Qabs away (conduction only takes heat down into the colder
    column).  Newton's method from the old surface temperature alone
    overshoots to about 1,000 K here and is still some 150 K high after three
    repeats."""
    M = 20
    w = 1.12 ** np.arange(M)
    z = np.concatenate([[0.0], np.cumsum(w / w.sum())])
    k, rhoc, emiss = 0.0015, 1.2e6, 0.95
    T = np.full((3, M + 1), 150.0)
    qn = np.array([0.0, 750.0, 1200.0])
    conv = ts.cn_step_balanced(T, qn, qn, 0.3 * 86400.0, z, k, rhoc, emiss, 0.0, newton=12)
    emit = emiss * ref.SIGMA_SB * conv[:, 0] ** 4
    res = qn + k / z[1] * (conv[:, 1] - conv[:, 0]) - emit
    assert np.max(np.abs(res)) <= 1e-12 * np.max(emit)
    x = ts.cn_step_balanced(T, qn, qn, 0.3 * 86400.0, z, k, rhoc, emiss, 0.0)
    assert np.max(np.abs(x[:, 0] - conv[:, 0]) / conv[:, 0]) < 1e-6
    assert np.all(x[1:, 0] < (qn[1:] / (emiss * ref.SIGMA_SB)) ** 0.25)


def test_balanced_second_order_in_time():
    fine = _radiating_day(86400.0 / 4096, step=ts.cn_step_balanced)
    errs = [np.max(np.abs(_radiating_day(86400.0 / n, step=ts.cn_step_balanced) - fine)) for n in (64, 128, 256)]
    ratios = [errs[0] / errs[1], errs[1] / errs[2]]
    assert all(3.6 < r < 4.4 for r in ratios), ratios


def test_surface_readings_agree_as_the_top_layer_thins():
    """The half-layer surface volume and the surface without heat capacity
    discretise the same heat equation with the same boundary condition: their
    surface temperatures after a day differ by an amount that halves with the
    layer thickness."""
    diffs = []
    for M, growth in ((10, 1.2), (20, 1.095), (40, 1.0465)):
        a = _radiating_day(86400.0 / 1024, M=M, growth=growth)
        b = _radiating_day(86400.0 / 1024, M=M, growth=growth, step=ts.cn_step_balanced)
        diffs.append(abs(a[0] - b[0]))
    assert all(1.8 < diffs[i] / diffs[i + 1] < 2.4 for i in range(2)), diffs
