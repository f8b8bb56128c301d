"""GPU parity of the time stepper (Algorithm 6 with a Crank-Nicolson column
under every facet, section 5.2) against the FP64 CPU reference, through the
C-ABI of include/rad_timestep.h.

The FP64 matrix is built at tol 1e-10 so that F-hat equals the exact F of
the reference to about 1e-10; the remaining differences are rounding (the GPU
eliminates each column from the bottom up, the reference from the top down).
Tolerances: FP64 matrix 1e-9 relative on temperatures and fluxes; FP32
matrix at tol 1e-6, 2e-5 (fluxes carry FP32 products, columns stay FP64).
"""
import numpy as np
import pytest

from oracle import reference as ref
from oracle import timestep as ots
from synth import CapSpec, cap_mesh

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
ALBEDO, EMISS, K, RHOC, DT, HB, H0 = 0.12, 0.95, 0.01, 1.2e6, 2000.0, 0.5, 0.3


@pytest.fixture(scope="module")
def bowl():
    verts, faces = cap_mesh(CapSpec(h=120.0, seed=3))
    fac = ref.Facets(verts, faces)
    F = ref.view_factor_matrix(fac)
    return verts, faces, fac, F


def _levels(fac, R, n, seed):
    """Direct insolation of R scenarios at levels 0..n: the sun of scenario r
    circles in azimuth (one turn per 96 levels) at its own elevation."""
    rng = np.random.default_rng(seed)
    el = np.deg2rad(rng.uniform(5.0, 30.0, R))
    az0 = rng.uniform(0.0, 2.0 * np.pi, R)
    Q = np.empty((n + 1, R, fac.N))
    for lvl in range(n + 1):
        az = az0 + 2.0 * np.pi * lvl / 96.0
        suns = np.column_stack([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)])
        Q[lvl] = ref.insolation(fac, suns, S=1365.0).T
    return Q


def _initial(fac, R, z, seed):
    rng = np.random.default_rng(seed)
    base = rng.uniform(150.0, 250.0, (R, fac.N))
    return base[None, :, :] + 20.0 * np.exp(-z / 0.1)[:, None, None] * rng.uniform(-1.0, 1.0, (len(z), R, fac.N))


def _oracle(F, Q, T0, z, dt=DT, step=ots.cn_step):
    R = Q.shape[1]
    outs = []
    for r in range(R):
        outs.append(ots.simulate(lambda x: F @ x, Q[:, r, :], ALBEDO, EMISS, T0[:, r, :].T, z, K, RHOC, dt,
                                 H_bottom=HB, H0=H0, step=step))
    return outs


def _stepper(verts, faces, R, z, storage="f64", tol=1e-10, dt=DT, **kw):
    from paper_2209_07632_amd import HMatrix
    from paper_2209_07632_amd.timestep import TimeStepper
    print(f"[build] N={faces.shape[0]} R={R} storage={storage} tol={tol} dt={dt} {kw}", flush=True)
    H = HMatrix(verts, faces, tol=tol, storage=storage, max_rhs=2 * R)
    return H, TimeStepper(H, z, K, RHOC, dt, ALBEDO, EMISS, bottom_flux=HB, R=R, **kw)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


# 2R = 6: column-major products; 2R = 24: matrix cores.  Up to 32 layers the
# column kernel keeps the column in registers (instances for 16, 24, 32
# layers); 40 layers take the LDS form.
@pytest.mark.parametrize("R,layers", [(3, 20), (12, 20), (3, 12), (4, 32), (5, 40)])
def test_stepper_matches_reference(bowl, R, layers):
    verts, faces, fac, F = bowl
    z = ots.layer_depths(layers, 0.5, 1.12)
    n = 30
    Q = _levels(fac, R, n, seed=R)
    T0 = _initial(fac, R, z, seed=R + 1)
    H, S = _stepper(verts, faces, R, z)
    S.init(torch.from_numpy(T0).to(DEV), torch.from_numpy(Q[0]).to(DEV), H0=H0)
    assert S.level == 0
    S.step(torch.from_numpy(Q[1:]).to(DEV).contiguous())
    assert S.level == n
    want = _oracle(F, Q, T0, z)
    T = S.read("T").cpu().numpy()
    for r in range(R):
        assert _rel(T[:, r, :].T, want[r]["T"]) < 1e-9
        for name in ("Q_abs", "Q_refl", "Q_ir", "Q_rad"):
            got = S.read(name).cpu().numpy()[r]
            assert _rel(got, want[r][name]) < 1e-9, (r, name)


# 40 layers to 1 m with a ratio of 1.05 (top layer 8 mm): with the 0.5 m,
# 1.12 grid of the other cases 40 layers make the top layer 0.65 mm, and at
# 0.3-day steps three Newton repeats from the old surface temperature then
# diverge in the reference itself
@pytest.mark.parametrize("R,layers,depth,ratio", [(3, 20, 0.5, 1.12), (8, 20, 0.5, 1.12), (3, 40, 1.0, 1.05)])
@pytest.mark.parametrize("dt_days", [0.1, 0.3])
def test_balanced_surface_matches_reference(bowl, dt_days, R, layers, depth, ratio):
    """The balanced surface reading (radiation boundary condition at the new
    level, Newton on the surface row) at the long steps of a lunation, against
    the reference's second reading of the column step."""
    import functools
    verts, faces, fac, F = bowl
    dt = dt_days * 86400.0
    z = ots.layer_depths(layers, depth, ratio)
    n = 24
    Q = _levels(fac, R, n, seed=30 + R)
    T0 = _initial(fac, R, z, seed=31 + R)
    H, S = _stepper(verts, faces, R, z, dt=dt, surface="balanced", newton=3)
    S.init(torch.from_numpy(T0).to(DEV), torch.from_numpy(Q[0]).to(DEV), H0=H0)
    S.step(torch.from_numpy(Q[1:]).to(DEV).contiguous())
    want = _oracle(F, Q, T0, z, dt=dt, step=functools.partial(ots.cn_step_balanced, newton=3))
    T = S.read("T").cpu().numpy()
    for r in range(R):
        err = _rel(T[:, r, :].T, want[r]["T"])
        assert err < 1e-9, (r, err)
        for name in ("Q_abs", "Q_ir", "Q_rad"):
            assert _rel(S.read(name).cpu().numpy()[r], want[r][name]) < 1e-9, (r, name)


def test_internal_layout_equals_caller_order(bowl):
    """The same run with every block in the library's internal layout (tree
    order, scenarios contiguous, as rad_insolation writes them) gives the
    same state bit for bit as with blocks in the caller's facet order."""
    from paper_2209_07632_amd.rad import ldr_of
    verts, faces, fac, F = bowl
    R, n = 12, 10
    z = ots.layer_depths(20, 0.5, 1.12)
    Q = _levels(fac, R, n, seed=77)
    T0 = _initial(fac, R, z, seed=78)
    H, S = _stepper(verts, faces, R, z, dt=0.1 * 86400.0, surface="balanced", newton=3)
    S.init(torch.from_numpy(T0).to(DEV), torch.from_numpy(Q[0]).to(DEV), H0=H0)
    S.step(torch.from_numpy(Q[1:]).to(DEV).contiguous())
    want = S.read("T").cpu().numpy()
    perm = H.perm()
    ld = ldr_of(R)

    def internal(blocks):                      # (..., R, N) caller order -> (..., N, ld)
        out = np.zeros(blocks.shape[:-2] + (fac.N, ld))
        out[..., :R] = np.swapaxes(blocks[..., perm], -1, -2)
        return torch.from_numpy(out).to(DEV).contiguous()

    from paper_2209_07632_amd.timestep import TimeStepper
    S2 = TimeStepper(H, z, K, RHOC, 0.1 * 86400.0, ALBEDO, EMISS, bottom_flux=HB, R=R, surface="balanced", newton=3)
    S2.init(internal(T0), internal(Q[0]), H0=H0, order="tree_rmajor")
    S2.step(internal(Q[1:]), order="tree_rmajor")
    got = S2.read("T", order="tree_rmajor").cpu().numpy()[..., :R]
    back = np.empty_like(want)
    back[..., perm] = np.swapaxes(got, -1, -2)
    np.testing.assert_array_equal(back, want)
    for name in ("Q_abs", "Q_rad"):
        g = S2.read(name, order="tree_rmajor").cpu().numpy()[:, :R]
        w = S.read(name).cpu().numpy()
        np.testing.assert_array_equal(g.T, w[:, perm])


def test_level_zero_state(bowl):
    verts, faces, fac, F = bowl
    R = 2
    z = ots.layer_depths(6, 0.2)
    Q = _levels(fac, R, 0, seed=7)
    T0 = _initial(fac, R, z, seed=8)
    H, S = _stepper(verts, faces, R, z)
    S.init(torch.from_numpy(T0).to(DEV), torch.from_numpy(Q[0]).to(DEV), H0=H0)
    assert np.array_equal(S.read("T").cpu().numpy(), T0)
    qa = (1.0 - ALBEDO) * Q[0] + H0
    assert _rel(S.read("Q_abs").cpu().numpy(), qa) < 1e-15
    assert _rel(S.read("Q_rad").cpu().numpy(), qa) < 1e-15
    assert not S.read("Q_refl").cpu().numpy().any() and not S.read("Q_ir").cpu().numpy().any()


def test_split_runs_equal_one_run(bowl):
    """Steps enqueued in several calls give the result of one call (the
    operand written by the last column step is rebuilt from the state at the
    start of the next call by the same arithmetic)."""
    verts, faces, fac, F = bowl
    R = 8
    z = ots.layer_depths(12, 0.3, 1.1)
    n = 12
    Q = torch.from_numpy(_levels(fac, R, n, seed=11)).to(DEV)
    T0 = torch.from_numpy(_initial(fac, R, z, seed=12)).to(DEV)
    H, S = _stepper(verts, faces, R, z)
    S.init(T0, Q[0], H0=H0)
    S.step(Q[1:].contiguous())
    one = [S.read(f) for f in ("T", "Q_abs", "Q_refl", "Q_ir", "Q_rad")]
    S.init(T0, Q[0], H0=H0)
    S.step(Q[1:6].contiguous())
    S.step(Q[6:7].contiguous())
    S.step(Q[7:].contiguous())
    two = [S.read(f) for f in ("T", "Q_abs", "Q_refl", "Q_ir", "Q_rad")]
    for a, b in zip(one, two):
        assert float((a - b).abs().max() / b.abs().max()) < 1e-13


def test_fp32_matrix(bowl):
    verts, faces, fac, F = bowl
    R = 9
    z = ots.layer_depths(20, 0.5, 1.12)
    n = 20
    Q = _levels(fac, R, n, seed=21)
    T0 = _initial(fac, R, z, seed=22)
    H, S = _stepper(verts, faces, R, z, storage="f32", tol=1e-6)
    S.init(torch.from_numpy(T0).to(DEV), torch.from_numpy(Q[0]).to(DEV, torch.float32), H0=H0)
    S.step(torch.from_numpy(Q[1:]).to(DEV, torch.float32).contiguous())
    want = _oracle(F, Q, T0, z)
    T = S.read("T").cpu().numpy()
    for r in range(R):
        assert _rel(T[:, r, :].T, want[r]["T"]) < 2e-5
        assert _rel(S.read("Q_ir").cpu().numpy()[r], want[r]["Q_ir"]) < 2e-5


def test_rejects_bad_arguments(bowl):
    from paper_2209_07632_amd import HMatrix
    from paper_2209_07632_amd.rad import RadError
    from paper_2209_07632_amd.timestep import TimeStepper
    verts, faces, fac, F = bowl
    H = HMatrix(verts, faces, tol=1e-3, storage="f64", max_rhs=4)
    z = ots.layer_depths(5, 0.1)
    with pytest.raises(RadError, match="max_rhs"):
        TimeStepper(H, z, K, RHOC, DT, ALBEDO, EMISS, R=3)
    with pytest.raises(RadError, match="strictly increasing"):
        TimeStepper(H, z[::-1] - z[-1], K, RHOC, DT, ALBEDO, EMISS, R=2)
    with pytest.raises(RadError, match="emissivity"):
        TimeStepper(H, z, K, RHOC, DT, ALBEDO, 0.0, R=2)
    with pytest.raises(RadError, match="newton"):
        TimeStepper(H, z, K, RHOC, DT, ALBEDO, EMISS, R=2, surface="balanced", newton=-1)
    S = TimeStepper(H, z, K, RHOC, DT, ALBEDO, EMISS, R=2)
    with pytest.raises(RadError, match="rad_ts_init"):
        S.step(torch.zeros((1, 2, fac.N), dtype=torch.float64, device=DEV))


def test_lunation_in_internal_layout_r64():
    """The benchmark's shape on a small cap: 64 scenarios (a 128-column
    operand), insolation written by the library straight into its internal
    layout, 20 layers to 1 m, one lunation of 0.3-day steps with the balanced
    surface, FP32 matrix at tol 1e-6.  Surface temperatures of three
    scenarios equal the FP64 reference's (fed the same direct insolation),
    and stay within a few kelvin of radiative equilibrium under a single sun."""
    from paper_2209_07632_amd import HMatrix
    from paper_2209_07632_amd.rad import ldr_of
    from paper_2209_07632_amd.timestep import TimeStepper
    verts, faces = cap_mesh(CapSpec(h=120.0, seed=3))
    fac = ref.Facets(verts, faces)
    F = ref.view_factor_matrix(fac)
    R, M, n = 64, 20, int(round(29.53 / 0.3))
    dt, k, albedo, emiss = 0.3 * 86400.0, 0.0015, 0.12, 0.95
    w = 1.12 ** np.arange(M)
    z = np.concatenate([[0.0], np.cumsum(w / w.sum())])
    H = HMatrix(verts, faces, tol=1e-6, storage="f32", max_rhs=2 * R)
    ld = ldr_of(R)
    rng = np.random.default_rng(11)
    el = np.deg2rad(rng.uniform(5.0, 30.0, R))
    az0 = rng.uniform(0.0, 2.0 * np.pi, R)
    Q = torch.zeros((n + 1, fac.N, ld), dtype=torch.float32, device=DEV)
    for lvl in range(n + 1):
        az = az0 + 2.0 * np.pi * lvl / n
        suns = np.column_stack([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)])
        H.insolation(suns, flux=1365.0, order="tree_rmajor", out=Q[lvl])
    S = TimeStepper(H, z, k, RHOC, dt, albedo, emiss, bottom_flux=0.0, R=R, surface="balanced", newton=3)
    T0 = torch.full((M + 1, fac.N, ld), 250.0, dtype=torch.float64, device=DEV)
    S.init(T0, Q[0], order="tree_rmajor")
    S.step(Q[1:], order="tree_rmajor")
    Ts = S.read("T", order="tree_rmajor")[0][:, :R].cpu().numpy()      # (N tree order, R)
    perm = H.perm()
    Qc = Q[:, :, :R].double().cpu().numpy()                            # (n+1, N tree, R)
    flat = ((1.0 - albedo) * 1365.0 / (emiss * 5.670374419e-8)) ** 0.25
    print(f"GPU surface T range {Ts.min():.2f} .. {Ts.max():.2f} K; flat equilibrium {flat:.2f} K", flush=True)
    assert Ts.max() < flat + 15.0
    for r in (0, 31, 63):
        qd = np.empty((n + 1, fac.N))
        qd[:, perm] = Qc[:, :, r]
        out = ots.simulate(lambda x: F @ x, qd, albedo, emiss, np.full((fac.N, M + 1), 250.0), z, k, RHOC, dt,
                           step=lambda T, qo, qn, d, zz, kk, rc, em, hb: ots.cn_step_balanced(
                               T, qo, qn, d, zz, kk, rc, em, hb, newton=3))
        want = out["T"][:, 0][perm]
        assert _rel(Ts[:, r], want) < 2e-5, (r, _rel(Ts[:, r], want))
