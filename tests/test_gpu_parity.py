"""GPU parity: librad's H-matvec and solve against the FP64 CPU reference.

Tolerances: the compressed product may differ from the exact F X by the
compression tolerance eps (truncation at sigma_{q+1} < eps sigma_1 per
block); FP64 and FP32 paths must stay within eps + 1e-6 relative L2.
"""
import numpy as np
import pytest

from oracle import reference as ref
from synth import CAP_SMALL, CapSpec, cap_mesh, sun_directions

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def cap():
    verts, faces = cap_mesh(CAP_SMALL)
    fac = ref.Facets(verts, faces)
    F = ref.view_factor_matrix(fac)
    return verts, faces, fac, F


def _hm(verts, faces, **kw):
    from paper_2209_07632_amd import HMatrix
    print(f"[build] N={faces.shape[0]} {kw}", flush=True)
    return HMatrix(verts, faces, **kw)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("tol", [1e-2, 1e-3, 1e-4, 1e-6])
def test_matvec_within_tol(cap, storage, tol):
    verts, faces, fac, F = cap
    H = _hm(verts, faces, tol=tol, storage=storage, max_rhs=5)
    X = np.random.default_rng(1).random((fac.N, 5))
    dt = torch.float64 if storage == "f64" else torch.float32
    Y = H.matvec(torch.from_numpy(X).to(DEV, dt)).double().cpu().numpy()
    err = _rel(Y, F @ X)
    print(f"tol={tol} {storage} err={err:.3e} stats={H.stats()}")
    assert err <= tol + 1e-6


def test_matvec_tight_tol_is_exact(cap):
    verts, faces, fac, F = cap
    H = _hm(verts, faces, tol=1e-10, storage="f64")
    X = np.random.default_rng(2).standard_normal(fac.N)
    Y = H.matvec(torch.from_numpy(X).to(DEV)).cpu().numpy()
    assert _rel(Y, F @ X) < 1e-9
    st = H.stats()
    assert st["n_lowrank"] > 0


@pytest.mark.parametrize("nearfield", ["dense", "csr"])
def test_nearfield_forms(cap, nearfield):
    verts, faces, fac, F = cap
    H = _hm(verts, faces, tol=1e-5, storage="f64", nearfield=nearfield, max_rhs=2)
    st = H.stats()
    if nearfield == "csr":
        assert st["n_dense"] == 0 and st["n_csr"] > 0
    else:
        assert st["n_csr"] == 0 and st["n_dense"] > 0
    X = np.random.default_rng(3).random((fac.N, 2))
    Y = H.matvec(torch.from_numpy(X).to(DEV)).cpu().numpy()
    assert _rel(Y, F @ X) <= 1e-5 + 1e-6


def test_orders_and_leading_dimension(cap):
    verts, faces, fac, F = cap
    H = _hm(verts, faces, tol=1e-4, storage="f64", max_rhs=3)
    perm = H.perm()
    assert np.array_equal(np.sort(perm), np.arange(fac.N))
    X = np.random.default_rng(4).random((fac.N, 3))
    big = torch.zeros((3, fac.N + 7), dtype=torch.float64, device=DEV)
    big[:, :fac.N] = torch.from_numpy(X.T).to(DEV)
    Xv = big.t()[: fac.N]                      # column-major view, ld = N + 7
    Y1 = H.matvec(Xv).cpu().numpy()
    Xt = torch.from_numpy(np.ascontiguousarray(X[perm])).to(DEV)
    Yt = H.matvec(Xt, order="tree").cpu().numpy()
    np.testing.assert_array_equal(Yt, Y1[perm])
    assert _rel(Y1, F @ X) <= 1e-4 + 1e-6


def test_solve_matches_lapack(cap):
    verts, faces, fac, F = cap
    suns = sun_directions(4, seed=1)
    Q = ref.insolation(fac, suns)
    E = 0.3 * Q
    H = _hm(verts, faces, tol=1e-3, storage="f64", max_rhs=4)
    B, info = H.solve(torch.from_numpy(E).to(DEV), rho=0.3, rtol=1e-10)
    B0 = ref.solve_direct(F, 0.3, E)
    err = _rel(B.cpu().numpy(), B0)
    print("solve err", err, info)
    assert err <= 1e-3
    assert info["converged"] and np.all(info["iters"] > 0)
    # per-column tolerance 1e-3 is met in a few iterations (spectral radius ~0.04)
    B2, info2 = H.solve(torch.from_numpy(E).to(DEV), rho=0.3, rtol=1e-3)
    for c in range(4):
        assert _rel(B2.cpu().numpy()[:, c], B0[:, c]) <= 1e-3
    assert info2["total_iters"] <= 5


def test_solve_rho_vector_ir_band(cap):
    verts, faces, fac, F = cap
    rng = np.random.default_rng(5)
    E = rng.uniform(0, 50, (fac.N, 2))
    rho = rng.uniform(0.2, 1.0, fac.N)
    H = _hm(verts, faces, tol=1e-5, storage="f64", max_rhs=2)
    B, info = H.solve(torch.from_numpy(E).to(DEV), rho=torch.from_numpy(rho).to(DEV), rtol=1e-12)
    B0 = ref.solve_direct(F, rho, E)
    assert _rel(B.cpu().numpy(), B0) <= 1e-5 + 1e-6


def test_single_leaf_and_deep_leaves():
    verts, faces = cap_mesh(CapSpec(h=350.0, seed=9))
    fac = ref.Facets(verts, faces)
    F = ref.view_factor_matrix(fac)
    assert fac.N <= 64
    H = _hm(verts, faces, tol=1e-8)
    X = np.random.default_rng(6).random(fac.N)
    assert _rel(H.matvec(torch.from_numpy(X).to(DEV)).cpu().numpy(), F @ X) < 1e-12
    verts, faces = cap_mesh(CapSpec(h=100.0, seed=9))
    fac = ref.Facets(verts, faces)
    F = ref.view_factor_matrix(fac)
    H = _hm(verts, faces, tol=1e-8, max_depth=1)  # leaves far above 64 rows
    X = np.random.default_rng(7).random(fac.N)
    assert _rel(H.matvec(torch.from_numpy(X).to(DEV)).cpu().numpy(), F @ X) < 1e-7


def test_insolation_matches_reference(cap):
    verts, faces, fac, F = cap
    suns = sun_directions(16, seed=2)
    Q0 = ref.insolation(fac, suns)
    H = _hm(verts, faces, tol=1e-3)
    Q = H.insolation(suns, flux=1365.0).cpu().numpy()
    assert np.array_equal(Q > 0, Q0 > 0)          # shadow decisions are bit-exact
    np.testing.assert_allclose(Q, Q0, rtol=1e-13, atol=1e-10)
    Qt = H.insolation(suns, flux=1365.0, order="tree").cpu().numpy()
    np.testing.assert_array_equal(Qt, Q[H.perm()])


def test_insolation_terrain_low_sun():
    from synth import DemSpec, dem_mesh, sun_grid_azimuth
    verts, faces = dem_mesh(DemSpec(n=24, seed=3))
    fac = ref.Facets(verts, faces)
    suns = sun_grid_azimuth(1.5, 24, 15.0)
    Q0 = ref.insolation(fac, suns)
    H = _hm(verts, faces, tol=1e-3)
    Q = H.insolation(suns).cpu().numpy()
    assert 0.05 < (Q0 == 0).mean() < 0.95
    assert np.array_equal(Q > 0, Q0 > 0)
    np.testing.assert_allclose(Q, Q0, rtol=1e-13, atol=1e-10)


@pytest.mark.parametrize("n", [12, 16])
def test_raycast_visibility_terrain(n):
    """V_ij by ray casting (section 3.2) on occluding terrain: with a tight
    tolerance the GPU product equals the reference F built with brute force."""
    from synth import DemSpec, dem_mesh
    verts, faces = dem_mesh(DemSpec(n=n, seed=3))
    fac = ref.Facets(verts, faces)
    vis = ref.pair_visibility(fac, "raycast")
    F = ref.view_factor_matrix(fac, vis)
    assert (vis != ref.pair_visibility(fac, "backface")).sum() > 1000
    H = _hm(verts, faces, tol=1e-12, visibility="raycast", leaf_size=16)
    X = np.random.default_rng(8).random(fac.N)
    Y = H.matvec(torch.from_numpy(X).to(DEV)).cpu().numpy()
    assert _rel(Y, F @ X) < 1e-10


# ------------------------------------------------------------ multi-RHS (MFMA) path
@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("R", [16, 37, 130])
def test_matmat_mfma(cap, storage, R):
    verts, faces, fac, F = cap
    H = _hm(verts, faces, tol=1e-4, storage=storage, max_rhs=R)
    X = np.random.default_rng(10 + R).random((fac.N, R))
    dt = torch.float64 if storage == "f64" else torch.float32
    Y = H.matvec(torch.from_numpy(X).to(DEV, dt)).double().cpu().numpy()
    assert _rel(Y, F @ X) <= 1e-4 + 1e-6
    cols = [0, R // 2, R - 1]
    for c in cols:                                   # every column is right, not only the norm
        assert _rel(Y[:, c], F @ X[:, c]) <= 1e-4 + 1e-6


@pytest.mark.parametrize("nearfield", ["dense", "csr"])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_matmat_nearfield(cap, nearfield, storage):
    verts, faces, fac, F = cap
    H = _hm(verts, faces, tol=1e-6, storage=storage, nearfield=nearfield, max_rhs=40)
    st = H.stats()
    assert (st["n_csr"] if nearfield == "csr" else st["n_dense"]) > 0
    X = np.random.default_rng(11).random((fac.N, 40))
    dt = torch.float64 if storage == "f64" else torch.float32
    Y = H.matvec(torch.from_numpy(X).to(DEV, dt)).double().cpu().numpy()
    assert _rel(Y, F @ X) <= 1e-6 + 1e-6


def test_matmat_big_leaves_and_terrain():
    verts, faces = cap_mesh(CapSpec(h=100.0, seed=9))
    fac = ref.Facets(verts, faces)
    F = ref.view_factor_matrix(fac)
    H = _hm(verts, faces, tol=1e-8, max_depth=1, max_rhs=20)
    X = np.random.default_rng(12).random((fac.N, 20))
    assert _rel(H.matvec(torch.from_numpy(X).to(DEV)).cpu().numpy(), F @ X) < 1e-7
    from synth import DemSpec, dem_mesh
    verts, faces = dem_mesh(DemSpec(n=16, seed=3))
    fac = ref.Facets(verts, faces)
    F = ref.view_factor_matrix(fac, ref.pair_visibility(fac, "raycast"))
    for nf in ("auto", "csr"):
        H = _hm(verts, faces, tol=1e-12, visibility="raycast", leaf_size=16, nearfield=nf, max_rhs=24)
        X = np.random.default_rng(13).random((fac.N, 24))
        assert _rel(H.matvec(torch.from_numpy(X).to(DEV)).cpu().numpy(), F @ X) < 1e-10


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_csr_near_field_multi_rhs_terrain(storage):
    """CSR near field of an occluded terrain through the multi-RHS expansion
    (each tile's CSR slices as one compressed panel over the union of their
    nonzero columns): 32 x 32 DEM, leaf 32 (several CSR slices per 64-row
    tile), ray-cast visibility, R = 37 (a ragged last column tile), against
    the oracle's dense F; the single-RHS product, which reads the CSR rows
    directly, agrees column by column."""
    from synth import DemSpec, dem_mesh
    verts, faces = dem_mesh(DemSpec(n=32, extent=320.0, seed=4))
    fac = ref.Facets(verts, faces)
    F = ref.view_factor_matrix(fac, ref.pair_visibility(fac, "raycast"))
    H = _hm(verts, faces, tol=1e-6, storage=storage, visibility="raycast", leaf_size=32, nearfield="csr",
            max_rhs=37)
    st = H.stats()
    assert st["n_csr"] > 0 and st["n_dense"] == 0
    X = np.random.default_rng(21).random((fac.N, 37))
    dt = torch.float64 if storage == "f64" else torch.float32
    Xd = torch.from_numpy(X).to(DEV, dt)
    Y = H.matvec(Xd).double().cpu().numpy()
    tol = 1e-6 + (1e-12 if storage == "f64" else 2e-6)
    assert _rel(Y, F @ X) <= tol
    for c in (0, 18, 36):
        assert _rel(Y[:, c], F @ X[:, c]) <= tol
        y1 = H.matvec(Xd[:, c].contiguous()).double().cpu().numpy()
        assert _rel(Y[:, c], y1) <= (1e-13 if storage == "f64" else 3e-6)


def test_matmat_agrees_with_single_rhs(cap):
    verts, faces, fac, F = cap
    H = _hm(verts, faces, tol=1e-3, storage="f64", max_rhs=16)
    X = np.random.default_rng(14).random((fac.N, 16))
    Xd = torch.from_numpy(X).to(DEV)
    Ym = H.matvec(Xd).cpu().numpy()
    Y1 = np.stack([H.matvec(Xd[:, c].contiguous()).cpu().numpy() for c in range(16)], axis=1)
    np.testing.assert_allclose(Ym, Y1, rtol=1e-12, atol=1e-15 * np.abs(Y1).max())


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_solve_many_rhs(cap, storage):
    verts, faces, fac, F = cap
    suns = sun_directions(64, seed=3)
    E = 0.3 * ref.insolation(fac, suns)
    B0 = ref.solve_direct(F, 0.3, E)
    H = _hm(verts, faces, tol=1e-3, storage=storage, max_rhs=64)
    dt = torch.float64 if storage == "f64" else torch.float32
    B, info = H.solve(torch.from_numpy(E).to(DEV, dt), rho=0.3, rtol=1e-3)
    Bn = B.double().cpu().numpy()
    errs = [_rel(Bn[:, c], B0[:, c]) for c in range(64)]
    assert max(errs) <= 1e-3
    assert info["converged"] and info["total_iters"] <= 5
    # IR band (rho = 1) on the same matrix
    B, info = H.solve(torch.from_numpy(E).to(DEV, dt), rho=1.0, rtol=1e-6, max_iter=200)
    B1 = ref.solve_direct(F, 1.0, E)
    assert _rel(B.double().cpu().numpy(), B1) <= 1e-3


# ------------------------------------------------------------ layouts and graphs
@pytest.mark.parametrize("R", [3, 20])
def test_rmajor_layout_matches_colmajor(cap, R):
    from paper_2209_07632_amd.rad import ldr_of
    verts, faces, fac, F = cap
    H = _hm(verts, faces, tol=1e-4, storage="f64", max_rhs=R)
    perm = H.perm()
    X = np.random.default_rng(20 + R).random((fac.N, R))
    Y = H.matvec(torch.from_numpy(X).to(DEV)).cpu().numpy()
    Xr = np.zeros((fac.N, ldr_of(R)))
    Xr[:, :R] = X[perm]
    Yr = H.matvec(torch.from_numpy(Xr).to(DEV), order="tree_rmajor", R=R).cpu().numpy()
    np.testing.assert_allclose(Yr[:, :R], Y[perm], rtol=1e-12, atol=1e-15)
    suns = sun_directions(R, seed=7)
    Qr = H.insolation(suns, order="tree_rmajor").cpu().numpy()
    Q = H.insolation(suns).cpu().numpy()
    np.testing.assert_array_equal(Qr[:, :R], Q[perm])
    E = torch.from_numpy(0.3 * Q).to(DEV)
    B, _ = H.solve(E, rho=0.3, rtol=1e-8)
    Br, _ = H.solve(torch.from_numpy(0.3 * Qr).to(DEV), rho=0.3, rtol=1e-8, order="tree_rmajor", R=R)
    np.testing.assert_allclose(Br.cpu().numpy()[:, :R], B.cpu().numpy()[perm], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("R", [1, 24])
def test_graph_replays_match_eager(cap, R):
    """Every replay of the cached iteration graphs equals the eager result, with
    eager work and synchronisation between the replays."""
    verts, faces, fac, F = cap
    H = _hm(verts, faces, tol=1e-4, storage="f32", max_rhs=R)
    rng = np.random.default_rng(30 + R)
    Es = [torch.from_numpy(rng.uniform(0, 100, (fac.N, R))).to(DEV, torch.float32) for _ in range(3)]
    ref_B = [H.solve(E, rho=0.3, rtol=1e-6, use_graph=False)[0].cpu().numpy() for E in Es]
    for rep in range(3):
        for E, B0 in zip(Es, ref_B):
            B, info = H.solve(E, rho=0.3, rtol=1e-6, use_graph=True)
            np.testing.assert_array_equal(B.cpu().numpy(), B0)
            # eager work on the same stream between replays
            H.matvec(E[:, 0].contiguous())
            torch.cuda.synchronize()


# ------------------------------------------------------------ two-band equilibrium
@pytest.mark.parametrize("R,order", [(1, "original"), (20, "original"), (20, "tree_rmajor")])
def test_equilibrium_temperature(cap, R, order):
    """GPU two-band T equals the FP64 reference chain (section 5.1) and the
    closed form of section 7.1 on shadowed facets."""
    from paper_2209_07632_amd.rad import ldr_of
    verts, faces, fac, F = cap
    e = 15.0
    suns = np.tile([np.cos(np.deg2rad(e)), 0.0, np.sin(np.deg2rad(e))], (R, 1))
    Q = ref.insolation(fac, suns, S=1365.0)
    out0 = ref.equilibrium_temperature(lambda X: F @ X, Q, 0.3, 0.99)
    H = _hm(verts, faces, tol=1e-6, storage="f64", max_rhs=R)
    if order == "tree_rmajor":
        perm = H.perm()
        Qr = np.zeros((fac.N, ldr_of(R)))
        Qr[:, :R] = Q[perm]
        T, Qv, Qi, info = H.equilibrium(torch.from_numpy(Qr).to(DEV), order=order, R=R)
        Tn = np.empty((fac.N, R))
        Tn[perm] = T.cpu().numpy()[:, :R]
        Qvn = np.empty((fac.N, R))
        Qvn[perm] = Qv.cpu().numpy()[:, :R]
    else:
        T, Qv, Qi, info = H.equilibrium(torch.from_numpy(Q).to(DEV))
        Tn, Qvn = T.cpu().numpy().reshape(fac.N, R), Qv.cpu().numpy().reshape(fac.N, R)
    assert np.max(np.abs(Tn - out0["T"]) / out0["T"]) < 1e-5
    assert _rel(Qvn, out0["Q_vis"]) < 1e-5
    shadow = Q[:, 0] == 0.0
    Tc = ref.crater_shadow_temperature(1365.0, e, 0.3, 0.99, ref.crater_f(5.0))
    assert abs(Tn[shadow, 0].mean() - Tc) / Tc < 5e-3
    assert np.all(info["iters_sw"] > 0) and np.all(info["iters_ir"] > 0)


def test_tall_block_orthogonalisation_path(cap, monkeypatch):
    """The many-workgroup CGS2 (used for blocks of thousands of rows) gives the
    same compression quality as the single-workgroup one, forced on small blocks."""
    verts, faces, fac, F = cap
    X = np.random.default_rng(40).random((fac.N, 2))
    monkeypatch.setenv("RAD_CGS2_TALL_ROWS", "100")
    for tol in (1e-4, 1e-8):
        H = _hm(verts, faces, tol=tol, storage="f64", max_rhs=2)
        Y = H.matvec(torch.from_numpy(X).to(DEV)).cpu().numpy()
        assert _rel(Y, F @ X) <= tol + 1e-6


# ------------------------------------------------------------ 16-bit operator + refinement
# unit roundoff of the 16-bit formats (round to nearest)
U16 = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}


@pytest.mark.parametrize("lowp", ["f16", "bf16"])
@pytest.mark.parametrize("R", [16, 130, 200, 256])
def test_lowp_matvec(cap, lowp, R):
    """The 16-bit copy of F-hat (power-of-two column scaling, FP32 accumulation)
    stays within tol + 2u of the exact product: each term of a dot product
    carries at most the rounding of its two operands."""
    verts, faces, fac, F = cap
    tol = 1e-4
    H = _hm(verts, faces, tol=tol, storage="f32", max_rhs=R, lowp=lowp)
    X = np.random.default_rng(50 + R).random((fac.N, R))
    Xd = torch.from_numpy(X).to(DEV, torch.float32)
    Y16 = H.matvec(Xd, lowp=True).double().cpu().numpy()
    Y32 = H.matvec(Xd).double().cpu().numpy()
    Y = F @ X
    err16, err32 = _rel(Y16, Y), _rel(Y32, Y)
    print(f"{lowp} R={R} err16={err16:.3e} err32={err32:.3e}")
    assert err32 <= tol + 1e-6
    assert err16 <= tol + 2 * U16[lowp]
    for c in (0, R - 1):
        assert _rel(Y16[:, c], Y[:, c]) <= tol + 2 * U16[lowp]
    assert _rel(Y16, Y32) > 1e-7            # the 16-bit operator really was applied


@pytest.mark.parametrize("lowp", ["f16", "bf16"])
def test_refined_solve_beats_16bit_roundoff(cap, lowp):
    """Iterative refinement with the 16-bit operator in the inner Jacobi sweeps
    and an FP32-operator residual accumulated in FP64 reaches 1e-6 relative
    residual, far below the 16-bit unit roundoff."""
    verts, faces, fac, F = cap
    R = 40
    suns = sun_directions(R, seed=5)
    E = 0.3 * ref.insolation(fac, suns)
    B0 = ref.solve_direct(F, 0.3, E)
    H = _hm(verts, faces, tol=1e-7, storage="f32", max_rhs=R, lowp=lowp)
    Ed = torch.from_numpy(E).to(DEV, torch.float32)
    for use_graph in (False, True):
        B, info = H.solve(Ed, rho=0.3, rtol=1e-6, refine=True, inner_iters=3, use_graph=use_graph)
        Bn = B.double().cpu().numpy()
        errs = [_rel(Bn[:, c], B0[:, c]) for c in range(R)]
        print(f"{lowp} graph={use_graph} outer={info['total_iters']} inner={info['inner_iters']} "
              f"max err={max(errs):.3e} res={info['rel_change'].max():.3e}")
        assert info["converged"] and info["total_iters"] <= 8
        assert info["inner_iters"] == 3 * info["total_iters"]
        assert np.all(info["rel_change"] <= 1e-6)
        assert max(errs) <= 5e-6
    # the same system by plain FP32 Jacobi agrees
    Bj, _ = H.solve(Ed, rho=0.3, rtol=1e-7)
    assert _rel(Bn, Bj.double().cpu().numpy()) <= 5e-6


@pytest.mark.parametrize("lowp", ["f16", "bf16"])
def test_refined_solve_ir_band_rho_vector(cap, lowp):
    """Refinement for the long-wave band (rho = 1) and for a per-facet rho, in
    the internal layout."""
    from paper_2209_07632_amd.rad import ldr_of
    verts, faces, fac, F = cap
    R = 20
    rng = np.random.default_rng(60)
    E = rng.uniform(0.0, 100.0, (fac.N, R))
    H = _hm(verts, faces, tol=1e-7, storage="f32", max_rhs=R, lowp=lowp)
    perm = H.perm()
    B, info = H.solve(torch.from_numpy(E).to(DEV, torch.float32), rho=1.0, rtol=1e-6, max_iter=60, refine=True)
    assert _rel(B.double().cpu().numpy(), ref.solve_direct(F, 1.0, E)) <= 1e-5
    rho = rng.uniform(0.1, 0.6, fac.N)
    Er = np.zeros((fac.N, ldr_of(R)))
    Er[:, :R] = E[perm]
    Br, info = H.solve(torch.from_numpy(Er).to(DEV, torch.float32), rho=torch.from_numpy(rho[perm]).to(DEV, torch.float32),
                       rtol=1e-6, order="tree_rmajor", R=R, refine=True)
    Bo = np.empty((fac.N, R))
    Bo[perm] = Br.double().cpu().numpy()[:, :R]
    assert _rel(Bo, ref.solve_direct(F, rho, E)) <= 5e-6
    assert np.all(info["iters"] > 0)


# ------------------------------------------------------------ the benchmark's own configuration
def test_full_size_cap_sampled_columns():
    """The 40k-facet cap with 1,024 suns, near field CSR, tol 1e-3, FP32, solved
    in the autotuned launch configuration the benchmark times: 16 columns
    spread over the sun elevations (the lowest and highest included) against
    the FP64 matrix-free reference (insolation and Jacobi), and shadows bit for
    bit on those columns."""
    from paper_2209_07632_amd import HMatrix
    from paper_2209_07632_amd.rad import ldr_of
    from synth import CAP_LARGE
    verts, faces = cap_mesh(CAP_LARGE)
    R = 1024
    suns = sun_directions(R, (5.0, 30.0), seed=1)
    print("[full] cap40k R=1024", flush=True)
    H = HMatrix(verts, faces, tol=1e-3, storage="f32", nearfield="csr", max_rhs=R)
    H.autotune(R, nrep=2)
    Q = H.insolation(suns, flux=1365.0, order="tree_rmajor")
    B, info = H.solve(0.3 * Q, rho=0.3, rtol=1e-3, order="tree_rmajor", R=R)
    assert info["converged"]
    perm = H.perm()
    order = np.argsort(np.arcsin(suns[:, 2]), kind="stable")
    cols = sorted(set(order[np.round(np.linspace(0, R - 1, 16)).astype(int)].tolist()))
    assert len(cols) == 16
    fac = ref.Facets(verts, faces)
    Q0 = ref.insolation(fac, suns[cols], S=1365.0)
    Qg = np.empty((fac.N, len(cols)))
    Qg[perm] = Q.double().cpu().numpy()[:, cols]
    np.testing.assert_array_equal(Qg == 0.0, Q0 == 0.0)
    B0, _ = ref.jacobi(lambda X: ref.matvec_free(fac, X), 0.3, 0.3 * Q0, tol=1e-10)
    Bg = np.empty((fac.N, len(cols)))
    Bg[perm] = B.double().cpu().numpy()[:, cols]
    for c in range(len(cols)):
        assert _rel(Bg[:, c], B0[:, c]) < 1e-3


def test_full_size_cap_single_rhs_products():
    """The single-RHS kernels (R < 16) on the 40k-facet cap at tol 1e-3, FP32,
    near field CSR: column nodes of up to 10k facets (the long-projection path,
    one workgroup per V column) and segmented tile reductions.  R = 1 and R = 3
    against the matrix-core product of the same columns (FP32 rounding order
    only: 1e-5 per column) and R = 1 against the FP64 matrix-free oracle
    product (within tol + 1e-6)."""
    from paper_2209_07632_amd import HMatrix
    from synth import CAP_LARGE
    verts, faces = cap_mesh(CAP_LARGE)
    print("[full] cap40k single-RHS products", flush=True)
    H = HMatrix(verts, faces, tol=1e-3, storage="f32", nearfield="csr", max_rhs=16)
    X = np.random.default_rng(44).random((H.N, 16))
    Xd = torch.from_numpy(X).to(DEV, torch.float32)
    Ymm = H.matvec(Xd).double().cpu().numpy()
    Y1 = H.matvec(Xd[:, 0].contiguous()).double().cpu().numpy()
    Y3 = H.matvec(Xd[:, 1:4].contiguous()).double().cpu().numpy()
    assert _rel(Y1, Ymm[:, 0]) <= 1e-5
    for c in range(3):
        assert _rel(Y3[:, c], Ymm[:, 1 + c]) <= 1e-5
    fac = ref.Facets(verts, faces)
    Y0 = ref.matvec_free(fac, X[:, :1])[:, 0]
    assert _rel(Y1, Y0) <= 1e-3 + 1e-6


# ------------------------------------------------------------ zero blocks only
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_flat_plane_is_all_zero_blocks(storage):
    """P9: on a flat plane every n_i . (x_j - x_i) is zero, so F = 0: every
    block is a zero block, the product is exactly zero and the solve returns
    B = E after one iteration, on both kernel paths."""
    from paper_2209_07632_amd import HMatrix
    g = np.linspace(0.0, 200.0, 21)
    xx, yy = np.meshgrid(g, g, indexing="ij")
    verts = np.column_stack([xx.ravel(), yy.ravel(), np.zeros(xx.size)])
    faces = []
    for i in range(20):
        for j in range(20):
            a, b, c, d = i * 21 + j, (i + 1) * 21 + j, (i + 1) * 21 + j + 1, i * 21 + j + 1
            faces += [[a, b, c], [a, c, d]]
    faces = np.array(faces, dtype=np.int32)
    fac = ref.Facets(verts, faces)
    assert not ref.view_factor_matrix(fac).any()
    H = _hm(verts, faces, tol=1e-3, storage=storage, visibility="raycast", max_rhs=20)
    st = H.stats()
    assert st["n_zero"] > 0 and st["n_dense"] == st["n_csr"] == st["n_lowrank"] == 0
    dt = torch.float64 if storage == "f64" else torch.float32
    for R in (1, 20):
        E = torch.rand((fac.N, R), dtype=dt, device=DEV) * 100.0
        assert not H.matvec(E).any()
        B, info = H.solve(E, rho=0.9, rtol=1e-12)
        assert torch.equal(B.reshape(E.shape), E)
        assert info["total_iters"] == 1 and np.all(info["iters"] == 1)
