"""GPU parity of matrix groups (many independent craters behind one
operator, one launch per kernel): products equal the per-instance products
bit for bit, solves track convergence per (instance, column) and agree with
per-instance solves and the FP64 reference."""
import numpy as np
import pytest

from oracle import reference as ref
from synth import CapSpec, cap_mesh, dem_instance, dem_mesh, sun_directions

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _meshes():
    out = [cap_mesh(CapSpec(h=h, seed=s)) for h, s in ((140.0, 1), (90.0, 2), (200.0, 3))]
    out += [dem_mesh(dem_instance(k, n)) for k, n in ((4, 800), (5, 1900))]
    return out


def _build(meshes, R, **kw):
    from paper_2209_07632_amd import HMatrix
    parts = []
    for i, (v, f) in enumerate(meshes):
        print(f"[build] instance {i} N={f.shape[0]} {kw}", flush=True)
        vis = "raycast" if i >= 3 else "backface"
        parts.append(HMatrix(v, f, max_rhs=R, visibility=vis, **kw))
    return parts


def _place(G, blocks, R):
    """Per-instance tree_rmajor blocks -> group layout (padding rows zero)."""
    from paper_2209_07632_amd.rad import ldr_of
    out = torch.zeros((G.N, ldr_of(R)), dtype=blocks[0].dtype, device=DEV)
    for k, b in enumerate(blocks):
        o, n = int(G.offsets[k]), int(G.sizes[k])
        out[o:o + n] = b
    return out


@pytest.mark.parametrize("storage,nearfield", [("f32", "auto"), ("f64", "auto"), ("f32", "csr")])
def test_group_product_equals_instances(storage, nearfield):
    """(With nearfield="csr" every instance stores its near field as CSR,
    which the products stream as compressed panels, the group's as well.)"""
    from paper_2209_07632_amd import HMatrix
    from paper_2209_07632_amd.rad import ldr_of
    R = 37
    meshes = _meshes()
    parts = _build(meshes, R, tol=1e-4, storage=storage, leaf_size=32, nearfield=nearfield)
    if nearfield == "csr":
        assert all(p.stats()["n_csr"] > 0 and p.stats()["bytes_csr_panels"] > 0 for p in parts)
    G = HMatrix.group(parts, R)
    assert G.n_inst == len(parts)
    assert np.all(G.offsets % 64 == 0) and list(G.sizes) == [p.N for p in parts]
    dt = torch.float64 if storage == "f64" else torch.float32
    rng = np.random.default_rng(1)
    X = [torch.from_numpy(rng.random((p.N, ldr_of(R)))).to(DEV, dt) for p in parts]
    Y = [p.matvec(x, order="tree_rmajor", R=R) for p, x in zip(parts, X)]
    YG = G.matvec(_place(G, X, R), order="tree_rmajor", R=R)
    for k, y in enumerate(Y):
        o, n = int(G.offsets[k]), int(G.sizes[k])
        assert torch.equal(YG[o:o + n, :R], y[:, :R]), k
    pad = torch.ones(G.N, dtype=torch.bool, device=DEV)
    for o, n in zip(G.offsets, G.sizes):
        pad[int(o):int(o + n)] = False
    assert torch.count_nonzero(YG[pad]) == 0
    st = G.stats()
    assert st["n"] == sum(p.N for p in parts)
    assert st["n_lowrank"] == sum(p.stats()["n_lowrank"] for p in parts)


@pytest.mark.parametrize("refine", [False, True])
def test_group_solve_per_instance_convergence(refine):
    from paper_2209_07632_amd import HMatrix
    R = 24
    meshes = _meshes()
    parts = _build(meshes, R, tol=1e-6, storage="f32", leaf_size=32, lowp="bf16" if refine else None)
    G = HMatrix.group(parts, R)
    Es, per_iters, per_B = [], [], []
    for k, ((v, f), p) in enumerate(zip(meshes, parts)):
        suns = sun_directions(R, seed=100 + k)
        E = 0.3 * p.insolation(suns, order="tree_rmajor")
        B, info = p.solve(E, rho=0.3, rtol=1e-6, order="tree_rmajor", R=R, refine=refine)
        Es.append(E)
        per_iters.append(info["iters"])
        per_B.append(B)
    BG, info = G.solve(_place(G, Es, R), rho=0.3, rtol=1e-6, order="tree_rmajor", R=R, refine=refine)
    print(f"refine={refine} group iterations {info['total_iters']}, per instance "
          f"{[int(i.max()) for i in per_iters]}")
    assert info["iters"].shape == (len(parts) * R,)
    np.testing.assert_array_equal(info["iters"].reshape(len(parts), R), np.stack(per_iters))
    for k, (B, p) in enumerate(zip(per_B, parts)):
        o, n = int(G.offsets[k]), int(G.sizes[k])
        Bk = BG[o:o + n, :R].double().cpu().numpy()
        Bp = B[:, :R].double().cpu().numpy()
        assert np.linalg.norm(Bk - Bp) <= 2e-6 * np.linalg.norm(Bp)
    # one instance against the FP64 reference (dense F, direct solve)
    v, f = meshes[1]
    fac = ref.Facets(v, f)
    F = ref.view_factor_matrix(fac)
    p = parts[1]
    perm = p.perm()
    o, n = int(G.offsets[1]), int(G.sizes[1])
    Eo = np.empty((n, R))
    Eo[perm] = Es[1][:, :R].double().cpu().numpy()
    B0 = ref.solve_direct(F, 0.3, Eo)
    Bo = np.empty((n, R))
    Bo[perm] = BG[o:o + n, :R].double().cpu().numpy()
    assert np.linalg.norm(Bo - B0) <= 1e-5 * np.linalg.norm(B0)


def test_group_rejects_unsupported_calls():
    from paper_2209_07632_amd import HMatrix
    from paper_2209_07632_amd.rad import RadError
    parts = _build(_meshes()[:2], 16, tol=1e-3, storage="f32")
    G = HMatrix.group(parts, 16)
    with pytest.raises(RadError):
        G.insolation(sun_directions(16, seed=1), order="tree_rmajor")
    with pytest.raises(RadError):
        G.matvec(torch.zeros(G.N, 16, device=DEV), order="original")
    with pytest.raises(RadError):
        HMatrix.group(parts, 8)
