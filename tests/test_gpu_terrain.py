"""Terrain-shaped products on the GPU: ray-cast visibility, dense near field
with large leaves, so that every 64-row tile reduces over thousands of panel
columns, the regime of the 131k-facet terrain (Algorithm 5 with R = 256).

Checks, at N = 8192 facets:
* the FP32 matrix-core product and the BF16 wide products (the one-tile
  kernel for leaves of 64 facets, the tile-pair kernel for leaves of 512)
  against the exported blocks of F-hat densified in FP64: arithmetic parity of
  the kernels on every row and column (FP32: 1e-5 relative per column; BF16:
  2u = 2^-7 per column);
* both against exact FP64 rows of F (ray-cast visibility by brute force in the
  reference) on 48 sampled rows: within eps + 1e-6 (FP32) and eps + 2u (BF16)
  of the sampled block (with a factor 2 on eps: a norm-wise eps compression
  need not hold it on every subset of rows);
* the refined BF16 solve against the FP32 Jacobi solve of the same system.
"""
import numpy as np
import pytest

from oracle import reference as ref
from synth import DemSpec, dem_mesh, sun_grid_azimuth
from hmat_blocks import densify, read_export

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
U_BF16 = 2.0 ** -8
TOL = 1e-3


@pytest.fixture(scope="module")
def terrain():
    verts, faces = dem_mesh(DemSpec(n=64, seed=3))
    fac = ref.Facets(verts, faces)
    rows = sorted(set(np.linspace(0, fac.N - 1, 48).round().astype(int).tolist()))
    Fr = ref.view_factor_rows(fac, rows, "raycast")
    return verts, faces, fac, rows, Fr


def _build(verts, faces, leaf, tmp_path):
    from paper_2209_07632_amd import HMatrix
    print(f"[build] terrain N={faces.shape[0]} leaf={leaf} dense near field, bf16 copy", flush=True)
    H = HMatrix(verts, faces, tol=TOL, storage="f32", visibility="raycast", nearfield="dense", leaf_size=leaf,
                max_rhs=256, lowp="bf16", max_rank=256)
    path = tmp_path / f"terrain{leaf}.bin"
    H.export(path)
    return H, densify(read_export(path))


def _colwise(Y, Yx):
    return np.max(np.linalg.norm(Y - Yx, axis=0) / np.linalg.norm(Yx, axis=0))


@pytest.mark.parametrize("leaf", [512, 64])
def test_long_reduction_products(terrain, tmp_path, leaf):
    verts, faces, fac, rows, Fr = terrain
    H, Fh = _build(verts, faces, leaf, tmp_path)
    st = H.stats()
    print(f"stats: dense {st['n_dense']} lowrank {st['n_lowrank']} zero {st['n_zero']} "
          f"widest panel {st['max_panel_cols']}")
    assert st["n_dense"] > 0 and st["max_panel_cols"] >= (4096 if leaf == 512 else 1024)
    X = np.random.default_rng(leaf).random((fac.N, 256))
    Xd = torch.from_numpy(X).to(DEV, torch.float32)
    Yx = Fh @ X
    Y32 = H.matvec(Xd).double().cpu().numpy()
    Y16 = H.matvec(Xd, lowp=True).double().cpu().numpy()
    e32, e16 = _colwise(Y32, Yx), _colwise(Y16, Yx)
    print(f"leaf {leaf}: vs densified F-hat: FP32 {e32:.2e}, BF16 {e16:.2e}")
    assert e32 <= 1e-5
    assert e16 <= 2 * U_BF16
    Yr = Fr @ X
    s32 = np.linalg.norm(Y32[rows] - Yr) / np.linalg.norm(Yr)
    s16 = np.linalg.norm(Y16[rows] - Yr) / np.linalg.norm(Yr)
    print(f"leaf {leaf}: vs exact sampled rows: FP32 {s32:.2e}, BF16 {s16:.2e}")
    assert s32 <= 2 * TOL + 1e-6
    assert s16 <= 2 * TOL + 2 * U_BF16
    # fewer columns than the wide kernel's 256 (ragged column tile)
    Y16b = H.matvec(Xd[:, :200].contiguous(), lowp=True).double().cpu().numpy()
    assert _colwise(Y16b, Yx[:, :200]) <= 2 * U_BF16


def test_refined_solve_on_terrain(terrain, tmp_path):
    verts, faces, fac, rows, Fr = terrain
    H, Fh = _build(verts, faces, 256, tmp_path)
    suns = sun_grid_azimuth(1.5, 256, 1.4)
    E = 0.3 * H.insolation(suns, flux=1365.0)
    Bj, ij = H.solve(E, rho=0.3, rtol=1e-7, max_iter=200)
    Br, ir = H.solve(E, rho=0.3, rtol=1e-4, refine=True, inner_iters=3, max_iter=50)
    Bd = ref.solve_direct(Fh, 0.3, E.double().cpu().numpy())
    ej = _colwise(Bj.double().cpu().numpy(), Bd)
    er = _colwise(Br.double().cpu().numpy(), Bd)
    print(f"FP32 Jacobi {ij['total_iters']} iterations err {ej:.2e}; BF16 refined {ir['total_iters']} steps err {er:.2e}")
    assert ej <= 1e-5 and er <= 2e-4


@pytest.mark.parametrize("leaf", [512, 64])
def test_csr_near_field_products(terrain, tmp_path, leaf):
    """The terrain with Algorithm 4's own near-field form (CSR): every tile's
    CSR slices run as one compressed panel in the FP32 products.  At leaf 512
    the tiles reduce over thousands of columns, so the single-RHS product is
    cut into segments that cross from the dense / low-rank panel into the
    compressed one, and the BF16 product takes the wide tile-pair kernels with
    one compressed panel per pair; at leaf 64 the tiles do not pair and the
    BF16 product walks the CSR rows.  The products match the exported blocks
    of F-hat densified in FP64 column by column (FP32: 1e-5, BF16: 2u), and
    the sampled exact rows; the refined BF16 solve matches the direct solve."""
    from paper_2209_07632_amd import HMatrix
    verts, faces, fac, rows, Fr = terrain
    print(f"[build] terrain N={faces.shape[0]} leaf={leaf} CSR near field, bf16 copy", flush=True)
    H = HMatrix(verts, faces, tol=TOL, storage="f32", visibility="raycast", nearfield="csr", leaf_size=leaf,
                max_rhs=64, max_rank=256, lowp="bf16")
    path = tmp_path / f"terrain_csr{leaf}.bin"
    H.export(path)
    Fh = densify(read_export(path))
    st = H.stats()
    print(f"stats: csr {st['n_csr']} lowrank {st['n_lowrank']} nnz {st['nnz_near']} "
          f"csr bytes {st['bytes_csr']} compressed panels {st['bytes_csr_panels']}")
    assert st["n_csr"] > 0 and st["n_dense"] == 0 and st["bytes_csr_panels"] > 0
    X = np.random.default_rng(leaf + 1).random((fac.N, 64))
    Xd = torch.from_numpy(X).to(DEV, torch.float32)
    Yx = Fh @ X
    Y32 = H.matvec(Xd).double().cpu().numpy()
    assert _colwise(Y32, Yx) <= 1e-5
    for c in (0, 31, 63):
        y1 = H.matvec(Xd[:, c].contiguous()).double().cpu().numpy()
        assert np.linalg.norm(y1 - Yx[:, c]) / np.linalg.norm(Yx[:, c]) <= 1e-5
    Yr = Fr @ X
    assert np.linalg.norm(Y32[rows] - Yr) / np.linalg.norm(Yr) <= 2 * TOL + 1e-6
    Y16 = H.matvec(Xd, lowp=True).double().cpu().numpy()
    e16 = _colwise(Y16, Yx)
    Y16b = H.matvec(Xd[:, :40].contiguous(), lowp=True).double().cpu().numpy()
    print(f"leaf {leaf} CSR: FP32 {_colwise(Y32, Yx):.2e}, BF16 {e16:.2e}")
    assert e16 <= 2 * U_BF16 and _colwise(Y16b, Yx[:, :40]) <= 2 * U_BF16
    suns = sun_grid_azimuth(1.5, 64, 5.0)
    E = 0.3 * H.insolation(suns, flux=1365.0)
    Br, ir = H.solve(E, rho=0.3, rtol=1e-4, refine=True, inner_iters=3, max_iter=50)
    Bd = ref.solve_direct(Fh, 0.3, E.double().cpu().numpy())
    er = _colwise(Br.double().cpu().numpy(), Bd)
    print(f"leaf {leaf} CSR: BF16 refined {ir['total_iters']} steps err {er:.2e}")
    assert er <= 2e-4


def test_csr_single_rhs_fp64_segments(terrain, tmp_path):
    """FP64 terrain with CSR near field at leaf 512, built for single
    right-hand sides only: the tiles' reductions (low-rank columns, then the
    compressed CSR panel) run longer than the FP64 segment length of 2,048
    columns, so the product is cut into segments, some inside the compressed
    panel; it matches the exported blocks densified in FP64 to 1e-12."""
    from paper_2209_07632_amd import HMatrix
    verts, faces, fac, rows, Fr = terrain
    print(f"[build] terrain N={faces.shape[0]} leaf=512 CSR near field, FP64, max_rhs 1", flush=True)
    H = HMatrix(verts, faces, tol=TOL, storage="f64", visibility="raycast", nearfield="csr", leaf_size=512,
                max_rhs=1, max_rank=256)
    path = tmp_path / "terrain_csr_f64.bin"
    H.export(path)
    Fh = densify(read_export(path))
    st = H.stats()
    print(f"stats: csr {st['n_csr']} widest panel {st['max_panel_cols']} compressed panels {st['bytes_csr_panels']}")
    assert st["n_csr"] > 0 and st["bytes_csr_panels"] > 0
    x = np.random.default_rng(5).random(fac.N)
    y = H.matvec(torch.from_numpy(x).to(DEV)).cpu().numpy()
    assert np.linalg.norm(y - Fh @ x) / np.linalg.norm(Fh @ x) <= 1e-12
