"""GPU parity of the octree build (rad_hmat_build_tree with tree_dims = 3) on
a closed bilobed body with ray-cast visibility, against the FP64 reference's
dense F.  The closed body is the zero-block-heavy regime of section 8's
comet study: most block pairs see nothing (back faces and occlusion).

Tolerances as for the quadtree: the compressed product within eps + 1e-6
relative L2 of F X; at eps 1e-10 within 1e-9.
"""
import numpy as np
import pytest

from oracle import reference as ref
from synth import BodySpec, body_mesh

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def body():
    verts, faces = body_mesh(BodySpec(level=3))
    fac = ref.Facets(verts, faces)
    F = ref.view_factor_matrix(fac, ref.pair_visibility(fac, "raycast"))
    return verts, faces, fac, F


@pytest.mark.parametrize("R", [3, 20])
@pytest.mark.parametrize("tol", [1e-2, 1e-4, 1e-10])
def test_octree_matvec_within_tol(body, tol, R):
    from paper_2209_07632_amd import HMatrix
    verts, faces, fac, F = body
    print(f"[build] octree N={fac.N} tol={tol} R={R}", flush=True)
    H = HMatrix(verts, faces, tol=tol, storage="f64", visibility="raycast", max_rhs=R, tree="oct")
    X = np.random.default_rng(R).random((fac.N, R))
    Y = H.matvec(torch.from_numpy(X).to(DEV)).cpu().numpy()
    err = np.linalg.norm(Y - F @ X) / np.linalg.norm(F @ X)
    assert err <= (1e-9 if tol < 1e-9 else tol + 1e-6), err


def test_octree_solve_matches_lapack(body):
    from paper_2209_07632_amd import HMatrix
    verts, faces, fac, F = body
    H = HMatrix(verts, faces, tol=1e-10, storage="f64", visibility="raycast", max_rhs=16, tree="oct")
    E = np.random.default_rng(5).random((fac.N, 16))
    B, info = H.solve(torch.from_numpy(E).to(DEV), rho=1.0, rtol=1e-12)
    Bd = ref.solve_direct(F, 1.0, E)
    assert np.max(np.abs(B.cpu().numpy() - Bd)) <= 1e-9 * np.max(np.abs(Bd))
