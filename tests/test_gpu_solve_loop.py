"""The Jacobi loop (sections 3 and 5.1), on the matrix-core kernels (R >= 16)
and on the single-RHS kernels (R < 16), both with the device-side stopping
test and one iteration queued ahead: per-column stopping against the oracle's
Jacobi, the max_iter cap, and solves that follow one another on one matrix
(the device-side stopping flag of a converged solve must not leak into the
next one)."""
import numpy as np
import pytest

from oracle import reference as ref
from synth import CAP_SMALL, cap_mesh, sun_directions

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def cap():
    verts, faces = cap_mesh(CAP_SMALL)
    fac = ref.Facets(verts, faces)
    return verts, faces, fac, ref.view_factor_matrix(fac)


def _hm(verts, faces, **kw):
    from paper_2209_07632_amd import HMatrix
    print(f"[build] N={faces.shape[0]} {kw}", flush=True)
    return HMatrix(verts, faces, **kw)


def _mixed_rhs(fac, R, seed):
    """Columns that converge at different iterations: sunlight, noise, a single
    lit facet and an all-zero column."""
    rng = np.random.default_rng(seed)
    E = np.empty((fac.N, R))
    E[:, : R // 2] = 0.3 * ref.insolation(fac, sun_directions(R // 2, seed=seed))
    E[:, R // 2:] = rng.uniform(0, 50, (fac.N, R - R // 2))
    E[:, -2] = 0.0
    E[rng.integers(fac.N), -2] = 400.0
    E[:, -1] = 0.0
    return E


@pytest.mark.parametrize("R", [40, 6])
@pytest.mark.parametrize("rho,rtol", [(0.3, 1e-6), (0.9, 1e-4)])
def test_per_column_iterations_match_oracle(cap, rho, rtol, R):
    verts, faces, fac, F = cap
    E = _mixed_rhs(fac, R, seed=int(10 * rho))
    H = _hm(verts, faces, tol=1e-10, storage="f64", max_rhs=R)
    B, info = H.solve(torch.from_numpy(E).to(DEV), rho=rho, rtol=rtol, max_iter=300)
    Bo, it_o = ref.jacobi(lambda X: F @ X, rho, E, tol=rtol, max_iter=300)
    print(f"rho={rho} rtol={rtol} iterations gpu {info['iters']} oracle {it_o}")
    assert len(set(it_o.tolist())) >= 3            # the columns really differ
    np.testing.assert_array_equal(info["iters"], it_o)
    assert info["total_iters"] == it_o.max()
    np.testing.assert_allclose(B.cpu().numpy(), Bo, rtol=1e-8, atol=1e-8 * np.abs(Bo).max())


@pytest.mark.parametrize("R", [24, 4])
def test_max_iter_cap_returns_that_iterate(cap, R):
    verts, faces, fac, F = cap
    E = _mixed_rhs(fac, R, seed=5)
    H = _hm(verts, faces, tol=1e-10, storage="f64", max_rhs=R)
    B, info = H.solve(torch.from_numpy(E).to(DEV), rho=0.5, rtol=1e-14, max_iter=2, raise_on_noconv=False)
    assert not info["converged"] and info["total_iters"] == 2
    B2 = E.copy()
    for _ in range(2):
        B2 = E + 0.5 * (F @ B2)
    np.testing.assert_allclose(B.cpu().numpy(), B2, rtol=1e-8, atol=1e-8 * np.abs(B2).max())


@pytest.mark.parametrize("R", [32, 5])
@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_consecutive_solves_do_not_interfere(cap, storage, R):
    """A quickly converging solve, then a tight one, then the quick one again on
    one matrix: each equals the same solve on a fresh matrix, bit for bit."""
    verts, faces, fac, F = cap
    dt = torch.float64 if storage == "f64" else torch.float32
    E = torch.from_numpy(_mixed_rhs(fac, R, seed=7)).to(DEV, dt)
    H = _hm(verts, faces, tol=1e-6, storage=storage, max_rhs=R)
    runs = [(1e-2, True), (1e-7, False), (1e-2, False)]
    got = [H.solve(E, rho=0.3, rtol=rt, use_graph=g) for rt, g in runs]
    for (rt, g), (B, info) in zip(runs, got):
        Hf = _hm(verts, faces, tol=1e-6, storage=storage, max_rhs=R)
        Bf, inf_f = Hf.solve(E, rho=0.3, rtol=rt, use_graph=g)
        assert torch.equal(B, Bf), rt
        np.testing.assert_array_equal(info["iters"], inf_f["iters"])
    assert got[1][1]["total_iters"] > got[0][1]["total_iters"]
