"""GPU test of rad_hmat_matvec_noalloc, the allocation-free product: it must
equal rad_hmat_matvec (the same kernels, bit for bit) and the FP64 oracle's
F X within the stated tolerance, on two calls in a row with the second on a
smaller input (fewer right-hand sides on a smaller matrix), in every layout
and both storage precisions; and it must refuse what its static scratch
cannot hold before any device work."""
import numpy as np
import pytest

from oracle import reference as ref
from synth import CAP_LARGE, CapSpec, cap_mesh

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def meshes():
    out = []
    for h in (63.0, 90.0):                  # N = 1,586 then a smaller mesh
        v, f = cap_mesh(CapSpec(h=h, seed=0 if h == 63.0 else 11))
        fac = ref.Facets(v, f)
        out.append((v, f, ref.view_factor_matrix(fac)))
    assert out[1][2].shape[0] < out[0][2].shape[0]
    return out


def _layout(H, X, order, R):
    """X (N, R) original-order numpy array as a device tensor in `order`."""
    from paper_2209_07632_amd.rad import ldr_of
    dt = H.torch_dtype
    if order == "original":
        return torch.from_numpy(X).to(DEV, dt).t().contiguous().t()
    Xt = X[H.perm()]
    if order == "tree":
        return torch.from_numpy(Xt).to(DEV, dt).t().contiguous().t()
    out = torch.zeros((H.N, ldr_of(R)), dtype=dt, device=DEV)
    out[:, :R] = torch.from_numpy(Xt).to(DEV, dt)
    return out


def _back(H, Y, order, R):
    Y = Y.double().cpu().numpy()
    if order == "original":
        return Y
    Y = Y[:, :R]
    out = np.empty_like(Y)
    out[H.perm()] = Y
    return out


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("order", ["original", "tree", "tree_rmajor"])
def test_noalloc_equals_matvec_twice(meshes, storage, order):
    from paper_2209_07632_amd import HMatrix
    tol = 1e-6
    bound = tol + 1e-6 if storage == "f64" else tol + 1e-5
    mats = [HMatrix(v, f, tol=tol, storage=storage, max_rhs=15) for v, f, _ in meshes]
    for call, (H, R) in enumerate(((mats[0], 7), (mats[1], 3))):
        F = meshes[call][2]
        X = np.random.default_rng(10 * call + R).random((H.N, R))
        print(f"[noalloc] call {call} storage={storage} order={order} N={H.N} R={R}", flush=True)
        Xd = _layout(H, X, order, R)
        Y_ref = torch.full_like(Xd, np.nan)
        Y_na = torch.full_like(Xd, np.nan)
        H.matvec(Xd, out=Y_ref, order=order, R=R)
        H.matvec_noalloc(Xd, out=Y_na, order=order, R=R)
        torch.cuda.synchronize()
        a, b = _back(H, Y_na, order, R), _back(H, Y_ref, order, R)
        assert np.array_equal(a, b), f"call {call}: max diff {np.max(np.abs(a - b))}"
        err = np.linalg.norm(a - F @ X) / np.linalg.norm(F @ X)
        assert err <= bound, err
    for H in mats:
        H.close()


def test_noalloc_refuses_what_the_scratch_cannot_hold(meshes):
    from paper_2209_07632_amd import HMatrix
    from paper_2209_07632_amd.rad import RAD_EINVAL, RadError, load
    limit = load().rad_noalloc_scratch_bytes()
    assert limit == 8 << 20
    v, f, _ = meshes[0]
    H = HMatrix(v, f, tol=1e-3, storage="f64", max_rhs=1)
    for R in (0, 16):
        # column-major (N, max(R, 1)) blocks, leading dimension N
        X = torch.zeros((max(R, 1), H.N), dtype=torch.float64, device=DEV).t()
        Y = torch.zeros((max(R, 1), H.N), dtype=torch.float64, device=DEV).t()
        with pytest.raises(RadError) as e:
            H.matvec_noalloc(X[:, :R], out=Y, order="tree")
        assert e.value.status == RAD_EINVAL
    H.close()
    # 40,017 facets x 15 columns x 8 bytes, twice, exceeds the array for the
    # original order (9.6 MB); in tree order only the projections are needed
    vL, fL = cap_mesh(CAP_LARGE)
    HL = HMatrix(vL, fL, tol=1e-2, storage="f64", max_rhs=1)
    X = torch.rand((HL.N, 15), dtype=torch.float64, device=DEV).t().contiguous().t()
    Y = torch.zeros_like(X)
    with pytest.raises(RadError) as e:
        HL.matvec_noalloc(X, out=Y, order="original")
    assert e.value.status == RAD_EINVAL and "scratch" in str(e.value)
    HL.matvec_noalloc(X, out=Y, order="tree")
    # the same matrix built with workspace for 15 columns: both entry points
    # agree bit for bit; the max_rhs = 1 build agrees within its tolerance
    HW = HMatrix(vL, fL, tol=1e-2, storage="f64", max_rhs=15)
    Y_ref, Y2 = torch.zeros_like(X), torch.zeros_like(X)
    HW.matvec(X, out=Y_ref, order="tree")
    HW.matvec_noalloc(X, out=Y2, order="tree")
    torch.cuda.synchronize()
    assert torch.equal(Y2, Y_ref)
    assert (torch.linalg.norm(Y - Y_ref) / torch.linalg.norm(Y_ref)).item() < 1e-2
    HW.close()
    HL.close()
