"""Host logic on the CPU: two numerical routines of librad's builder.

The one-sided Jacobi SVD that the rank search (Algorithm 3) runs on each
block's small factor is checked against LAPACK's singular values, the
reconstruction A = (U Sigma) V^T and the orthogonality of V, on random,
graded and rank-deficient matrices.  The facet geometry (centroid, normal by
the right-hand rule, area) is checked against the reference's."""
import subprocess

import numpy as np
import pytest

from host_build import compile_harness
from oracle import reference as ref
from synth import BodySpec, CapSpec, body_mesh, cap_mesh


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    return compile_harness("builder_harness", tmp_path_factory.mktemp("builder"))


def _svd(exe, A):
    l = A.shape[0]
    text = f"{l}\n" + " ".join(repr(float(v)) for v in A.ravel(order="F")) + "\n"
    out = subprocess.run([exe, "svd"], input=text, capture_output=True, text=True, check=True).stdout.split("\n")
    sv = np.array(out[0].split(), dtype=np.float64)
    US = np.array(out[1].split(), dtype=np.float64).reshape(l, l, order="F")
    V = np.array(out[2].split(), dtype=np.float64).reshape(l, l, order="F")
    return sv, US, V


def _matrices():
    rng = np.random.default_rng(0)
    yield rng.standard_normal((1, 1))
    yield rng.standard_normal((2, 2))
    for l in (5, 16, 40):
        yield rng.standard_normal((l, l))
    # graded spectrum 1 .. 1e-14 and a rank-deficient block (rank 6 of 24)
    Q1, _ = np.linalg.qr(rng.standard_normal((24, 24)))
    Q2, _ = np.linalg.qr(rng.standard_normal((24, 24)))
    yield Q1 @ np.diag(np.logspace(0, -14, 24)) @ Q2.T
    yield rng.standard_normal((24, 6)) @ rng.standard_normal((6, 24))


def test_jacobi_svd_matches_lapack(harness):
    for A in _matrices():
        sv, US, V = _svd(harness, A)
        s0 = np.linalg.svd(A, compute_uv=False)
        assert np.all(np.diff(sv) <= 0)                                   # sorted, largest first
        assert np.max(np.abs(sv - s0)) <= 1e-13 * s0[0] * A.shape[0]
        assert np.max(np.abs(US @ V.T - A)) <= 1e-13 * s0[0] * A.shape[0]
        assert np.max(np.abs(V.T @ V - np.eye(A.shape[0]))) <= 1e-13 * A.shape[0]


def _geom(exe, v, f):
    text = f"{v.shape[0]} {f.shape[0]}\n" + " ".join(repr(float(a)) for a in v.ravel()) + "\n" + \
        " ".join(str(int(a)) for a in f.ravel()) + "\n"
    out = subprocess.run([exe, "geom"], input=text, capture_output=True, text=True, check=True).stdout
    return np.array(out.split(), dtype=np.float64).reshape(-1, 7)


@pytest.mark.parametrize("mesh", ["cap", "body"])
def test_facet_geometry_matches_reference(harness, mesh):
    v, f = cap_mesh(CapSpec(h=120.0, seed=3)) if mesh == "cap" else body_mesh(BodySpec(level=2))
    g = _geom(harness, v, f)
    fac = ref.Facets(v, f)
    scale = np.max(np.abs(v))
    assert np.max(np.abs(g[:, 0:3] - fac.x)) <= 1e-15 * scale
    assert np.max(np.abs(g[:, 3:6] - fac.n)) <= 1e-14
    np.testing.assert_allclose(g[:, 6], fac.A, rtol=1e-14)
