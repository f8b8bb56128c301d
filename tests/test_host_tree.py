"""Host logic on the CPU: librad's tree builder (quadtree and octree) gives
the same facet permutation and leaves as the reference's Algorithm 2."""
import subprocess

import numpy as np
import pytest

from host_build import compile_harness
from oracle import hmatrix as hm
from oracle import reference as ref
from synth import BodySpec, CapSpec, body_mesh, cap_mesh


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    return compile_harness("tree_harness", tmp_path_factory.mktemp("tree"))


def _tree(exe, x, leaf, dims):
    text = f"{x.shape[0]} {leaf} {dims}\n" + " ".join(repr(float(v)) for v in x.ravel()) + "\n"
    out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout.split("\n")
    return int(out[0]), np.array(out[1].split(), dtype=np.int64), np.array(out[2].split(), dtype=np.int64)


@pytest.mark.parametrize("leaf", [16, 64])
def test_quadtree_equals_reference(harness, leaf):
    v, f = cap_mesh(CapSpec(h=90.0, seed=5))
    x = ref.Facets(v, f).x
    n, perm, _ = _tree(harness, x, leaf, 2)
    root = hm.quadtree(x[:, :2], leaf)
    assert n == len(list(hm.leaves(root)))
    assert np.array_equal(perm, hm.tree_permutation(root))


@pytest.mark.parametrize("leaf", [16, 32])
def test_octree_equals_reference(harness, leaf):
    v, f = body_mesh(BodySpec(level=3))
    x = ref.Facets(v, f).x
    n, perm, spans = _tree(harness, x, leaf, 3)
    root = hm.octree(x, leaf)
    leaves = list(hm.leaves(root))
    assert n == len(leaves)
    assert np.array_equal(perm, hm.tree_permutation(root))
    spans = spans.reshape(-1, 2)
    spans = spans[np.argsort(spans[:, 0])]            # leaves by first facet = depth-first order
    assert np.array_equal(spans[:, 1], [lf.size for lf in leaves])
    assert np.array_equal(spans[:, 0], np.cumsum([0] + [lf.size for lf in leaves[:-1]]))


def test_coincident_centroids_stay_one_leaf(harness):
    x = np.tile([[1.0, 2.0, 3.0]], (50, 1))
    for dims in (2, 3):
        n, perm, _ = _tree(harness, x, 8, dims)
        assert n == 1 and np.array_equal(perm, np.arange(50))
