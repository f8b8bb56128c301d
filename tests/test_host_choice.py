"""Host logic on the CPU: librad's block choice (Algorithm 4) equals the
reference's on the same inputs.

The builder's pair enumeration and its bottom-up decision (fewest bytes among
zero / dense / CSR / low-rank / hierarchical, ties to the simpler form, then
coalescing) run in a host-only program.  They get the reference's non-zero
counts and the reference's Algorithm 3 ranks for every pair; the final
partition and the form of every block must equal the reference's assembly.
(The builder finds ranks with a randomized sketch on the GPU instead; that
part is checked by the GPU parity tests.)"""
import subprocess

import numpy as np
import pytest

from host_build import compile_harness
from oracle import hmatrix as hm
from oracle import reference as ref
from synth import BodySpec, CapSpec, body_mesh, cap_mesh

KINDS = {0: "zero", 1: "dense", 2: "csr", 3: "svd", 4: "hier"}


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    return compile_harness("choice_harness", tmp_path_factory.mktemp("choice"))


def _header(x, leaf, dims, s):
    return f"{x.shape[0]} {leaf} {dims} 0 {s}\n" + " ".join(repr(float(v)) for v in x.ravel()) + "\n"


def _product_blocks(exe, F, x, leaf, dims, eps, s):
    head = _header(x, leaf, dims, s)
    out = subprocess.run([exe, "pairs"], input=head, capture_output=True, text=True, check=True).stdout.split("\n")
    perm = np.array(out[0].split(), dtype=np.int64)
    npairs = int(out[1])
    lines = []
    for row in out[2:2 + npairs]:
        i0, m, j0, n, first, nchild, level = (int(v) for v in row.split())
        blk = F[np.ix_(perm[i0:i0 + m], perm[j0:j0 + n])]
        nnz = int(np.count_nonzero(blk))
        q, sb = 0, 0
        if first >= 0 and nnz > 0:
            est = hm.estimate_rank(blk, eps, s)
            if est is not None:
                q, sb = est[0], hm.svd_bytes(m, n, est[0], s)
        lines.append(f"{nnz} {q} {sb}")
    out = subprocess.run([exe, "decide"], input=head + "\n".join(lines) + "\n", capture_output=True, text=True,
                         check=True).stdout
    got = set()
    for row in out.strip().split("\n"):
        i0, m, j0, n, kind = (int(v) for v in row.split())
        got.add((tuple(sorted(perm[i0:i0 + m])), tuple(sorted(perm[j0:j0 + n])), KINDS[kind]))
    return got


def _reference_blocks(F, pts, leaf, eps, s):
    H = hm.assemble(F, pts, eps=eps, s=s, leaf_size=leaf)
    return {(tuple(sorted(b.rows)), tuple(sorted(b.cols)), b.kind) for b in hm.leaf_blocks(H)}


@pytest.mark.parametrize("eps", [1e-2, 1e-4])
def test_quadtree_choice_equals_reference(harness, eps):
    v, f = cap_mesh(CapSpec(h=120.0, seed=3))
    fac = ref.Facets(v, f)
    F = ref.view_factor_matrix(fac)
    got = _product_blocks(harness, F, fac.x, 32, 2, eps, 8)
    want = _reference_blocks(F, fac.x[:, :2], 32, eps, 8)
    assert got == want
    assert {k for *_, k in want} >= {"dense", "svd"}


def test_octree_choice_equals_reference(harness):
    v, f = body_mesh(BodySpec(level=3))
    fac = ref.Facets(v, f)
    F = ref.view_factor_matrix(fac, ref.pair_visibility(fac, "raycast"))
    got = _product_blocks(harness, F, fac.x, 32, 3, 1e-2, 4)
    want = _reference_blocks(F, fac.x, 32, 1e-2, 4)
    assert got == want
    assert {k for *_, k in want} >= {"zero", "csr"}
