"""Checks of the seeded synthetic inputs (geometry only)."""
import numpy as np

from synth import BodySpec, CapSpec, body_mesh, cap_mesh


def test_body_mesh_is_a_closed_consistently_wound_sphere():
    """Every edge is shared by exactly two faces that traverse it in opposite
    directions, and V - E + F = 2: a closed, orientable surface of genus 0."""
    v, f = body_mesh(BodySpec(level=3))
    assert f.shape[0] == 20 * 4 ** 3
    directed = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]])
    assert len({tuple(e) for e in directed}) == len(directed)          # no edge twice in one direction
    undirected = {tuple(sorted(e)) for e in directed}
    assert len(directed) == 2 * len(undirected)                          # each edge in two faces
    assert {tuple(e[::-1]) for e in directed} == {tuple(e) for e in directed}
    assert v.shape[0] - len(undirected) + f.shape[0] == 2


def test_body_mesh_outward_normals_and_waist():
    spec = BodySpec(level=3, radius=1000.0, neck=0.5)
    v, f = body_mesh(spec)
    c = v[f].mean(axis=1)
    n = np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]])
    assert np.all(np.einsum("ij,ij->i", n, c) > 0)                     # star-shaped, wound outward
    r = np.linalg.norm(v, axis=1)
    assert abs(r.max() - 1500.0) < 1e-9 and r.min() >= 500.0 - 1e-9


def test_generators_are_deterministic():
    a = cap_mesh(CapSpec(h=120.0, seed=3))
    b = cap_mesh(CapSpec(h=120.0, seed=3))
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert np.array_equal(body_mesh()[1], body_mesh()[1])
