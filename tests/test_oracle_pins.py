"""Pins of the CPU reference against facts fixed by the paper or by mathematics.

Each test checks the reference against something other than itself: a
closed form, an invariant, a special case with a textbook answer, or brute
force.  A plausible slip in the reference (a dropped term, a wrong sign or
index, a transposed operand) fails at least one of them.
"""
import numpy as np
import pytest

from oracle import hmatrix as hm
from oracle import reference as ref
from synth import CAP_SMALL, CapSpec, cap_mesh


def sphere_facets(N, r=2.0, seed=0):
    """Centroids on a sphere with inward radial normals and random areas."""
    rng = np.random.default_rng(seed)
    p = rng.standard_normal((N, 3))
    p /= np.linalg.norm(p, axis=1, keepdims=True)
    x = r * p
    n = -p
    A = rng.uniform(0.5, 1.5, N) * 1e-2
    return ref.Facets.from_arrays(x, n, A)


# ---------------------------------------------------------------- P1, eq. FF-def
def test_sphere_kernel_is_constant():
    """On a sphere with inward normals the kernel of eq. FF-def is A_j / (4 pi r^2) exactly."""
    r = 2.0
    fac = sphere_facets(300, r=r)
    F = ref.view_factor_matrix(fac)
    expect = np.tile(fac.A / (4 * np.pi * r * r), (fac.N, 1))
    np.fill_diagonal(expect, 0.0)
    assert np.max(np.abs(F - expect) / expect.max()) < 1e-12


# ---------------------------------------------------------------- P2, Jacobi
@pytest.mark.parametrize("rho", [0.3, 1.0])
def test_jacobi_sherman_morrison(rho):
    """F = c(1 A^T - diag A) gives (I - rho F)B = E in closed form (Sherman-Morrison)."""
    r = 2.0
    fac = sphere_facets(400, r=r, seed=1)
    F = ref.view_factor_matrix(fac)
    c = 1.0 / (4 * np.pi * r * r)
    E = np.random.default_rng(2).uniform(0.0, 10.0, (fac.N, 3))
    D = 1.0 + rho * c * fac.A
    s = (fac.A @ (E / D[:, None])) / (1.0 - rho * c * np.sum(fac.A / D))
    B_exact = (E + rho * c * s[None, :]) / D[:, None]
    B, iters = ref.jacobi(lambda X: F @ X, rho, E, tol=1e-15)
    assert np.max(np.abs(B - B_exact)) / np.max(np.abs(B_exact)) < 1e-13
    assert np.all(iters > 0)


# ---------------------------------------------------------------- P3, section 7.1
def test_closed_form_constants_agree():
    """The two printed forms of the shadowed-crater temperature are the same number,
    and f equals sin^2(beta/2), the view factor of a spherical cap seen from itself."""
    alpha, emiss, S, e = 0.3, 0.99, 1365.0, 15.0
    f = ref.crater_f(5.0)  # D/d = 5
    T1 = ref.crater_shadow_temperature(S, e, alpha, emiss, f)
    T2 = ref.crater_temperature(S, np.sin(np.deg2rad(e)), 0.0, True, alpha, emiss, f)
    assert abs(T1 - T2) < 1e-10 * T1
    rc, d = 1000.0, 400.0
    r = (rc * rc + d * d) / (2 * d)
    beta = np.arcsin(rc / r)           # half-angle of the cap seen from the sphere centre
    assert abs(f - np.sin(beta / 2) ** 2) < 1e-14 * 10 and abs(f - 1 / 7.25) < 1e-15


def _cap_temperature(spec):
    v, f = cap_mesh(spec)
    fac = ref.Facets(v, f)
    F = ref.view_factor_matrix(fac)
    e = 15.0
    s = np.array([[np.cos(np.deg2rad(e)), 0.0, np.sin(np.deg2rad(e))]])
    Q = ref.insolation(fac, s, S=1365.0)
    out = ref.equilibrium_temperature(lambda X: F @ X, Q, 0.3, 0.99)
    shadow = Q[:, 0] == 0.0
    fcr = ref.crater_f(5.0)
    Tc = ref.crater_temperature(1365.0, np.sin(np.deg2rad(e)), fac.n @ s[0], shadow,
                                0.3, 0.99, fcr)
    rel = np.abs(out["T"][:, 0] - Tc) / Tc
    return rel, shadow


def test_cap_matches_closed_form():
    """Discrete equilibrium T on the ~1,600-facet bowl vs the closed form of section 7.1."""
    rel, shadow = _cap_temperature(CAP_SMALL)
    assert 0.4 < shadow.mean() < 0.8
    assert rel[shadow].mean() < 5e-3 and rel[shadow].max() < 3e-2
    assert rel[~shadow].mean() < 2e-3


@pytest.mark.slow
def test_cap_converges_to_closed_form():
    """Halving the mesh spacing shrinks the shadowed-region error (first-order scheme)."""
    rel1, sh1 = _cap_temperature(CAP_SMALL)
    rel2, sh2 = _cap_temperature(CapSpec(h=CAP_SMALL.h / 2))
    assert rel2[sh2].mean() < 0.7 * rel1[sh1].mean()


# ---------------------------------------------------------------- P4, P5
def test_reciprocity_and_row_sums():
    v, f = cap_mesh(CAP_SMALL)
    fac = ref.Facets(v, f)
    F = ref.view_factor_matrix(fac)
    M = fac.A[:, None] * F
    assert np.max(np.abs(M - M.T)) <= 1e-14 * M.max()
    rs = F.sum(axis=1)
    assert rs.max() < 1.0
    fcr = ref.crater_f(5.0)
    assert abs(rs.mean() - fcr) < 0.01 * fcr
    assert np.all(np.diag(F) == 0.0)


# ---------------------------------------------------------------- P6, section 3.2
def _tri(a, b, c):
    return np.array([a, b, c], dtype=np.float64).reshape(9)


def test_visibility_blocker():
    """Two facing facets; a triangle across the segment hides them, one beside does not."""
    x = np.array([[0, 0, 0], [0, 0, 2.0], [0, 0, 1.0], [5, 5, 1.0]], dtype=np.float64)
    n = np.array([[0, 0, 1], [0, 0, -1], [1, 0, 0], [1, 0, 0]], dtype=np.float64)
    A = np.ones(4)
    tris = np.stack([
        _tri([-.1, -.1, 0], [.1, -.1, 0], [0, .1, 0]),
        _tri([-.1, -.1, 2], [0, .1, 2], [.1, -.1, 2]),
        _tri([-1, -1, 1], [1, -1, 1], [0, 1, 1]),        # blocker across the segment
        _tri([4, 4, 1], [6, 4, 1], [5, 6, 1]),           # far away
    ])
    fac = ref.Facets.from_arrays(x, n, A, tris)
    vis = ref.pair_visibility(fac, "raycast")
    assert vis[0, 1] == 0 and vis[1, 0] == 0
    tris2 = tris.copy()
    tris2[2] = _tri([3, 3, 1], [4, 3, 1], [3, 4, 1])   # move the blocker aside
    fac2 = ref.Facets.from_arrays(x, n, A, tris2)
    assert ref.pair_visibility(fac2, "raycast")[0, 1] == 1
    # a hit exactly on the blocker's edge still blocks (edges are inclusive)
    tris3 = tris.copy()
    tris3[2] = _tri([0, 0, 1], [1, 0, 1], [0, 1, 1])   # vertex on the segment
    fac3 = ref.Facets.from_arrays(x, n, A, tris3)
    assert ref.pair_visibility(fac3, "raycast")[0, 1] == 0
    # back-face culling: facet 3 faces +x, away from facet 0's column
    assert vis[0, 3] == 0 or np.dot(n[3], x[0] - x[3]) > 0


def test_convex_bowl_all_facing_pairs_visible():
    """Inside a convex bowl no segment between facets leaves the bowl: brute-force
    ray casting and the back-face test agree on every pair."""
    v, f = cap_mesh(CapSpec(h=120.0, seed=3))
    fac = ref.Facets(v, f)
    assert np.array_equal(ref.pair_visibility(fac, "raycast"), ref.pair_visibility(fac, "backface"))


def test_bowl_shadow_matches_sphere():
    """Sun shadowing on the meshed bowl agrees with the exact sphere away from the
    shadow line: a ray from a point on the bowl leaves through the opening iff its
    second intersection with the sphere lies above the rim plane."""
    spec = CAP_SMALL
    v, f = cap_mesh(spec)
    fac = ref.Facets(v, f)
    r, d = spec.sphere_radius, spec.depth
    c = np.array([0.0, 0.0, r - d])
    e = np.deg2rad(15.0)
    s = np.array([np.cos(e), 0.0, np.sin(e)])
    lit = ref.sun_visibility(fac, s[None, :])[:, 0].astype(bool)
    p = fac.x - c
    b = p @ s
    disc = b * b - (np.sum(p * p, axis=1) - r * r)
    t2 = -b + np.sqrt(np.maximum(disc, 0.0))
    zexit = fac.x[:, 2] + t2 * s[2]
    margin = 0.4 * spec.h * s[2]
    facing = fac.n @ s > 0.05          # facets turned away are dark by the cosine factor
    sure_lit = facing & (zexit > margin)
    sure_dark = facing & (zexit < -margin)
    assert sure_lit.sum() > 100 and sure_dark.sum() > 100
    assert np.all(lit[sure_lit]) and not np.any(lit[sure_dark])


# ---------------------------------------------------------------- P7
def test_jacobi_matches_lapack():
    v, f = cap_mesh(CAP_SMALL)
    fac = ref.Facets(v, f)
    F = ref.view_factor_matrix(fac)
    E = np.random.default_rng(3).uniform(0, 100, (fac.N, 2))
    for rho in (0.3, 1.0):
        B, _ = ref.jacobi(lambda X: F @ X, rho, E, tol=1e-14)
        B2 = ref.solve_direct(F, rho, E)
        assert np.linalg.norm(B - B2) / np.linalg.norm(B2) < 1e-12


# ---------------------------------------------------------------- P9
def test_flat_plane_has_no_exchange():
    g = np.linspace(0, 1, 9)
    X, Y = np.meshgrid(g, g, indexing="ij")
    verts = np.column_stack([X.ravel(), Y.ravel(), np.zeros(X.size)])
    m = g.size
    faces = []
    for i in range(m - 1):
        for j in range(m - 1):
            a, b, c, d = i * m + j, (i + 1) * m + j, (i + 1) * m + j + 1, i * m + j + 1
            faces += [[a, b, c], [a, c, d]]
    fac = ref.Facets(verts, np.array(faces, dtype=np.int32))
    F = ref.view_factor_matrix(fac, ref.pair_visibility(fac, "raycast"))
    assert np.all(F == 0.0)
    E = np.ones((fac.N, 1))
    B, iters = ref.jacobi(lambda X: F @ X, 0.5, E)
    assert np.array_equal(B, E) and iters[0] == 1


def test_matvec_free_matches_dense():
    v, f = cap_mesh(CapSpec(h=100.0, seed=5))
    fac = ref.Facets(v, f)
    F = ref.view_factor_matrix(fac)
    X = np.random.default_rng(0).random((fac.N, 3))
    np.testing.assert_allclose(ref.matvec_free(fac, X), F @ X, rtol=1e-13, atol=0)
    rows = np.array([0, 5, fac.N - 1])
    np.testing.assert_array_equal(ref.view_factor_rows(fac, rows), F[rows])



def grazing_pairs(M=200, seed=0):
    """M far-apart facet pairs (a, b), each with a third triangle whose edge
    crosses the midpoint of the segment a-b.  Mathematically the segment
    touches the edge (a hit: edges count); in FP64 the rounding of the two
    directions of the ray test can disagree, which is what the test needs."""
    rng = np.random.default_rng(seed)
    x, n, A, tri = [], [], [], []
    for m in range(M):
        off = np.array([100.0 * m, 0.0, 0.0])
        a = off + rng.uniform(-0.3, 0.3, 3)
        b = off + np.array([1.0, 0.0, 0.0]) + rng.uniform(-0.3, 0.3, 3)
        d = b - a
        p = a + 0.5 * d
        e = np.cross(d, rng.standard_normal(3))
        e /= np.linalg.norm(e)
        q = np.cross(d, e)
        q /= np.linalg.norm(q)
        dn = d / np.linalg.norm(d)
        na = dn + 0.3 * rng.standard_normal(3)
        nb = -dn + 0.3 * rng.standard_normal(3)
        v0, v1, v2 = p + 0.25 * e, p - 0.25 * e, p + rng.uniform(0.2, 0.6) * q
        kn = np.cross(v1 - v0, v2 - v0)
        small = np.array([[0, 0.01, 0], [0.01, 0, 0], [0, 0, 0.01]])
        x += [a, b, (v0 + v1 + v2) / 3]
        n += [na / np.linalg.norm(na), nb / np.linalg.norm(nb), kn / np.linalg.norm(kn)]
        A += [1e-2, 1e-2, 1e-2]
        tri += [(a + small).ravel(), (b + small).ravel(), np.concatenate([v0, v1, v2])]
    return ref.Facets.from_arrays(np.array(x), np.array(n), np.array(A), np.array(tri))


def test_raycast_rows_cast_once_per_pair():
    """Section 3.2, reading 12: rows evaluated on the fly use the same
    visibility as the dense F, the segment cast once per unordered pair from
    the smaller index.  On grazing pairs the two directions of the cast
    disagree, so a row cast from its own facet would differ from F."""
    fac = grazing_pairs()
    D = ref.directed_visibility(fac)
    asym = np.argwhere(np.triu(D != D.T))
    assert len(asym) >= 10                       # the fixture has teeth
    V = ref.pair_visibility(fac, "raycast")
    assert np.array_equal(V, V.T)
    F = ref.view_factor_matrix(fac, V)
    rows = np.unique(asym.ravel())
    Fr = ref.view_factor_rows(fac, rows, "raycast")
    np.testing.assert_array_equal(Fr, F[rows])
    # casting each row from its own facet is the row-directed matrix, not F
    assert not np.array_equal(ref.view_factor_matrix(fac, D)[rows], F[rows])
    # the smaller index decides: V equals the directed test read from above the diagonal
    iu = np.triu_indices(fac.N, 1)
    assert np.array_equal(V[iu], D[iu])


def test_raycast_rows_on_terrain():
    from synth import DemSpec, dem_mesh
    v, f = dem_mesh(DemSpec(n=16, seed=3))
    fac = ref.Facets(v, f)
    F = ref.view_factor_matrix(fac, ref.pair_visibility(fac, "raycast"))
    assert np.count_nonzero(F) < np.count_nonzero(ref.view_factor_matrix(fac))   # something is occluded
    rows = np.arange(0, fac.N, 7)
    np.testing.assert_array_equal(ref.view_factor_rows(fac, rows, "raycast"), F[rows])


def test_matvec_free_with_visibility():
    """The matrix-free product with a visibility matrix equals the pinned
    dense F with the same visibility, on occluded terrain and on grazing
    pairs; an all-zero V gives zero, an all-one V the back-face product."""
    from synth import DemSpec, dem_mesh
    v, f = dem_mesh(DemSpec(n=12, seed=1))
    for fac in (ref.Facets(v, f), grazing_pairs(60, seed=1)):
        V = ref.pair_visibility(fac, "raycast")
        F = ref.view_factor_matrix(fac, V)
        X = np.random.default_rng(4).random((fac.N, 3))
        np.testing.assert_allclose(ref.matvec_free(fac, X, V), F @ X, rtol=1e-13, atol=0)
        assert np.all(ref.matvec_free(fac, X, np.zeros_like(V)) == 0.0)
        np.testing.assert_allclose(ref.matvec_free(fac, X, np.ones_like(V)), ref.matvec_free(fac, X),
                                   rtol=1e-15, atol=0)
        # a single blocked pair removes exactly its two terms
        i, j = np.argwhere(np.triu(V, 1))[0]
        V2 = V.copy()
        V2[i, j] = V2[j, i] = 0
        dY = ref.matvec_free(fac, X, V) - ref.matvec_free(fac, X, V2)
        expect = np.zeros_like(X)
        expect[i] = F[i, j] * X[j]
        expect[j] = F[j, i] * X[i]
        np.testing.assert_allclose(dY, expect, rtol=1e-12, atol=1e-15 * np.abs(F @ X).max())


# ---------------------------------------------------------------- Algorithm 4 by hand
def _two_level(rows, half):
    """A node over `rows` with two leaf children of `half` rows each."""
    return hm.Node(idx=np.asarray(rows), depth=0,
                   children=[hm.Node(idx=np.asarray(rows[:half]), depth=1),
                             hm.Node(idx=np.asarray(rows[half:]), depth=1)])


def _block_of(Fb):
    """Place an 8 x 8 block at rows 0..7, columns 8..15 of a 16 x 16 F."""
    F = np.zeros((16, 16))
    F[:8, 8:] = Fb
    return F, _two_level(list(range(8)), 4), _two_level(list(range(8, 16)), 4)


def test_assembly_choice_by_hand():
    """Algorithm 4 with eq. nbytes-comparison (value s = 8 bytes, index 4),
    each expected form and byte count worked out by hand; leaf_size 2, so the
    8 x 8 pair is not a leaf pair and its 4 x 4 children are."""
    s, ls = 8, 2
    rng = np.random.default_rng(7)
    # all-zero block: a zero block of no bytes
    F, I, J = _block_of(np.zeros((8, 8)))
    b = hm.assemble_block(F, I, J, 1e-3, s, ls)
    assert b.kind == "zero" and b.nbytes == 0
    # exactly rank one, no zeros: SVD of (m + n) q s + q s = 136 bytes beats
    # dense 512, CSR 4*9 + 64*12 = 804 and the four dense children (512)
    u, v = rng.uniform(0.5, 1.5, 8), rng.uniform(0.5, 1.5, 8)
    F, I, J = _block_of(np.outer(u, v))
    b = hm.assemble_block(F, I, J, 1e-3, s, ls)
    assert b.kind == "svd" and b.nbytes == (8 + 8 + 1) * 8
    U, sv, V = b.data
    assert U.shape == (8, 1)
    np.testing.assert_allclose((U * sv) @ V.T, np.outer(u, v), rtol=1e-13)
    # random full-rank dense block: dense 512 ties with the four dense
    # children (4 x 128); the tie goes to the simpler dense form
    F, I, J = _block_of(rng.uniform(0.5, 1.5, (8, 8)))
    b = hm.assemble_block(F, I, J, 1e-3, s, ls)
    assert b.kind == "dense" and b.nbytes == 512
    # eight scattered non-zeros of full rank: CSR 4*9 + 8*12 = 132; children
    # are CSR 4*5 + 2*12 = 44 each (176); dense 512; SVD would need q = 8
    Fb = np.zeros((8, 8))
    perm = [1, 0, 3, 2, 5, 4, 7, 6]
    for r in range(8):
        Fb[r, perm[r]] = 1.0 + r
    F, I, J = _block_of(Fb)
    b = hm.assemble_block(F, I, J, 1e-3, s, ls)
    assert b.kind == "csr" and b.nbytes == 132
    # non-zeros only inside one child (3 on its diagonal): that child is CSR
    # 4*5 + 3*12 = 56, the rest zero, so the hierarchical form (56) beats
    # CSR 4*9 + 3*12 = 72; children all CSR or zero coalesce into one CSR
    # block over the whole pair, of 72 bytes
    Fb = np.zeros((8, 8))
    Fb[5, 4], Fb[6, 6], Fb[7, 5] = 2.0, 3.0, 5.0
    F, I, J = _block_of(Fb)
    b = hm.assemble_block(F, I, J, 1e-3, s, ls)
    assert b.kind == "csr" and b.nbytes == 72
    assert np.array_equal(b.rows, np.arange(8)) and np.array_equal(b.cols, np.arange(8, 16))
    # a full child (dense 128) and one non-zero in the opposite child (CSR
    # 4*5 + 12 = 32): hierarchical 160 beats CSR 4*9 + 17*12 = 240, dense 512
    # and SVD (rank 5: 16*5*8 + 40 = 680); mixed children are not coalesced
    Fb = np.zeros((8, 8))
    Fb[:4, :4] = rng.uniform(0.5, 1.5, (4, 4))
    Fb[6, 5] = 1.0
    F, I, J = _block_of(Fb)
    b = hm.assemble_block(F, I, J, 1e-3, s, ls)
    assert b.kind == "hier" and b.nbytes == 160
    assert [c.kind for c in b.data] == ["dense", "zero", "zero", "csr"]
    assert [c.nbytes for c in b.data] == [128, 0, 0, 32]
    # one full child and three zero children: hierarchical 128 beats CSR
    # 4*9 + 16*12 = 228; children dense and zero are not coalesced (a dense
    # block over the pair would cost 512)
    Fb = np.zeros((8, 8))
    Fb[4:, 4:] = rng.uniform(0.5, 1.5, (4, 4))
    F, I, J = _block_of(Fb)
    b = hm.assemble_block(F, I, J, 1e-3, s, ls)
    assert b.kind == "hier" and b.nbytes == 128
    assert [c.kind for c in b.data] == ["zero", "zero", "zero", "dense"]
    # CSR ties the hierarchical form: a child with 11 non-zeros (dense 128 <
    # CSR 20 + 11*12), two children with one non-zero (CSR 32 each), one
    # zero: hierarchical 192 = CSR 4*9 + 13*12 = 192 (rank >= 2, so SVD >= 272);
    # the tie goes to the simpler CSR form
    Fb = np.zeros((8, 8))
    cells = [(r, c) for r in range(4) for c in range(4)][:11]
    for k, (r, c) in enumerate(cells):
        Fb[r, c] = 1.0 + 0.1 * k
    Fb[1, 6], Fb[6, 2] = 4.0, 5.0
    F, I, J = _block_of(Fb)
    b = hm.assemble_block(F, I, J, 1e-3, s, ls)
    assert b.kind == "csr" and b.nbytes == 192
    # (children all dense tie the dense form exactly, so the dense coalescing
    # and the tie rule give the same block there)


def test_assembly_splits_the_non_leaf_side():
    """Reading 5: a leaf row node against an internal column node is not a
    leaf pair while |I||J| exceeds leaf_size^2; only J splits.  An exactly
    rank-one 8 x 8 block then becomes an SVD of (8 + 8 + 1) * 8 = 136 bytes,
    not the leaf choice (dense 512)."""
    rng = np.random.default_rng(9)
    F, _, J = _block_of(np.outer(rng.uniform(0.5, 1.5, 8), rng.uniform(0.5, 1.5, 8)))
    leaf_i = hm.Node(idx=np.arange(8), depth=1)
    b = hm.assemble_block(F, leaf_i, J, 1e-3, 8, 2)
    assert b.kind == "svd" and b.nbytes == 136
    # at leaf_size 8 the same pair is a leaf pair (64 <= 8^2): dense 512
    b = hm.assemble_block(F, leaf_i, J, 1e-3, 8, 8)
    assert b.kind == "dense" and b.nbytes == 512


def test_leaf_choice_tie_goes_to_dense():
    """A 1 x 4 leaf block with two non-zeros: dense 4*8 = 32 bytes equals CSR
    4*2 + 2*12 = 32; the tie goes to the simpler dense form.  One more
    column (dense 40 vs CSR 32) makes CSR strictly smaller."""
    leaf_i = hm.Node(idx=np.array([0]), depth=0)
    F = np.zeros((6, 6))
    F[0, 1], F[0, 3] = 1.0, 2.0
    b = hm.assemble_block(F, leaf_i, hm.Node(idx=np.array([1, 2, 3, 4]), depth=0), 1e-3, 8, 64)
    assert b.kind == "dense" and b.nbytes == 32
    b = hm.assemble_block(F, leaf_i, hm.Node(idx=np.array([1, 2, 3, 4, 5]), depth=0), 1e-3, 8, 64)
    assert b.kind == "csr" and b.nbytes == 32

# ---------------------------------------------------------------- H-matrix reference
def test_quadtree_partition():
    v, f = cap_mesh(CAP_SMALL)
    fac = ref.Facets(v, f)
    root = hm.quadtree(fac.x[:, :2], leaf_size=64)
    perm = hm.tree_permutation(root)
    assert np.array_equal(np.sort(perm), np.arange(fac.N))
    for lf in hm.leaves(root):
        assert 1 <= lf.size <= 64

    def check(node):
        if node.is_leaf:
            return
        p = fac.x[node.idx, :2]
        xmid = 0.5 * (p[:, 0].min() + p[:, 0].max())
        ymid = 0.5 * (p[:, 1].min() + p[:, 1].max())
        for c in node.children:
            q = fac.x[c.idx, :2]
            assert np.all(q[:, 0] < xmid) or np.all(q[:, 0] >= xmid)
            assert np.all(q[:, 1] < ymid) or np.all(q[:, 1] >= ymid)
            check(c)
    check(root)


def test_rank_rule_on_known_spectrum():
    rng = np.random.default_rng(0)
    m, n = 120, 90
    U, _ = np.linalg.qr(rng.standard_normal((m, 40)))
    V, _ = np.linalg.qr(rng.standard_normal((n, 40)))
    sv = np.array([1.0, 0.5, 0.1, 0.01, 0.001] + [1e-6] * 35)
    A = (U * sv) @ V.T
    q, *_ = hm.estimate_rank(A, 0.05, 8)
    assert q == 3                      # sigma_4 / sigma_1 = 0.01 is the first below 0.05
    q, *_ = hm.estimate_rank(A, 2e-3, 8)
    assert q == 4
    q, *_ = hm.estimate_rank(A, 1e-7, 8)
    assert q == 40                     # beyond the rank sigma is 0
    # a rank that does not pay for itself in bytes fails
    full = rng.standard_normal((40, 40))
    assert hm.estimate_rank(full, 1e-12, 8) is None


def test_hmatrix_exact_sphere_blocks_rank_one():
    """Off-diagonal blocks of the sphere kernel are exactly rank one."""
    fac = sphere_facets(600, seed=4)
    F = ref.view_factor_matrix(fac)
    # project the sphere to 2D by longitude/latitude for the quadtree
    xy = np.column_stack([np.arctan2(fac.x[:, 1], fac.x[:, 0]), fac.x[:, 2]])
    H = hm.assemble(F, xy, eps=1e-8, leaf_size=32)
    for b in hm.leaf_blocks(H):
        if b.kind == "svd" and not np.intersect1d(b.rows, b.cols).size:
            assert b.data[0].shape[1] == 1
    X = np.random.default_rng(1).random((fac.N, 2))
    Y = hm.multiply(H, X)
    assert np.linalg.norm(Y - F @ X) / np.linalg.norm(F @ X) < 1e-7


def test_hmatrix_tiles_matrix_and_error_tracks_eps():
    v, f = cap_mesh(CapSpec(h=90.0, seed=11))
    fac = ref.Facets(v, f)
    F = ref.view_factor_matrix(fac)
    xy = fac.x[:, :2]
    X = np.random.default_rng(2).random((fac.N, 4))
    Y0 = F @ X
    prev = None
    for eps in (1e-2, 1e-4, 1e-6):
        H = hm.assemble(F, xy, eps=eps)
        blocks = hm.leaf_blocks(H)
        cover = np.zeros((fac.N, fac.N), dtype=np.int32)
        for b in blocks:
            cover[np.ix_(b.rows, b.cols)] += 1
        assert np.all(cover == 1)
        err = np.linalg.norm(hm.multiply(H, X) - Y0) / np.linalg.norm(Y0)
        assert err <= eps
        if prev is not None:
            assert H.nbytes() >= prev
        prev = H.nbytes()
    H = hm.assemble(F, xy, eps=1e-15)
    np.testing.assert_allclose(hm.multiply(H, X), Y0, rtol=1e-10)


# ---------------------------------------------------------------- octree, sections 4.1 and 8
def test_octree_partition():
    """Every child of an octree node lies on one side of each of the node's three
    mid-planes; leaves hold 1..leaf_size facets and partition the body."""
    from synth import BodySpec, body_mesh
    v, f = body_mesh(BodySpec(level=3))
    fac = ref.Facets(v, f)
    root = hm.octree(fac.x, leaf_size=32)
    perm = hm.tree_permutation(root)
    assert np.array_equal(np.sort(perm), np.arange(fac.N))
    assert all(1 <= lf.size <= 32 for lf in hm.leaves(root))
    assert max(len(n.children) for n in _nodes(root)) == 8

    def check(node):
        if node.is_leaf:
            return
        p = fac.x[node.idx]
        mid = 0.5 * (p.min(axis=0) + p.max(axis=0))
        for c in node.children:
            q = fac.x[c.idx]
            for a in range(3):
                assert np.all(q[:, a] < mid[a]) or np.all(q[:, a] >= mid[a])
            check(c)
    check(root)


def _nodes(node):
    yield node
    for c in node.children:
        yield from _nodes(c)


def test_octree_of_flat_points_is_the_quadtree():
    """With every centroid at one height the z split never separates anything,
    and the octree has the quadtree's leaves in the quadtree's order."""
    v, f = cap_mesh(CAP_SMALL)
    fac = ref.Facets(v, f)
    flat = np.column_stack([fac.x[:, :2], np.full(fac.N, 7.0)])
    a = [lf.idx for lf in hm.leaves(hm.octree(flat, leaf_size=40))]
    b = [lf.idx for lf in hm.leaves(hm.quadtree(fac.x[:, :2], leaf_size=40))]
    assert len(a) == len(b) and all(np.array_equal(x, y) for x, y in zip(a, b))


def test_octree_sphere_blocks_rank_one():
    """Inside a sphere the kernel is A_j / (4 pi r^2): with the octree on the
    3-D centroids every off-diagonal low-rank block has rank one."""
    fac = sphere_facets(700, seed=6)
    F = ref.view_factor_matrix(fac)
    H = hm.assemble(F, fac.x, eps=1e-8, leaf_size=32)
    svd = [b for b in hm.leaf_blocks(H) if b.kind == "svd" and not np.intersect1d(b.rows, b.cols).size]
    assert svd and all(b.data[0].shape[1] == 1 for b in svd)
    X = np.random.default_rng(3).random((fac.N, 2))
    assert np.linalg.norm(hm.multiply(H, X) - F @ X) / np.linalg.norm(F @ X) < 1e-7


def test_convex_body_seen_from_outside_has_no_exchange():
    """Outward normals on a convex closed body: no facet faces another, so F = 0
    and the compressed matrix is all zero blocks of no bytes."""
    from synth import BodySpec, body_mesh
    v, f = body_mesh(BodySpec(level=2, neck=0.0))
    fac = ref.Facets(v, f)
    F = ref.view_factor_matrix(fac)
    assert not F.any()
    H = hm.assemble(F, fac.x, eps=1e-3, leaf_size=16)
    assert H.nbytes() == 0 and {b.kind for b in hm.leaf_blocks(H)} == {"zero"}


def test_bilobed_body_is_zero_block_heavy_and_error_tracks_eps():
    """The closed two-lobed body (ray-cast visibility) compressed on an octree:
    blocks tile F once, the product error stays below eps, zero blocks cover
    over a quarter of the matrix (about a third here; on the all-visible
    crater none) and the bytes are a small fraction of dense storage."""
    from synth import BodySpec, body_mesh
    v, f = body_mesh(BodySpec(level=3))
    fac = ref.Facets(v, f)
    F = ref.view_factor_matrix(fac, ref.pair_visibility(fac, "raycast"))
    assert 0.01 < np.count_nonzero(F) / F.size < 0.1
    X = np.random.default_rng(4).random((fac.N, 3))
    Y0 = F @ X
    for eps in (1e-2, 1e-4):
        H = hm.assemble(F, fac.x, eps=eps, leaf_size=32)
        blocks = hm.leaf_blocks(H)
        cover = np.zeros(F.shape, dtype=np.int32)
        for b in blocks:
            cover[np.ix_(b.rows, b.cols)] += 1
        assert np.all(cover == 1)
        assert np.linalg.norm(hm.multiply(H, X) - Y0) / np.linalg.norm(Y0) <= eps
        assert sum(b.rows.size * b.cols.size for b in blocks if b.kind == "zero") > 0.25 * F.size
        assert H.nbytes() < 0.1 * F.size * 8


# ---------------------------------------------------------------- Chebyshev acceleration
@pytest.fixture(scope="module")
def hemisphere_bowl():
    """Bowl with depth / diameter 0.5 (f = 1/2): Jacobi converges only as 2^-k."""
    v, f = cap_mesh(CapSpec(h=90.0, depth_ratio=0.5, seed=2))
    fac = ref.Facets(v, f)
    return fac, ref.view_factor_matrix(fac)


def test_view_factor_spectrum_is_real(hemisphere_bowl):
    """Reciprocity makes diag(A) F symmetric, so F is self-adjoint in the
    area-weighted inner product and its eigenvalues are real, with the Perron
    root below the largest row sum."""
    fac, F = hemisphere_bowl
    AF = fac.A[:, None] * F
    assert np.max(np.abs(AF - AF.T)) <= 1e-14 * np.max(AF)
    ev = np.linalg.eigvals(F)
    assert np.max(np.abs(ev.imag)) <= 1e-12
    assert 0.45 < ev.real.max() <= F.sum(axis=1).max()


def test_chebyshev_matches_lapack_and_beats_jacobi(hemisphere_bowl):
    fac, F = hemisphere_bowl
    ev = np.linalg.eigvals(F).real
    E = np.random.default_rng(7).random((fac.N, 3))
    Bd = ref.solve_direct(F, 1.0, E)
    B, it = ref.chebyshev(lambda X: F @ X, 1.0, E, ev.min(), ev.max(), tol=1e-13)
    assert np.max(np.abs(B - Bd)) <= 1e-12 * np.max(np.abs(Bd))
    _, itj = ref.jacobi(lambda X: F @ X, 1.0, E, tol=1e-13)
    assert np.all(it < 0.5 * itj)


def test_chebyshev_error_bound(hemisphere_bowl):
    """In the area-weighted norm the error after k iterations is at most the
    initial error over T_k(theta / delta), for the exact spectral interval and
    for the row-sum bound [-r, r]."""
    fac, F = hemisphere_bowl
    ev = np.linalg.eigvals(F).real
    r = F.sum(axis=1).max()
    E = np.random.default_rng(8).random((fac.N, 2))
    Bd = ref.solve_direct(F, 1.0, E)

    def anorm(x):
        return np.sqrt((fac.A[:, None] * x * x).sum(axis=0))

    e0 = anorm(E - Bd)
    for lo, hi in ((ev.min(), ev.max()), (-r, r)):
        theta, delta = 1.0 - 0.5 * (lo + hi), 0.5 * (hi - lo)
        for k in range(1, 16):
            Bk, _ = ref.chebyshev(lambda X: F @ X, 1.0, E, lo, hi, tol=0.0, max_iter=k, strict=False)
            bound = 1.0 / np.cosh(k * np.arccosh(theta / delta))
            assert np.all(anorm(Bk - Bd) / e0 <= bound * (1 + 1e-6) + 1e-12), (lo, hi, k)


# ---------------------------------------------------------------- GMRES
def test_gmres_matches_lapack(hemisphere_bowl):
    fac, F = hemisphere_bowl
    E = np.random.default_rng(9).random((fac.N, 3))
    Bd = ref.solve_direct(F, 1.0, E)
    for restart in (50, 3):
        B, it, hist = ref.gmres(lambda X: F @ X, 1.0, E, tol=1e-13, restart=restart)
        assert np.max(np.abs(B - Bd)) <= 1e-11 * np.max(np.abs(Bd))
        true_res = np.linalg.norm(E - (B - F @ B), axis=0)
        assert np.all(true_res <= 1e-12 * np.linalg.norm(E, axis=0))


def test_gmres_minimal_residual_beats_jacobi(hemisphere_bowl):
    """Jacobi's k-th iterate from B^0 = E lies in the Krylov space of k + 1
    GMRES steps, so GMRES's residual after k + 1 steps is never larger, and
    its residual history never increases."""
    fac, F = hemisphere_bowl
    E = np.random.default_rng(10).random((fac.N, 2))
    _, _, hist = ref.gmres(lambda X: F @ X, 1.0, E, tol=1e-14, restart=100)
    Bj = E.copy()
    for k in range(12):
        if k:
            Bj = E + F @ Bj
        rj = np.linalg.norm(E - (Bj - F @ Bj), axis=0)
        for c, h in enumerate(hist):
            if k + 1 < len(h):
                assert h[k + 1] <= rj[c] * (1 + 1e-10) + 1e-14
    for h in hist:
        assert np.all(np.diff(h) <= 1e-12 * h[0])


def test_gmres_finite_termination():
    """Without restarts GMRES solves an n x n system in at most n steps."""
    rng = np.random.default_rng(11)
    n = 12
    F = rng.uniform(0.0, 1.0, (n, n)) / n
    rho = rng.uniform(0.2, 0.9, n)
    E = rng.standard_normal((n, 2))
    B, it, _ = ref.gmres(lambda X: F @ X, rho, E, tol=1e-13, restart=n)
    assert np.all(it <= n)
    np.testing.assert_allclose(B, ref.solve_direct(F, rho, E), rtol=1e-10, atol=1e-12)


def test_gmres_residuals_equal_krylov_least_squares(hemisphere_bowl):
    """The k-th GMRES residual is the least-squares minimum of ||E - M x|| over
    the Krylov space span{E, M E, ..., M^(k-1) E} (M = I - F), computed here by
    brute force; GMRES stops at the first k where that minimum meets tol."""
    fac, F = hemisphere_bowl
    E = np.random.default_rng(12).random((fac.N, 1))
    M = np.eye(fac.N) - F
    tol = 1e-6
    _, it, hist = ref.gmres(lambda X: F @ X, 1.0, E, tol=tol, restart=100)
    e = E[:, 0]
    best, k_first = [np.linalg.norm(e)], None
    K = [e / np.linalg.norm(e)]
    for k in range(1, 9):
        Q, _ = np.linalg.qr(np.column_stack(K))
        y, *_ = np.linalg.lstsq(M @ Q, e, rcond=None)
        best.append(np.linalg.norm(e - M @ Q @ y))
        if k_first is None and best[-1] <= tol * np.linalg.norm(e):
            k_first = k
        nxt = M @ K[-1]
        K.append(nxt / np.linalg.norm(nxt))
    h = hist[0]
    for k in range(1, min(len(h), 9)):
        assert abs(h[k] - best[k]) <= 1e-6 * best[k] + 1e-13 * best[0]
    assert it[0] == k_first


@pytest.mark.slow
def test_octree_compresses_closed_body_better_than_quadtree():
    """Section 4.1 motivates octrees for small bodies: on the closed 5,120-facet
    body a quadtree on (x, y) puts facets of the top and bottom into one cell,
    and its compressed matrix is about twice the octree's at eps = 1e-2."""
    from synth import BodySpec, body_mesh
    v, f = body_mesh(BodySpec(level=4))
    fac = ref.Facets(v, f)
    F = ref.view_factor_matrix(fac, ref.pair_visibility(fac, "raycast"))
    quad = hm.assemble(F, fac.x[:, :2], eps=1e-2, leaf_size=32)
    octo = hm.assemble(F, fac.x, eps=1e-2, leaf_size=32)
    assert octo.nbytes() < 0.6 * quad.nbytes()
    X = np.random.default_rng(13).random((fac.N, 2))
    for H in (quad, octo):
        assert np.linalg.norm(hm.multiply(H, X) - F @ X) / np.linalg.norm(F @ X) <= 1e-2
