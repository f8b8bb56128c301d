"""Hierarchically compressed view-factor matrix, CPU reference (TEST INFRASTRUCTURE ONLY).

A plain numpy rendering of the paper's compression scheme, in the paper's
order, used to check what compression at tolerance eps does to F before the
GPU library is compared against it:

  * quadtree on facet centroids ................... Algorithm 2 (section 4.1)
  * octree, its 3-D analogue for closed bodies ...... section 4.1, section 8
  * numerical rank by truncated SVD with doubling . Algorithm 3 (section 4.2)
  * hierarchical min-bytes assembly ............... Algorithm 4 (section 4.3)
  * product with the compressed matrix ............ Algorithm 5 (section 4.4)

The dense F comes from ``reference.view_factor_matrix`` (Algorithm 1's
entries); a block's CSR form is only used for its byte count.  The SVD of a
block is numpy's LAPACK SVD (a library primitive standing in for ARPACK).

Readings of passages that are silent or garbled (listed in the design notes):
  * the quadtree split uses the node's own bounding-box midpoints
    (the printed sets compare with x_min / y_min, which would be empty);
    ``<`` goes to the low side; children ordered I1..I4 as printed;
  * the octree splits at the three midpoints into at most eight sets, ordered
    like I1..I4 with x the most significant side, then y, then z;
  * recursion stops at ``leaf_size`` points, at ``max_depth``, or when all
    centroids of a node coincide;
  * a block pair is a leaf block when both index sets are tree leaves or
    ``|I||J| <= leaf_size^2``; a leaf side is not split while the other
    side recurses;
  * bytes: value size s, index size 4; dense m n s; CSR 4(m+1) + nnz(4+s);
    truncated SVD (m+n) q s + q s; a zero block costs nothing;
  * ties go to the simpler form: zero < dense < CSR < SVD < hierarchical;
  * coalescing: children all dense -> one dense block; children all CSR or
    zero (not all zero) -> one CSR block;
  * q >= 1; an all-zero block is a zero block.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


# ----------------------------------------------------------------------------
# Algorithm 2: quadtree
# ----------------------------------------------------------------------------
@dataclass
class Node:
    idx: np.ndarray
    depth: int
    children: list = field(default_factory=list)

    @property
    def is_leaf(self) -> bool:
        return not self.children

    @property
    def size(self) -> int:
        return int(self.idx.size)


def spatial_tree(pts: np.ndarray, leaf_size: int = 64, max_depth: int | None = None) -> Node:
    """Algorithm 2 on the columns of pts: a quadtree for (x, y), an octree for
    (x, y, z).  Root holds every centroid; a node splits at its bounding-box
    midpoint along every axis, into at most 2^d non-empty children."""
    d = pts.shape[1]

    def build(idx: np.ndarray, depth: int) -> Node:
        node = Node(idx=idx, depth=depth)
        if idx.size <= leaf_size or (max_depth is not None and depth >= max_depth):
            return node
        p = pts[idx]
        lo, hi = p.min(axis=0), p.max(axis=0)
        if np.all(lo == hi):
            return node
        low = p < 0.5 * (lo + hi)
        for code in range(1 << d):
            m = np.ones(idx.size, dtype=bool)
            for a in range(d):
                high_side = (code >> (d - 1 - a)) & 1
                m &= ~low[:, a] if high_side else low[:, a]
            if m.any():
                node.children.append(build(idx[m], depth + 1))
        return node

    return build(np.arange(pts.shape[0]), 0)


def quadtree(xy: np.ndarray, leaf_size: int = 64, max_depth: int | None = None) -> Node:
    """Algorithm 2 on the (x, y) centroids."""
    return spatial_tree(np.asarray(xy)[:, :2], leaf_size, max_depth)


def octree(xyz: np.ndarray, leaf_size: int = 64, max_depth: int | None = None) -> Node:
    """The octree of section 4.1 on the (x, y, z) centroids."""
    return spatial_tree(np.asarray(xyz)[:, :3], leaf_size, max_depth)


def leaves(node: Node):
    if node.is_leaf:
        yield node
    else:
        for c in node.children:
            yield from leaves(c)


def tree_permutation(root: Node) -> np.ndarray:
    """Facet order in which every node is a contiguous range (leaves in DFS order)."""
    return np.concatenate([lf.idx for lf in leaves(root)])


# ----------------------------------------------------------------------------
# Blocks and their byte counts
# ----------------------------------------------------------------------------
KIND_ORDER = {"zero": 0, "dense": 1, "csr": 2, "svd": 3, "hier": 4}


@dataclass
class Block:
    kind: str
    rows: np.ndarray            # original facet indices of I
    cols: np.ndarray            # original facet indices of J
    nbytes: int
    data: object = None         # dense array / (U, s, V) / list of child Blocks


def dense_bytes(m: int, n: int, s: int) -> int:
    return m * n * s


def csr_bytes(m: int, nnz: int, s: int) -> int:
    return 4 * (m + 1) + nnz * (4 + s)


def svd_bytes(m: int, n: int, q: int, s: int) -> int:
    return (m + n) * q * s + q * s


# ----------------------------------------------------------------------------
# Algorithm 3: numerical rank with a doubling k-term SVD
# ----------------------------------------------------------------------------
def estimate_rank(FIJ: np.ndarray, eps: float, s: int, k0: int = 8):
    """Return (q, U_q, sigma_q, V_q) if a q-term SVD beats the CSR bytes, else None."""
    m, n = FIJ.shape
    nnz = int(np.count_nonzero(FIJ))
    U, sv, Vt = np.linalg.svd(FIJ, full_matrices=False)
    r = sv.size
    k = k0
    while True:
        kk = min(k, r)
        q = None
        # sigma_{q+1} is known for q+1 <= kk; beyond the full rank it is 0
        for qq in range(1, kk + 1):
            nxt = sv[qq] if qq < r else 0.0
            if qq < kk or kk == r:
                if nxt / sv[0] < eps:
                    q = qq
                    break
        if q is not None:
            if svd_bytes(m, n, q, s) < csr_bytes(m, nnz, s):
                return q, U[:, :q], sv[:q], Vt[:q, :].T
            return None
        if kk == r:
            return None
        k *= 2


# ----------------------------------------------------------------------------
# Algorithm 4: hierarchical min-bytes assembly
# ----------------------------------------------------------------------------
def _leaf_choice(FIJ, rows, cols, s):
    m, n = FIJ.shape
    nnz = int(np.count_nonzero(FIJ))
    if nnz == 0:
        return Block("zero", rows, cols, 0)
    db = dense_bytes(m, n, s)
    cb = csr_bytes(m, nnz, s)
    if db <= cb:
        return Block("dense", rows, cols, db, FIJ.copy())
    return Block("csr", rows, cols, cb, FIJ.copy())


def assemble_block(F: np.ndarray, I: Node, J: Node, eps: float, s: int, leaf_size: int):
    rows, cols = I.idx, J.idx
    FIJ = F[np.ix_(rows, cols)]
    m, n = FIJ.shape
    nnz = int(np.count_nonzero(FIJ))
    if nnz == 0:
        return Block("zero", rows, cols, 0)
    if (I.is_leaf and J.is_leaf) or m * n <= leaf_size * leaf_size:
        return _leaf_choice(FIJ, rows, cols, s)
    cands = [Block("dense", rows, cols, dense_bytes(m, n, s)),
             Block("csr", rows, cols, csr_bytes(m, nnz, s))]
    est = estimate_rank(FIJ, eps, s)
    if est is not None:
        q, U, sv, V = est
        cands.append(Block("svd", rows, cols, svd_bytes(m, n, q, s), (U, sv, V)))
    CI = I.children if not I.is_leaf else [I]
    CJ = J.children if not J.is_leaf else [J]
    kids = [assemble_block(F, ci, cj, eps, s, leaf_size) for ci in CI for cj in CJ]
    cands.append(Block("hier", rows, cols, sum(b.nbytes for b in kids), kids))
    best = min(cands, key=lambda b: (b.nbytes, KIND_ORDER[b.kind]))
    if best.kind == "dense":
        best.data = FIJ.copy()
    elif best.kind == "csr":
        best.data = FIJ.copy()
    elif best.kind == "hier":
        kinds = {b.kind for b in kids}
        if kinds == {"dense"}:
            best = Block("dense", rows, cols, dense_bytes(m, n, s), FIJ.copy())
        elif kinds <= {"csr", "zero"} and "csr" in kinds:
            best = Block("csr", rows, cols, csr_bytes(m, nnz, s), FIJ.copy())
    return best


@dataclass
class HMatrix:
    N: int
    root: Node
    blocks: list  # top-level blocks (pairs of the root's children)

    def nbytes(self) -> int:
        return sum(b.nbytes for b in self.blocks)


def assemble(F: np.ndarray, pts: np.ndarray, eps: float, s: int = 8, leaf_size: int = 64,
             max_depth: int | None = None) -> HMatrix:
    """Compress F starting from the pairs of the root's children: at most 16
    for a quadtree (pts = x, y centroids), 64 for an octree (x, y, z)."""
    root = spatial_tree(pts, leaf_size=leaf_size, max_depth=max_depth)
    if root.is_leaf:
        return HMatrix(F.shape[0], root, [_leaf_choice(F, root.idx, root.idx, s)])
    blocks = [assemble_block(F, ci, cj, eps, s, leaf_size)
              for ci in root.children for cj in root.children]
    return HMatrix(F.shape[0], root, blocks)


# ----------------------------------------------------------------------------
# Algorithm 5: Y = F_hat X
# ----------------------------------------------------------------------------
def _apply(b: Block, X: np.ndarray, Y: np.ndarray) -> None:
    if b.kind == "zero":
        return
    if b.kind in ("dense", "csr"):
        Y[b.rows] += b.data @ X[b.cols]
    elif b.kind == "svd":
        U, sv, V = b.data
        Y[b.rows] += U @ (sv[:, None] * (V.T @ X[b.cols]))
    else:
        for c in b.data:
            _apply(c, X, Y)


def multiply(H: HMatrix, X: np.ndarray) -> np.ndarray:
    X2 = X.reshape(H.N, -1)
    Y = np.zeros_like(X2, dtype=np.float64)
    for b in H.blocks:
        _apply(b, X2, Y)
    return Y.reshape(X.shape)


def block_stats(H: HMatrix) -> dict:
    out = {k: 0 for k in KIND_ORDER}
    nb = {k: 0 for k in KIND_ORDER}

    def walk(b):
        if b.kind == "hier":
            for c in b.data:
                walk(c)
        else:
            out[b.kind] += 1
            nb[b.kind] += b.nbytes

    for b in H.blocks:
        walk(b)
    return {"count": out, "bytes": nb, "total_bytes": H.nbytes()}


def leaf_blocks(H: HMatrix):
    """Flatten the block tree into its non-hierarchical blocks."""
    out = []

    def walk(b):
        if b.kind == "hier":
            for c in b.data:
                walk(c)
        else:
            out.append(b)

    for b in H.blocks:
        walk(b)
    return out
