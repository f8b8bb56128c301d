"""Reader of the block files written by rad_hmat_export (format stated in
include/rad.h), and the dense F-hat they describe.  Test-side only."""
import struct

import numpy as np

KIND_DENSE, KIND_CSR, KIND_LOWRANK = 1, 2, 3


def read_export(path):
    """Parse the file: {"dtype", "N", "perm", "blocks": [...]}; each block has
    kind, i0, m, j0, n, rank, nnz, its arrays and dense() -> its m x n values."""
    data = open(path, "rb").read()
    if data[:8] != b"RADHBLKS":
        raise ValueError("not a block export")
    version, dtype = struct.unpack_from("<Ii", data, 8)
    if version != 1:
        raise ValueError(f"unknown version {version}")
    N, nb = struct.unpack_from("<qq", data, 16)
    off = 32
    perm = np.frombuffer(data, np.int32, N, off).copy()
    off += 4 * N
    blocks = []

    def take(dt, count):
        nonlocal off
        a = np.frombuffer(data, dt, count, off).copy()
        off += a.nbytes
        return a

    for _ in range(nb):
        kind, i0, m, j0, n, rank = struct.unpack_from("<6i", data, off)
        off += 24
        (nnz,) = struct.unpack_from("<q", data, off)
        off += 8
        b = {"kind": kind, "i0": i0, "m": m, "j0": j0, "n": n, "rank": rank, "nnz": nnz}
        if kind == KIND_DENSE:
            A = take(np.float64, m * n).reshape(n, m).T
            b["dense"] = (lambda A=A: A)
        elif kind == KIND_CSR:
            rowptr = take(np.int32, m + 1)
            cols = take(np.int32, nnz)
            vals = take(np.float64, nnz)
            b.update(rowptr=rowptr, cols=cols, vals=vals)

            def dense(m=m, n=n, rowptr=rowptr, cols=cols, vals=vals):
                A = np.zeros((m, n))
                for r in range(m):
                    for e in range(rowptr[r], rowptr[r + 1]):
                        A[r, cols[e]] += vals[e]
                return A
            b["dense"] = dense
        elif kind == KIND_LOWRANK:
            U = take(np.float64, m * rank).reshape(rank, m).T
            V = take(np.float64, n * rank).reshape(rank, n).T
            b.update(U=U, V=V)
            b["dense"] = (lambda U=U, V=V: U @ V.T)
        else:
            raise ValueError(f"unknown block kind {kind}")
        blocks.append(b)
    if off != len(data):
        raise ValueError("trailing bytes in block export")
    return {"dtype": dtype, "N": N, "perm": perm, "blocks": blocks}


def densify(ex, original_order=True):
    """Sum of all blocks as a dense N x N FP64 matrix (rows and columns in the
    caller's facet order unless original_order is False)."""
    N = ex["N"]
    Ft = np.zeros((N, N))
    for b in ex["blocks"]:
        Ft[b["i0"]:b["i0"] + b["m"], b["j0"]:b["j0"] + b["n"]] += b["dense"]()
    if not original_order:
        return Ft
    F = np.empty_like(Ft)
    p = ex["perm"]
    F[np.ix_(p, p)] = Ft
    return F
