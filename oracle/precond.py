"""Cluster block-Jacobi preconditioner (oracle; test infrastructure only).

The paper preconditions its iterative solver with the inverses of the
diagonal blocks, one block per wire (Sec. II-B).  The cluster variant groups
wires that lie close together and inverts each group's whole diagonal
submatrix of the sparsified impedance matrix (eq. 9); with one wire per group
it is the paper's block-Jacobi preconditioner.  A preconditioner changes how
fast a Krylov method reaches the solution of Z x = u, never the solution.

Groups are runs of `size` consecutive wires of one cloud in *cell order*:
wires sorted by (cloud, Morton code of their grid cell), ties kept in caller
order.  The grid is the one the neighbour search uses for eq. (9): origin at
the cloud's minimum centre coordinates, cubic cells with a side just above
d_c (enlarged by factors of 1.25 while the table would exceed max(4 n, 64)
cells or 65000 cells per axis), and a single cell when d_c is infinite or
not below the cloud's extent.  The last group of a cloud may be shorter.

Every function here is a plain definition: a stable sort for the order, a
dense inverse per group for the preconditioner, dense products to apply it.

The neighbourhood-inverse preconditioner is the same idea centred on every
wire: wire p's neighbourhood is p and its nearest near-set neighbours (at most
`size` wires); its row of the preconditioner is p's row block of the inverse
of the neighbourhood's submatrix, and the rows are symmetrised
(M_pq = (W_p[p,q] + W_q[q,p]^T)/2) so that M is complex symmetric like Z.
A dense inverse per wire, plainly written, again.
"""
from __future__ import annotations

import math

import numpy as np

NB = 7   # unknowns per wire (8 segments, 7 interior rooftops)


def grid(center: np.ndarray, d_c: float):
    """(origin[3], inv_h, dims[3]) of one cloud's cell grid."""
    c = np.asarray(center, dtype=np.float64).reshape(-1, 3)
    if c.shape[0] == 0:
        return np.zeros(3), 0.0, (1, 1, 1)
    mn, mx = c.min(axis=0), c.max(axis=0)
    ext = max(float((mx - mn).max()), 0.0)
    if not (math.isfinite(d_c) and d_c * (1.0 + 1e-9) < ext):
        return mn, 0.0, (1, 1, 1)
    h = max(d_c * (1.0 + 1e-9), ext / 65000.0, 1e-30)
    cap = max(4 * c.shape[0], 64)
    while True:
        a = (mx - mn) / h
        dims = tuple(int(math.floor(v)) + 1 for v in a)
        if dims[0] * dims[1] * dims[2] <= cap and bool((a < 65000).all()):
            break
        h *= 1.25
    return mn, 1.0 / h, dims


def morton3(ix: np.ndarray, iy: np.ndarray, iz: np.ndarray) -> np.ndarray:
    """Interleave the bits of the cell indices: x -> bit 3b, y -> 3b+1, z -> 3b+2."""
    code = np.zeros(ix.shape, dtype=np.int64)
    for b in range(21):
        code |= ((ix.astype(np.int64) >> b) & 1) << (3 * b)
        code |= ((iy.astype(np.int64) >> b) & 1) << (3 * b + 1)
        code |= ((iz.astype(np.int64) >> b) & 1) << (3 * b + 2)
    return code


def cells(center: np.ndarray, d_c: float) -> np.ndarray:
    """[n, 3] integer cell of every centre of one cloud (clamped into the grid)."""
    c = np.asarray(center, dtype=np.float64).reshape(-1, 3)
    o, inv_h, dims = grid(c, d_c)
    if inv_h == 0.0:
        return np.zeros((c.shape[0], 3), dtype=np.int64)
    f = np.floor((c - o) * inv_h)
    hi = np.array(dims, dtype=np.float64) - 1.0
    return np.minimum(np.maximum(f, 0.0), hi).astype(np.int64)


def cell_order(cloud) -> np.ndarray:
    """perm[i] = caller index of the i-th wire in cell order (all clouds)."""
    off = np.asarray(cloud.cloud_off, dtype=np.int64)
    out = []
    for k in range(len(off) - 1):
        idx = np.arange(off[k], off[k + 1])
        cl = cells(np.asarray(cloud.center)[idx], float(cloud.d_c))
        code = morton3(cl[:, 0], cl[:, 1], cl[:, 2])
        out.append(idx[np.argsort(code, kind="stable")])
    return np.concatenate(out) if out else np.zeros(0, dtype=np.int64)


def clusters(cloud, size: int = 8):
    """Caller indices of every group, in cell order, cloud by cloud."""
    perm = cell_order(cloud)
    off = np.asarray(cloud.cloud_off, dtype=np.int64)
    groups = []
    for k in range(len(off) - 1):
        for w0 in range(int(off[k]), int(off[k + 1]), size):
            groups.append(perm[w0:min(w0 + size, int(off[k + 1]))])
    return groups


def rows_of(group: np.ndarray) -> np.ndarray:
    """Unknown indices (caller order) of a group's wires, wire-major."""
    g = np.asarray(group, dtype=np.int64)
    return (NB * g[:, None] + np.arange(NB)[None, :]).reshape(-1)


def cluster_inverse(Zs, groups, size: int = 8) -> np.ndarray:
    """[len(groups), 7 size, 7 size]: inverse of each group's diagonal submatrix.

    Zs is the sparsified matrix in caller order (any SciPy sparse format or a
    dense array).  A short group's block is its inverse padded with the
    identity, so that every block has one shape."""
    n = NB * size
    Zc = Zs.tocsr() if hasattr(Zs, "tocsr") else np.asarray(Zs)
    out = np.zeros((len(groups), n, n), dtype=np.complex128)
    for k, g in enumerate(groups):
        r = rows_of(g)
        D = Zc[r][:, r]
        D = D.toarray() if hasattr(D, "toarray") else np.asarray(D)
        m = r.size
        out[k, :m, :m] = np.linalg.inv(D)
        out[k, m:, m:] = np.eye(n - m)
    return out


def cluster_apply(Minv: np.ndarray, groups, X: np.ndarray) -> np.ndarray:
    """Y = M X in caller order: each group's rows get its inverse block times
    the same rows of X; X is [N*7] or [N*7, s]."""
    X = np.asarray(X)
    Y = np.zeros_like(X, dtype=np.complex128)
    for k, g in enumerate(groups):
        r = rows_of(g)
        Y[r] = Minv[k, :r.size, :r.size] @ X[r]
    return Y


def condition_numbers(Zs, groups) -> np.ndarray:
    """2-norm condition number of every group's diagonal submatrix."""
    Zc = Zs.tocsr() if hasattr(Zs, "tocsr") else np.asarray(Zs)
    out = np.zeros(len(groups))
    for k, g in enumerate(groups):
        r = rows_of(g)
        D = Zc[r][:, r]
        D = D.toarray() if hasattr(D, "toarray") else np.asarray(D)
        out[k] = np.linalg.cond(D)
    return out


# --------------------------------------------------------------------------- neighbourhood inverse

def neighbourhoods(cloud, size: int):
    """For every wire p (caller order): [p] followed by at most size - 1 wires of
    p's near set (eq. 9: same cloud, centroid distance <= d_c), nearest first.

    Order: the FP64 squared centroid distance ((dx*dx + dy*dy) + dz*dz), each
    operation rounded (the near-set test of eq. 9), then the lower caller index.
    """
    from . import mom
    if size < 1:
        raise ValueError("a neighbourhood holds at least the wire itself")
    c = np.asarray(cloud.center, dtype=np.float64)
    I, J = mom.near_pairs(c, cloud.cloud_off, float(cloud.d_c))
    d2 = mom._d2(c[I], c[J])
    out = []
    starts = np.searchsorted(I, np.arange(cloud.n + 1))
    for p in range(cloud.n):
        a, b = int(starts[p]), int(starts[p + 1])
        js, ds = J[a:b], d2[a:b]
        order = np.lexsort((js, ds))        # distance first, then caller index
        out.append(np.concatenate([[p], js[order][:size - 1]]).astype(np.int64))
    return out


def neighbourhood_raw_blocks(Zs, nbhd, nb: int = NB) -> dict:
    """{(p, q): W_p[p, q]} for q in nbhd[p]: the row block of wire p of W_p, the
    inverse of the sparsified matrix restricted to the wires of nbhd[p] (their
    diagonal blocks and every near-pair block between them)."""
    Zc = Zs.tocsr() if hasattr(Zs, "tocsr") else np.asarray(Zs)
    out = {}
    for p, g in enumerate(nbhd):
        r = (nb * np.asarray(g)[:, None] + np.arange(nb)[None, :]).reshape(-1)
        A = Zc[r][:, r]
        A = A.toarray() if hasattr(A, "toarray") else np.asarray(A)
        W = np.linalg.inv(A)
        for k, q in enumerate(g):
            out[(p, int(q))] = W[:nb, nb * k:nb * k + nb]
    return out


def symmetrise(raw: dict, n: int, nb: int = NB):
    """M (scipy BSR, caller order) from raw row blocks {(p, q): R_p[p, q]}:
    M_pq = (R_p[p,q] + R_q[q,p]^T) / 2, a missing raw block counting as zero."""
    import scipy.sparse as sp
    keys = set(raw) | {(q, p) for (p, q) in raw}
    I = np.array(sorted(keys), dtype=np.int64).reshape(-1, 2)
    blocks = np.zeros((I.shape[0], nb, nb), dtype=np.complex128)
    for t, (p, q) in enumerate(I):
        a = raw.get((int(p), int(q)))
        b = raw.get((int(q), int(p)))
        v = np.zeros((nb, nb), dtype=np.complex128)
        if a is not None:
            v = v + a
        if b is not None:
            v = v + b.T
        blocks[t] = 0.5 * v
    indptr = np.searchsorted(I[:, 0], np.arange(n + 1)) if I.size else np.zeros(n + 1, dtype=np.int64)
    return sp.bsr_matrix((blocks, I[:, 1], indptr), shape=(nb * n, nb * n), blocksize=(nb, nb))


def neighbourhood_inverse(Zs, nbhd, nb: int = NB):
    """The neighbourhood-inverse preconditioner M (scipy BSR, caller order).

    M_pq = (W_p[p,q] + W_q[q,p]^T) / 2, a raw block that does not exist (q not
    in nbhd[p]) counting as zero; M is complex symmetric like Z, with blocks
    only on pairs where one wire is in the other's neighbourhood (a subset of
    the near set).  One wire per neighbourhood gives the block-diagonal
    preconditioner of Sec. II-B; neighbourhoods that contain whole groups of
    mutually coupled wires give the exact inverse on those groups."""
    return symmetrise(neighbourhood_raw_blocks(Zs, nbhd, nb), len(nbhd), nb)
