"""Solvers for Z x = u in complex128 (oracle; test infrastructure only).

The method's result is the solution of the S-NFC system (eq. 3 with the
sparsified matrix of eq. 9); how it is reached does not change it.  The
oracle therefore uses library solvers as single steps:

* ``dense_solve``   -- LAPACK LU (the paper's "entire coupling (LU)");
* ``sparse_solve``  -- SuperLU on the block-sparse matrix;
* ``gmres_solve``   -- SciPy GMRES with a block-diagonal (block-Jacobi)
                       preconditioner to a tight FP64 tolerance, for systems
                       too large to factor.  The paper's iterative solver is
                       GCR with a block-diagonal preconditioner (Sec. II-B);
                       any convergent Krylov method gives the same solution.
"""
from __future__ import annotations

import numpy as np


def dense_solve(Z: np.ndarray, u: np.ndarray) -> np.ndarray:
    return np.linalg.solve(Z, u)


def sparse_solve(Zs, u: np.ndarray) -> np.ndarray:
    import scipy.sparse.linalg as spla
    lu = spla.splu(Zs.tocsc())
    u = np.asarray(u)
    if u.ndim == 1:
        return lu.solve(u)
    return np.stack([lu.solve(u[:, r]) for r in range(u.shape[1])], axis=1)


def block_jacobi(Zs, nb: int):
    """Inverse diagonal blocks of a BSR matrix -> [N, nb, nb]."""
    Zb = Zs.tobsr(blocksize=(nb, nb))
    n = Zb.shape[0] // nb
    D = np.zeros((n, nb, nb), dtype=np.complex128)
    for i in range(n):
        for e in range(Zb.indptr[i], Zb.indptr[i + 1]):
            if Zb.indices[e] == i:
                D[i] = Zb.data[e]
    return np.linalg.inv(D)


def gmres_solve(Zs, u: np.ndarray, nb: int, rtol: float = 1e-12, restart: int = 60,
                maxiter: int = 400, apply_m=None, stats: dict | None = None) -> np.ndarray:
    """GMRES(restart) on each column of u with a preconditioner M ~ Z^-1.

    M is the block-Jacobi inverse of Sec. II-B unless ``apply_m`` (v -> M v)
    is given, e.g. the cluster inverse of ``oracle.precond``; the
    preconditioner changes only the iteration count.  ``stats`` (optional)
    receives the inner-iteration count of every column under "iterations".
    """
    import scipy.sparse.linalg as spla
    if apply_m is None:
        Pinv = block_jacobi(Zs, nb)
        n = Pinv.shape[0]

        def apply_p(v):
            return np.einsum("nij,nj->ni", Pinv, v.reshape(n, nb)).ravel()
    else:
        apply_p = apply_m

    M = spla.LinearOperator(Zs.shape, matvec=apply_p, dtype=np.complex128)
    u = np.asarray(u)
    cols = [u] if u.ndim == 1 else [u[:, r] for r in range(u.shape[1])]
    out = []
    for b in cols:
        count = [0]

        def cb(_res, count=count):
            count[0] += 1

        x, info = spla.gmres(Zs, b, M=M, rtol=rtol, atol=0.0, restart=restart,
                             maxiter=maxiter, callback=cb, callback_type="pr_norm")
        if info != 0:
            raise RuntimeError(f"oracle GMRES did not converge (info={info})")
        if stats is not None:
            stats.setdefault("iterations", []).append(count[0])
        out.append(x)
    return out[0] if u.ndim == 1 else np.stack(out, axis=1)


def relative_residual(Zs, x: np.ndarray, u: np.ndarray) -> np.ndarray:
    r = u - Zs @ x
    return np.linalg.norm(r, axis=0) / np.linalg.norm(u, axis=0)
