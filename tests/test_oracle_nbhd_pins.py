"""Pins for the neighbourhood-inverse preconditioner of the oracle
(oracle.precond.neighbourhoods / neighbourhood_inverse).

The preconditioner extends the block-diagonal preconditioner of Sec. II-B:
wire p's row is its row block of the inverse of the submatrix of p and its
nearest near-set neighbours (eq. 9), symmetrised.  It is pinned by things
outside its own code:

* neighbourhoods of hand-placed wires, worked out by hand (distances, the
  d_c cut and the tie rule);
* one wire per neighbourhood equals the block-Jacobi inverses of
  oracle.solve (an independent routine);
* clouds made of separated groups of mutually coupled wires, each group no
  larger than a neighbourhood: Z is block diagonal by group, every
  neighbourhood is its whole group, so M is the exact inverse and M Z = I;
* two wires: the textbook 2 x 2 block inverse through the Schur complement;
* a chain A - B - C (A and C not near): M_AB = (W_A[A,B] + (Z^-1)_AB)/2 with
  W_A the inverse of the A-B submatrix, M_BB the Z^-1 block of B
  (B's neighbourhood is the whole cloud), and M_AC = 0 although
  (Z^-1)_AC is not;
* complex symmetry and the pattern (a subset of the near set).
"""
import math

import numpy as np
import pytest

from oracle import mom, precond, solve
from paper_2410_03060_amd import workloads as W

LAM = W.WAVELENGTH
NB = 7


def _line_cloud(xs, d_c, seed=0):
    """Wires centred on the x axis at xs (in wavelengths), random orientations."""
    rng = np.random.default_rng(seed)
    c = np.zeros((len(xs), 3))
    c[:, 0] = np.asarray(xs, dtype=np.float64) * LAM
    t = rng.normal(size=(len(xs), 3))
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    L = rng.uniform(0.4, 0.6, len(xs)) * LAM
    return W.single_cloud(c, t, L, LAM, d_c * LAM)


def test_neighbourhoods_by_hand():
    # wires at x = 0, 1, 2.5, 4.5, -1 (wavelengths); d_c = 1.6
    cl = _line_cloud([0.0, 1.0, 2.5, 4.5, -1.0], 1.6)
    nb = precond.neighbourhoods(cl, 3)
    # wire 0: neighbours 1 (1.0) and 4 (1.0): tie broken by the lower caller index
    assert nb[0].tolist() == [0, 1, 4]
    # wire 1: 0 (1.0), 2 (1.5); 4 is 2.0 away: outside d_c
    assert nb[1].tolist() == [1, 0, 2]
    assert nb[2].tolist() == [2, 1]          # 3 is 2.0 away
    assert nb[3].tolist() == [3]             # isolated
    assert nb[4].tolist() == [4, 0]
    nb2 = precond.neighbourhoods(cl, 2)
    assert [g.tolist() for g in nb2] == [[0, 1], [1, 0], [2, 1], [3], [4, 0]]
    nb1 = precond.neighbourhoods(cl, 1)
    assert [g.tolist() for g in nb1] == [[0], [1], [2], [3], [4]]


def test_one_wire_per_neighbourhood_is_block_jacobi():
    cl = W.random_cloud(5, 24, box_lam=2.0, d_c_lam=1.0)
    Zs, _ = mom.snfc_matrix(cl)
    M = precond.neighbourhood_inverse(Zs, precond.neighbourhoods(cl, 1)).toarray()
    P = solve.block_jacobi(Zs, NB)
    D = np.zeros_like(M)
    for p in range(cl.n):
        D[NB * p:NB * p + NB, NB * p:NB * p + NB] = P[p]
    assert np.max(np.abs(M - D)) <= 1e-14 * np.max(np.abs(D))


def _groups_cloud(sizes, seed=1, spread=0.3, gap=6.0, d_c=1.0):
    """Groups of wires inside balls of radius `spread` wavelengths, ball centres
    `gap` wavelengths apart (>> d_c): every pair inside a group is near, no pair
    across groups is."""
    rng = np.random.default_rng(seed)
    cs = []
    for g, m in enumerate(sizes):
        base = np.array([g * gap, 0.0, 0.0])
        off = rng.normal(size=(m, 3))
        off *= spread * rng.uniform(0, 1, (m, 1)) ** (1 / 3) / np.linalg.norm(off, axis=1, keepdims=True)
        cs.append((base + off) * LAM)
    c = np.concatenate(cs)
    t = rng.normal(size=c.shape)
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    L = rng.uniform(0.4, 0.6, c.shape[0]) * LAM
    return W.single_cloud(c, t, L, LAM, d_c * LAM)


@pytest.mark.parametrize("size", [3, 4, 6])
def test_groups_within_a_neighbourhood_give_the_exact_inverse(size):
    cl = _groups_cloud([3, 1, 2, 3, 2])
    Zs, _ = mom.snfc_matrix(cl)
    Zd = Zs.toarray()
    M = precond.neighbourhood_inverse(Zs, precond.neighbourhoods(cl, size)).toarray()
    assert np.max(np.abs(M @ Zd - np.eye(Zd.shape[0]))) <= 1e-11
    assert np.max(np.abs(M - np.linalg.inv(Zd))) <= 1e-11 * np.max(np.abs(M))


def test_two_wires_schur_complement():
    cl = _line_cloud([0.0, 0.3], 1.0, seed=3)
    Zs, _ = mom.snfc_matrix(cl)
    Zd = Zs.toarray()
    A, B, C = Zd[:NB, :NB], Zd[:NB, NB:], Zd[NB:, NB:]
    S = A - B @ np.linalg.solve(C, B.T)          # Schur complement of C
    M11 = np.linalg.inv(S)
    M12 = -M11 @ B @ np.linalg.inv(C)
    M22 = np.linalg.inv(C) + np.linalg.inv(C) @ B.T @ M11 @ B @ np.linalg.inv(C)
    M = precond.neighbourhood_inverse(Zs, precond.neighbourhoods(cl, 2)).toarray()
    ref = np.block([[M11, M12], [M12.T, M22]])
    assert np.max(np.abs(M - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_chain_symmetrisation_and_truncation():
    # A - B - C on a line, A and C farther apart than d_c
    cl = _line_cloud([0.0, 0.8, 1.6], 1.0, seed=4)
    Zs, _ = mom.snfc_matrix(cl)
    Zd = Zs.toarray()
    nb = precond.neighbourhoods(cl, 3)
    assert [sorted(g.tolist()) for g in nb] == [[0, 1], [0, 1, 2], [1, 2]]
    M = precond.neighbourhood_inverse(Zs, nb).toarray()
    Zi = np.linalg.inv(Zd)
    blk = lambda X, i, j: X[NB * i:NB * i + NB, NB * j:NB * j + NB]
    WA = np.linalg.inv(Zd[:2 * NB, :2 * NB])             # A's neighbourhood: A, B
    WC = np.linalg.inv(Zd[NB:, NB:])                     # C's neighbourhood: B, C
    tol = 1e-11 * np.max(np.abs(Zi))
    assert np.max(np.abs(blk(M, 0, 1) - 0.5 * (blk(WA, 0, 1) + blk(Zi, 0, 1)))) <= tol
    assert np.max(np.abs(blk(M, 2, 1) - 0.5 * (blk(WC, 1, 0) + blk(Zi, 2, 1)))) <= tol
    assert np.max(np.abs(blk(M, 1, 1) - blk(Zi, 1, 1))) <= tol
    assert np.max(np.abs(blk(M, 0, 0) - 0.5 * (blk(WA, 0, 0) + blk(WA, 0, 0).T))) <= tol
    assert np.max(np.abs(blk(M, 0, 2))) == 0.0 and np.max(np.abs(blk(Zi, 0, 2))) > 1e-5 * np.max(np.abs(Zi))


def test_symmetric_and_inside_the_near_set():
    cl = W.random_cloud(9, 40, box_lam=2.5, d_c_lam=0.9)
    Zs, (indptr, indices, rows) = mom.snfc_matrix(cl)
    M = precond.neighbourhood_inverse(Zs, precond.neighbourhoods(cl, 4))
    Md = M.toarray()
    assert np.array_equal(Md, Md.T) or np.max(np.abs(Md - Md.T)) == 0.0
    near = set(zip(rows.tolist(), indices.tolist()))
    Mb = M.tobsr(blocksize=(NB, NB))
    for p in range(cl.n):
        for e in range(Mb.indptr[p], Mb.indptr[p + 1]):
            assert (p, int(Mb.indices[e])) in near
