"""Pins of the cluster block-Jacobi oracle (oracle/precond.py).

The cell order is checked against orders worked out by hand from the Morton
definition; the inverse blocks against the paper's one-wire block-Jacobi
(an independent oracle routine) and against the exact inverse of a matrix
that is block diagonal by construction (groups of wires farther apart than
d_c do not couple under eq. 9).
"""
import math

import numpy as np
import pytest

from oracle import mom, precond, solve
from paper_2410_03060_amd import workloads as W

LAM = W.WAVELENGTH
Z_AXIS = (0.0, 0.0, 1.0)


def _cloud(centres_lam, d_c_lam, tangents=None, L=0.5):
    c = np.asarray(centres_lam, dtype=np.float64) * LAM
    n = c.shape[0]
    t = np.tile(Z_AXIS, (n, 1)) if tangents is None else np.asarray(tangents, dtype=np.float64)
    return W.single_cloud(c, t, np.full(n, L * LAM), LAM, d_c_lam * LAM)


def test_cell_order_of_a_2x2x2_block():
    """Cells of side just above 0.6 lambda; one wire per cell of a 2x2x2 block.

    Morton code = x | y << 1 | z << 2, so the cells (x, y, z) come in the order
    (000)(100)(010)(110)(001)(101)(011)(111)."""
    cells = [(1, 1, 1), (0, 0, 0), (1, 0, 1), (0, 1, 0), (1, 1, 0), (0, 0, 1), (1, 0, 0), (0, 1, 1)]
    cl = _cloud([(0.5 + x, 0.5 + y, 0.5 + z) for x, y, z in cells], 0.6)
    o, inv_h, dims = precond.grid(cl.center, cl.d_c)
    assert dims == (2, 2, 2)
    assert np.allclose(o, 0.5 * LAM)
    # worked out by hand: codes of the caller wires are 7,0,5,2,3,4,1,6
    assert precond.cell_order(cl).tolist() == [1, 6, 3, 4, 5, 2, 7, 0]


def test_cell_order_keeps_caller_order_inside_a_cell():
    # wires 0 and 1 share cell (1,0,0); wire 2 sits in cell (0,0,0); wire 3 in (0,1,0)
    cl = _cloud([(1.2, 0.1, 0.1), (1.3, 0.2, 0.0), (0.0, 0.0, 0.0), (0.1, 1.3, 0.2)], 1.0)
    assert precond.grid(cl.center, cl.d_c)[2] == (2, 2, 1)
    assert precond.cell_order(cl).tolist() == [2, 0, 1, 3]


def test_cell_order_is_per_cloud_and_single_cell_without_cutoff():
    a = _cloud([(1.2, 0.1, 0.1), (0.0, 0.0, 0.0)], 1.0)
    b = _cloud([(0.0, 1.5, 0.0), (0.0, 0.0, 0.0), (3.0, 0.0, 0.0)], 1.0)
    cl = W.concat_clouds([a, b])
    # cloud a: (1,0,0) after (0,0,0); cloud b (cells of side ~1): (0,1,0)=2, (0,0,0)=0, (3,0,0)=binary 11 -> 9
    assert precond.cell_order(cl).tolist() == [1, 0, 3, 2, 4]
    dense = _cloud([(1.2, 0.1, 0.1), (0.0, 0.0, 0.0), (5.0, 5.0, 5.0)], math.inf)
    assert precond.cell_order(dense).tolist() == [0, 1, 2]
    near = _cloud([(1.2, 0.1, 0.1), (0.0, 0.0, 0.0)], 1.5)   # d_c above the extent: one cell
    assert precond.cell_order(near).tolist() == [0, 1]


def test_grid_grows_until_the_table_fits():
    """Two wires 100 lambda apart with d_c = 1 lambda: 100 cells along x exceed
    the cap of 64, so the side grows by 1.25: 81 cells, then 100 / (1.5625 (1 + 1e-9))
    = 63.9999999 gives floor 63 + 1 = 64 cells, which fits."""
    cl = _cloud([(0.0, 0.0, 0.0), (100.0, 0.0, 0.0)], 1.0)
    o, inv_h, dims = precond.grid(cl.center, cl.d_c)
    assert dims == (64, 1, 1)
    assert inv_h == pytest.approx(1.0 / (LAM * (1.0 + 1e-9) * 1.25 ** 2), rel=1e-14)


def test_clusters_are_runs_of_the_cell_order_per_cloud():
    a = W.random_cloud(3, 19, box_lam=3.0, d_c_lam=0.7)
    b = W.random_cloud(4, 6, box_lam=2.0, d_c_lam=0.7)
    cl = W.concat_clouds([a, b])
    g = precond.clusters(cl, 8)
    assert [len(x) for x in g] == [8, 8, 3, 6]
    perm = precond.cell_order(cl)
    assert np.concatenate(g).tolist() == perm.tolist()
    assert sorted(perm.tolist()) == list(range(25))
    assert all((x < 19).all() or (x >= 19).all() for x in g)


def test_one_wire_per_group_is_the_block_jacobi_preconditioner():
    cl = W.random_cloud(5, 14, box_lam=2.0, d_c_lam=1.0)
    Zs, _ = mom.snfc_matrix(cl)
    g = precond.clusters(cl, 1)
    M = precond.cluster_inverse(Zs, g, size=1)
    P = solve.block_jacobi(Zs, 7)
    for k, w in enumerate(g):
        assert np.allclose(M[k], P[int(w[0])], rtol=1e-12, atol=0)


def _isolated_groups(seed, sizes, spacing=6.0, ball=0.3):
    rng = np.random.default_rng(seed)
    c, t, groups, i = [], [], [], 0
    for gi, m in enumerate(sizes):
        base = np.array([gi * spacing, (gi % 2) * spacing, 0.0])
        pts = base + rng.uniform(-ball, ball, (m, 3))
        c.append(pts)
        t.append(W._isotropic(rng, m))
        groups.append(np.arange(i, i + m))
        i += m
    cl = W.single_cloud(np.concatenate(c) * LAM, np.concatenate(t),
                        rng.uniform(0.4, 0.6, i) * LAM, LAM, 1.5 * LAM)
    return cl, groups


def test_isolated_groups_are_inverted_exactly():
    """Groups farther apart than d_c: the sparsified matrix is block diagonal by
    group, so the cluster preconditioner with those groups is its exact inverse
    (short groups included: their blocks are padded with the identity)."""
    cl, groups = _isolated_groups(7, [8, 8, 5, 8])
    Zs, _ = mom.snfc_matrix(cl)
    Zd = Zs.toarray()
    for a in range(len(groups)):
        for b in range(len(groups)):
            if a != b:
                ra, rb = precond.rows_of(groups[a]), precond.rows_of(groups[b])
                assert not Zd[np.ix_(ra, rb)].any()
    M = precond.cluster_inverse(Zs, groups, size=8)
    assert np.array_equal(M[2, 35:, 35:], np.eye(21))
    assert not M[2, :35, 35:].any() and not M[2, 35:, :35].any()
    rng = np.random.default_rng(1)
    X = rng.standard_normal((Zd.shape[0], 3)) + 1j * rng.standard_normal((Zd.shape[0], 3))
    Y = precond.cluster_apply(M, groups, Zd @ X)
    assert np.linalg.norm(Y - X) <= 1e-10 * np.linalg.norm(X)
    u = mom.excitation(cl, np.array([[1.0, 0.0, 0.0]]), np.array([[0.0, 0.0, 1.0]]))
    assert np.allclose(precond.cluster_apply(M, groups, u), solve.dense_solve(Zd, u), rtol=1e-10, atol=1e-14)


def test_cluster_preconditioner_is_complex_symmetric():
    """Z is complex symmetric (Galerkin), so each diagonal submatrix and its
    inverse are too: COCG stays valid with the cluster preconditioner."""
    cl = W.random_cloud(9, 24, box_lam=2.5, d_c_lam=1.0)
    Zs, _ = mom.snfc_matrix(cl)
    M = precond.cluster_inverse(Zs, precond.clusters(cl, 8), size=8)
    for k in range(M.shape[0]):
        assert np.allclose(M[k], M[k].T, rtol=1e-10, atol=1e-12 * np.abs(M[k]).max())
