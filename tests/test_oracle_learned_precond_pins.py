"""Pins for the learned neighbourhood-inverse preconditioner of the oracle
(oracle.learned_precond): its canonical frame, features and the map between
raw row blocks and network outputs.

* The canonical frame against the MoM itself: reversing a wire's tangent and
  rebuilding Z (oracle.mom) and the raw rows of the neighbourhood inverse
  leaves every target unchanged — the map S = sigma P (rooftops reversed and
  negated) is the one the Galerkin blocks obey.
* Rigid motions that keep every canonical sign (translations, rotations
  about z) leave features and targets unchanged (targets through the MoM
  again: rebuilt blocks, new raw rows).
* Features of a hand-placed pair worked out by hand.
* targets and raw_from_outputs are inverse maps, and symmetrising the raw
  rows recovered from the targets gives the computed preconditioner.
* The targets are departures from the block-diagonal preconditioner: an
  isolated wire's target is zero, and zero outputs give exactly the
  block-Jacobi inverses of oracle.solve (an independent routine).
"""
import math

import numpy as np
import pytest

from oracle import learned_precond as lp
from oracle import mom, precond
from paper_2410_03060_amd import workloads as W

LAM = W.WAVELENGTH
K = 2.0 * math.pi / LAM


def _cloud(seed=3, n=30, box=2.0, d_c=1.0):
    return W.random_cloud(seed, n, box_lam=box, d_c_lam=d_c)


def _raw_and_targets(cloud, size):
    Zs, _ = mom.snfc_matrix(cloud)
    nb = precond.neighbourhoods(cloud, size)
    raw = precond.neighbourhood_raw_blocks(Zs, nb)
    return nb, raw, lp.targets(cloud, nb, size, raw)


def test_reversing_tangents_leaves_targets_and_features_unchanged():
    cl = _cloud()
    size = 4
    nb, raw, T = _raw_and_targets(cl, size)
    F = lp.features(cl, nb, size)
    flip = np.zeros(cl.n, dtype=bool)
    flip[[0, 3, 7, 11, 20]] = True
    t2 = np.where(flip[:, None], -cl.tangent, cl.tangent)
    cl2 = W.single_cloud(cl.center, t2, cl.length, cl.wavelength, cl.d_c, cl.radius)
    nb2, raw2, T2 = _raw_and_targets(cl2, size)
    assert all(np.array_equal(a, b) for a, b in zip(nb, nb2))
    assert np.max(np.abs(T2 - T)) <= 1e-9 * np.max(np.abs(T))
    assert np.max(np.abs(lp.features(cl2, nb2, size) - F)) <= 1e-12
    # and the raw rows did change: the frame is doing the work
    assert max(np.max(np.abs(raw2[k] - raw[k])) for k in raw) > 1e-3 * max(np.max(np.abs(v)) for v in raw.values())


def test_translation_and_rotation_about_z():
    cl = _cloud(seed=5)
    size = 3
    nb, raw, T = _raw_and_targets(cl, size)
    F = lp.features(cl, nb, size)
    a = 0.7
    R = np.array([[math.cos(a), -math.sin(a), 0.0], [math.sin(a), math.cos(a), 0.0], [0.0, 0.0, 1.0]])
    c2 = cl.center @ R.T + np.array([3.0, -1.0, 2.0]) * LAM
    t2 = cl.tangent @ R.T
    cl2 = W.single_cloud(c2, t2, cl.length, cl.wavelength, cl.d_c, cl.radius)
    nb2, raw2, T2 = _raw_and_targets(cl2, size)
    assert all(np.array_equal(x, y) for x, y in zip(nb, nb2))
    assert np.max(np.abs(lp.features(cl2, nb2, size) - F)) <= 1e-9
    assert np.max(np.abs(T2 - T)) <= 1e-7 * np.max(np.abs(T))


def test_features_of_a_hand_placed_pair():
    # p at the origin along -z (canonical +z), q 0.3 lambda along x, tangent +y; d_c = 0.5 lambda
    c = np.array([[0.0, 0.0, 0.0], [0.3 * LAM, 0.0, 0.0]])
    t = np.array([[0.0, 0.0, -1.0], [0.0, 1.0, 0.0]])
    L = np.array([0.5, 0.45]) * LAM
    cl = W.single_cloud(c, t, L, LAM, 0.5 * LAM)
    nb = precond.neighbourhoods(cl, 2)
    assert [g.tolist() for g in nb] == [[0, 1], [1, 0]]
    F = lp.features(cl, nb, 2).reshape(2, 2, 7, 192)
    f = F[0, 1, 2]                     # wire 0, slot 1 (q = wire 1), column 2
    assert f[2] == 1.0 and f[7 + 1] == 1.0 and np.sum(f[:15]) == 2.0
    assert f[15] == pytest.approx(0.0, abs=1e-12) and f[16] == pytest.approx(10 * (0.45 - 0.5))
    e = np.exp(-1j * K * 0.3 * LAM)
    assert np.allclose(f[17:23], [0.6, 0.0, 0.0, 0.0, e.real, e.imag], atol=1e-12)
    assert f[23] == pytest.approx(2 / 8)
    # member 0 is p itself: distance 0 to p, 0.3 lambda to q
    b = 24
    assert np.allclose(f[b:b + 15], [1, 0.0, 0, 0, 0, 1, 1, 0, 0.6, 0.0, 0.0, 0.0, e.real, e.imag, 1], atol=1e-12)
    # member 1 is q
    b = 24 + 15
    assert np.allclose(f[b:b + 15], [1, -0.5, 0.6, 0.0, 0.0, 0.0, e.real, e.imag, 0, 0, 0, 1, 1, 0, 1], atol=1e-12)
    assert np.all(f[24 + 30:] == 0)
    # an isolated wire: one slot, the other row empty
    assert np.all(lp.features(W.single_cloud(c[:1], t[:1], L[:1], LAM, 0.5 * LAM), [np.array([0])], 2)
                  .reshape(2, 7, 192)[1] == 0)


def test_output_map_inverts_the_targets_and_rebuilds_the_preconditioner():
    cl = _cloud(seed=9, n=25)
    size = 5
    nb, raw, T = _raw_and_targets(cl, size)
    back = lp.raw_from_outputs(cl, nb, size, T)
    assert set(back) == set(raw)
    big = max(np.max(np.abs(v)) for v in raw.values())
    assert max(np.max(np.abs(back[k] - raw[k])) for k in raw) <= 1e-13 * big
    Zs, _ = mom.snfc_matrix(cl)
    M = precond.neighbourhood_inverse(Zs, nb).toarray()
    M2 = precond.symmetrise(back, cl.n).toarray()
    assert np.max(np.abs(M - M2)) <= 1e-14 * np.max(np.abs(M))


def test_zero_output_is_the_block_diagonal_preconditioner():
    # an isolated wire's target is zero (its raw row is Z_pp^-1), and a network
    # that outputs zero gives exactly the block-Jacobi inverses of oracle.solve
    from oracle import solve as osolve
    cl = _cloud(seed=11, n=20, box=6.0, d_c=0.6)
    size = 4
    nb, raw, T = _raw_and_targets(cl, size)
    iso = [p for p in range(cl.n) if len(nb[p]) == 1]
    assert iso, "the draw should hold isolated wires"
    Tr = T.reshape(cl.n, size, 7, 14)
    for p in iso:
        assert np.max(np.abs(Tr[p])) <= 1e-12 * lp.TARGET_SCALE * np.max(np.abs(raw[(p, p)]))
    Zs, _ = mom.snfc_matrix(cl)
    M0 = precond.symmetrise(lp.raw_from_outputs(cl, nb, size, np.zeros_like(T)), cl.n).toarray()
    P = osolve.block_jacobi(Zs, 7)
    D = np.zeros_like(M0)
    for p in range(cl.n):
        D[7 * p:7 * p + 7, 7 * p:7 * p + 7] = P[p]
    assert np.max(np.abs(M0 - D)) <= 1e-13 * np.max(np.abs(D))
