"""Pins of the learned-guess oracle (oracle.mlp) against outside facts.

* the network and its gradient against torch.nn / autograd in float64 and
  against central finite differences;
* Adam against torch.optim.Adam;
* BF16 rounding against torch's float32 -> bfloat16 conversion;
* the neighbour lists against brute force;
* the features against the physics they encode: invariance under rigid
  motions of the whole scene (wires and incident wave), under reversal of any
  wire's tangent, and agreement with the excitation of eq. (4) computed by
  the oracle's independent triangle transform;
* the targets against the solved physics: reversing a wire's tangent in the
  MoM system, or translating the whole cloud, leaves them unchanged.
"""
import math

import numpy as np
import pytest
import torch

from oracle import mlp, mom, solve
from paper_2410_03060_amd import workloads as W

LAM = W.WAVELENGTH
K = 2.0 * math.pi / LAM


def _rand_rows(seed, B):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((B, mlp.N_FEAT)), rng.standard_normal((B, mlp.N_OUT))


def _torch_net(theta):
    layers = []
    for li, (W_, b_) in enumerate(mlp.unpack(theta)):
        lin = torch.nn.Linear(W_.shape[0], W_.shape[1], dtype=torch.float64)
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(W_.T.copy()))
            lin.bias.copy_(torch.from_numpy(b_.copy()))
        layers.append(lin)
        if li < 3:
            layers.append(torch.nn.SiLU())
    return torch.nn.Sequential(*layers)


def _theta(seed):
    th = W.mlp_init(seed)
    # non-zero biases so that a dropped bias term shows
    lay, _ = mlp.param_layout()
    rng = np.random.default_rng(seed + 1)
    for _, b, _, o in lay:
        th[b:b + o] = 0.1 * rng.standard_normal(o)
    return th


def test_param_layout_count():
    _, n = mlp.param_layout()
    assert n == 192 * 128 + 128 + 2 * (128 * 128 + 128) + 128 * 14 + 14
    assert W.mlp_init(0).shape == (n,)


def test_forward_matches_torch():
    th = _theta(3)
    X, _ = _rand_rows(4, 37)
    Y, _ = mlp.forward(th, X)
    Yt = _torch_net(th)(torch.from_numpy(X)).detach().numpy()
    np.testing.assert_allclose(Y, Yt, rtol=1e-12, atol=1e-12)


def test_gradient_matches_autograd_and_finite_differences():
    th = _theta(5)
    X, T = _rand_rows(6, 23)
    loss, g = mlp.loss_and_grad(th, X, T)
    net = _torch_net(th)
    Y = net(torch.from_numpy(X))
    lt = torch.mean((Y - torch.from_numpy(T)) ** 2)
    lt.backward()
    assert abs(loss - lt.item()) < 1e-12 * max(1.0, abs(loss))
    lay, _ = mlp.param_layout()
    mods = [m for m in net if isinstance(m, torch.nn.Linear)]
    for (w, b, i, o), m in zip(lay, mods):
        np.testing.assert_allclose(g[w:w + i * o].reshape(i, o), m.weight.grad.numpy().T,
                                   rtol=1e-9, atol=1e-14)
        np.testing.assert_allclose(g[b:b + o], m.bias.grad.numpy(), rtol=1e-9, atol=1e-14)
    # central differences on a spread of parameters (every layer, weights and biases)
    rng = np.random.default_rng(7)
    idx = np.concatenate([rng.choice(np.arange(w, w + i * o), 6, replace=False) for w, _, i, o in lay]
                         + [np.arange(b, b + 2) for _, b, _, _ in lay])
    h = 1e-6
    for j in idx:
        tp = th.copy()
        tp[j] += h
        tm = th.copy()
        tm[j] -= h
        fd = (mlp.loss_and_grad(tp, X, T)[0] - mlp.loss_and_grad(tm, X, T)[0]) / (2 * h)
        assert abs(fd - g[j]) <= 1e-7 * max(1e-3, abs(g[j])) + 1e-10, (j, fd, g[j])


def test_emulated_bf16_gradient_stays_close_to_exact():
    th = _theta(8)
    X, T = _rand_rows(9, 256)
    _, g = mlp.loss_and_grad(th, X, T)
    _, gb = mlp.loss_and_grad(th, X, T, emulate_bf16=True)
    lay, _ = mlp.param_layout()
    for w, b, i, o in lay:
        a, c = g[w:b + o], gb[w:b + o]
        cos = a @ c / (np.linalg.norm(a) * np.linalg.norm(c))
        assert cos > 0.999
        assert np.linalg.norm(a - c) / np.linalg.norm(a) < 2e-2


def test_adam_matches_torch():
    rng = np.random.default_rng(10)
    th = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    p = torch.nn.Parameter(torch.from_numpy(th.copy()))
    opt = torch.optim.Adam([p], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 5):
        g = rng.standard_normal(50)
        th, m, v = mlp.adam(th, m, v, g, t, 3e-3)
        p.grad = torch.from_numpy(g.copy())
        opt.step()
        np.testing.assert_allclose(th, p.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(11)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-20, 20, 10000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 65504.0, 1e-40]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(x), ref)
    assert mlp.bf16(np.array([1.0 + 2 ** -8]))[0] == 1.0          # tie to even
    np.testing.assert_array_equal(mlp.from_bf16_bits(mlp.bf16_bits(x)), ref)


def test_knn_matches_brute_force():
    cl = W.random_cloud(12, 300, box_lam=5.0, d_c_lam=1.5)
    nbr, count = mlp.knn(cl)
    c = cl.center
    for p in range(cl.n):
        d2 = [((c[q, 0] - c[p, 0]) ** 2 + (c[q, 1] - c[p, 1]) ** 2) + (c[q, 2] - c[p, 2]) ** 2
              for q in range(cl.n)]
        near = sorted((d2[q], q) for q in range(cl.n) if q != p and d2[q] <= cl.d_c ** 2)
        assert count[p] == len(near)
        want = [q for _, q in near[:16]] + [-1] * max(0, 16 - len(near))
        assert list(nbr[p]) == want
    assert count.max() > 16           # the cap is exercised


def _scene(seed, n=60, box=3.0):
    cl = W.random_cloud(seed, n, box_lam=box, d_c_lam=1.2)
    inc = W.random_incidences(np.random.default_rng(seed + 100), 3)
    return cl, inc


def _rotation(seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def test_features_invariant_under_rigid_motion_of_the_scene():
    cl, inc = _scene(13)
    F0 = mlp.features(cl, inc.k_hat, inc.e_hat)
    Q = _rotation(14)
    shift = np.array([0.37, -1.1, 0.52])
    cl2 = W.single_cloud(cl.center @ Q.T + shift, cl.tangent @ Q.T, cl.length, LAM, cl.d_c)
    F1 = mlp.features(cl2, inc.k_hat @ Q.T, inc.e_hat @ Q.T, nbrs=mlp.knn(cl))
    np.testing.assert_allclose(F1, F0, atol=1e-9)
    assert np.count_nonzero(F0[:, 16::11]) > 0           # neighbours present


def test_features_invariant_under_tangent_reversal():
    cl, inc = _scene(15)
    F0 = mlp.features(cl, inc.k_hat, inc.e_hat)
    t = cl.tangent.copy()
    t[::3] *= -1.0
    cl2 = W.single_cloud(cl.center, t, cl.length, LAM, cl.d_c)
    np.testing.assert_allclose(mlp.features(cl2, inc.k_hat, inc.e_hat), F0, atol=1e-12)


def test_own_drive_features_are_the_canonical_excitation():
    cl, inc = _scene(16)
    F = mlp.features(cl, inc.k_hat, inc.e_hat).reshape(cl.n, 3, mlp.N_FEAT)
    u = mom.excitation(cl, inc.k_hat, inc.e_hat).reshape(cl.n, 7, 3)
    s = mlp.canonical_sign(cl.tangent, inc.e_hat)
    D = cl.length / 8.0
    for r in range(3):
        ph = np.exp(1j * K * (cl.center @ inc.k_hat[r]))
        uc = np.where(s[:, r:r + 1] > 0, u[:, :, r], u[:, ::-1, r]) * s[:, r:r + 1]
        want = uc * ph[:, None] / D[:, None]
        got = F[:, r, 2:16:2] + 1j * F[:, r, 3:16:2]
        np.testing.assert_allclose(got, want, atol=1e-12)


def test_neighbour_drive_features_match_the_neighbours_excitation():
    cl, inc = _scene(17)
    nbr, _ = mlp.knn(cl)
    F = mlp.features(cl, inc.k_hat, inc.e_hat).reshape(cl.n, 3, mlp.N_FEAT)
    u = mom.excitation(cl, inc.k_hat, inc.e_hat).reshape(cl.n, 7, 3)
    s = mlp.canonical_sign(cl.tangent, inc.e_hat)
    D = cl.length / 8.0
    checked = 0
    for p in range(cl.n):
        for j in range(16):
            q = nbr[p, j]
            if q < 0:
                continue
            for r in range(3):
                beta = K * (cl.tangent[q] @ inc.k_hat[r])
                env = D[q] * np.sinc(beta * D[q] / (2 * math.pi)) ** 2
                want = s[q, r] * u[q, 3, r] / env * np.exp(1j * K * (cl.center[p] @ inc.k_hat[r]))
                b = 16 + 11 * j
                assert abs(F[p, r, b + 4] + 1j * F[p, r, b + 5] - want) < 1e-11
                d = cl.center[q] - cl.center[p]
                assert abs(F[p, r, b] - np.linalg.norm(d) / cl.d_c) < 1e-14
                assert F[p, r, b + 10] == 1.0
                kd = K * np.linalg.norm(d)
                assert abs(F[p, r, b + 8] + 1j * F[p, r, b + 9] - np.exp(-1j * kd)) < 1e-12
                checked += 1
    assert checked > 50


def _solve_dense(cl, inc):
    Z, _ = mom.snfc_matrix(cl)
    u = mom.excitation(cl, inc.k_hat, inc.e_hat)
    return solve.dense_solve(Z.toarray(), u)


def test_targets_unchanged_when_a_wire_is_reversed_in_the_mom_system():
    cl, inc = _scene(18, n=25, box=2.0)
    Y0 = mlp.targets(cl, inc.k_hat, inc.e_hat, _solve_dense(cl, inc))
    t = cl.tangent.copy()
    t[[0, 4, 7]] *= -1.0
    cl2 = W.single_cloud(cl.center, t, cl.length, LAM, cl.d_c)
    Y1 = mlp.targets(cl2, inc.k_hat, inc.e_hat, _solve_dense(cl2, inc))
    assert np.max(np.abs(Y1 - Y0)) < 1e-9 * np.max(np.abs(Y0))
    # ... whereas the raw currents of the reversed wires do change
    x0 = _solve_dense(cl, inc).reshape(25, 7, 3)
    x1 = _solve_dense(cl2, inc).reshape(25, 7, 3)
    assert np.max(np.abs(x1[0] - x0[0])) > 1e-3 * np.max(np.abs(x0[0]))
    np.testing.assert_allclose(x1[0], -x0[0, ::-1], atol=1e-9 * np.max(np.abs(x0)))


def test_targets_unchanged_when_the_cloud_is_translated():
    cl, inc = _scene(19, n=20, box=2.0)
    Y0 = mlp.targets(cl, inc.k_hat, inc.e_hat, _solve_dense(cl, inc))
    cl2 = W.single_cloud(cl.center + np.array([1.234, -0.77, 3.1]), cl.tangent, cl.length, LAM, cl.d_c)
    Y1 = mlp.targets(cl2, inc.k_hat, inc.e_hat, _solve_dense(cl2, inc))
    assert np.max(np.abs(Y1 - Y0)) < 1e-9 * np.max(np.abs(Y0))


def test_currents_round_trip_through_targets():
    cl, inc = _scene(20, n=30)
    x = (np.random.default_rng(21).standard_normal((30 * 7, 3))
         + 1j * np.random.default_rng(22).standard_normal((30 * 7, 3)))
    Y = mlp.targets(cl, inc.k_hat, inc.e_hat, x)
    np.testing.assert_allclose(mlp.currents_from_outputs(cl, inc.k_hat, inc.e_hat, Y), x, atol=1e-13)


def test_features_need_finite_dc():
    cl = W.random_cloud(23, 5)
    with pytest.raises(ValueError):
        mlp.knn(cl)


def test_neighbour_features_swap_consistently_between_the_two_wires_of_a_pair():
    """Seen from p' the roles of the two wires exchange and d changes sign;
    the neighbour's length and k.tau must equal what p' reports about itself."""
    cl, inc = _scene(24, n=80)
    nbr, count = mlp.knn(cl)
    F = mlp.features(cl, inc.k_hat, inc.e_hat).reshape(cl.n, 3, mlp.N_FEAT)
    D = cl.length / 8.0
    checked = 0
    for p in range(cl.n):
        for j in range(16):
            q = nbr[p, j]
            if q < 0 or p not in list(nbr[q]):
                continue
            jq = list(nbr[q]).index(p)
            a = F[p, :, 16 + 11 * j:16 + 11 * j + 11]
            b = F[q, :, 16 + 11 * jq:16 + 11 * jq + 11]
            np.testing.assert_allclose(b[:, 0], a[:, 0], atol=1e-15)
            np.testing.assert_allclose(b[:, 1], -a[:, 2], atol=1e-13)
            np.testing.assert_allclose(b[:, 2], -a[:, 1], atol=1e-13)
            np.testing.assert_allclose(b[:, 3], a[:, 3], atol=1e-15)
            np.testing.assert_allclose(b[:, 8:11], a[:, 8:11], atol=1e-15)
            np.testing.assert_allclose(a[:, 6], F[q, :, 0], atol=1e-13)
            np.testing.assert_allclose(b[:, 6], F[p, :, 0], atol=1e-13)
            # k_hat . tau_q from the phase slope of q's own drive features
            psi = F[q, :, 2:16:2] + 1j * F[q, :, 3:16:2]
            ok = np.abs(psi[:, 0]) > 1e-6
            slope = -np.angle(psi[ok, 1] / psi[ok, 0]) / (K * D[q])
            np.testing.assert_allclose(a[ok, 7], slope, atol=1e-9)
            checked += 1
    assert checked > 30


def test_features_of_a_hand_built_three_wire_scene():
    """Values worked out by hand: A along x at the origin, B along y at 0.5
    lambda on the y axis, C along -x at 0.3 lambda on the x axis; the wave
    travels along -z with e = x, d_c = 1 lambda."""
    c = np.array([[0.0, 0.0, 0.0], [0.0, 0.5, 0.0], [0.3, 0.0, 0.0]]) * LAM
    t = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [-1.0, 0.0, 0.0]])
    L = np.array([0.5, 0.45, 0.55]) * LAM
    cl = W.single_cloud(c, t, L, LAM, 1.0 * LAM)
    F = mlp.features(cl, np.array([[0.0, 0.0, -1.0]]), np.array([[1.0, 0.0, 0.0]]))
    a = F[0]
    assert a[0] == 0.0 and abs(a[1] - 2 / 16) < 1e-15
    # broadside incidence: no phase along A, drive (tau.e) sinc^2(0) = 1 on every rooftop
    np.testing.assert_allclose(a[2:16:2], 1.0, atol=1e-15)
    np.testing.assert_allclose(a[3:16:2], 0.0, atol=1e-15)
    # retardation exp(-j 2 pi |d|/lambda): 0.3 lambda -> angle -108 deg, 0.5 lambda -> -1
    c3, s3 = math.cos(0.6 * math.pi), -math.sin(0.6 * math.pi)
    # nearest: C (0.3 lambda), canonical tangent +x (its raw -x is flipped)
    np.testing.assert_allclose(a[16:27], [0.3, 0.3, 0.3, 1.0, 1.0, 0.0, 0.5, 0.0, c3, s3, 1.0], atol=1e-14)
    # then B (0.5 lambda), tangent y: perpendicular and undriven
    np.testing.assert_allclose(a[27:38], [0.5, 0.0, 0.5, 0.0, 0.0, 0.0, -0.5, 0.0, -1.0, 0.0, 1.0], atol=1e-14)
    assert np.all(a[38:] == 0.0)
    b = F[1]      # B sees A (0.5) then C (sqrt(0.34)); B itself is undriven
    assert abs(b[0] - (-0.5)) < 1e-14 and np.all(np.abs(b[2:16]) < 1e-15)
    d = math.sqrt(0.34)
    cd, sd = math.cos(2 * math.pi * d), -math.sin(2 * math.pi * d)
    np.testing.assert_allclose(b[16:27], [0.5, -0.5, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, -1.0, 0.0, 1.0], atol=1e-14)
    np.testing.assert_allclose(b[27:38], [d, -0.5, 0.3, 0.0, 1.0, 0.0, 0.5, 0.0, cd, sd, 1.0], atol=1e-14)


def test_targets_vanish_for_uncoupled_wires():
    """With d_c below every spacing the S-NFC matrix is block diagonal, each wire
    carries its isolated response, and the network has nothing to predict."""
    cl = W.random_cloud(25, 30, box_lam=4.0, d_c_lam=0.05)
    inc = W.random_incidences(np.random.default_rng(26), 2)
    assert mom.near_pairs(cl.center, cl.cloud_off, cl.d_c)[0].size == 0
    x = _solve_dense(cl, inc)
    Y = mlp.targets(cl, inc.k_hat, inc.e_hat, x)
    assert np.max(np.abs(Y)) < 1e-10 * np.max(np.abs(x))
    # with coupling the targets do not vanish
    cl2 = W.single_cloud(cl.center, cl.tangent, cl.length, LAM, 2.0 * LAM)
    Y2 = mlp.targets(cl2, inc.k_hat, inc.e_hat, _solve_dense(cl2, inc))
    assert np.max(np.abs(Y2)) > 1e-3
