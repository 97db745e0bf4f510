"""GPU parity of the learned neighbourhood-inverse preconditioner (the network
of the learned guess used as a block preconditioner) against the oracle
(oracle.learned_precond, oracle.mlp, oracle.precond), all through the C ABI.

* features: BF16 values, >= 99 % identical (a zero may carry either sign) and
  every value within one BF16 ulp of the oracle's FP64 features rounded once
  (only FP64 last-bit differences at a rounding boundary can differ);
* targets: the library's map from its own raw rows and inverse self blocks
  equals the oracle's map applied to the same blocks, to FP32 rounding
  (<= 1e-6 of the largest);
* the learned preconditioner for given parameters: the oracle runs the same
  network (BF16 rounding points emulated) on the same features, maps the
  outputs back to raw rows (adding its own FP64 inverse self blocks) and
  symmetrises them; blocks within 2e-3 of the largest (FP32 accumulation
  order, BF16 boundary cases, the library's FP32 inverse self blocks);
* trained by the library on a few clouds of the 10^6-wire cloud's density,
  the learned preconditioner drives COCG to the oracle's currents (<= 1e-4,
  FP32 with FP64 refinement) on a held-out cloud in fewer steps than the
  block-diagonal preconditioner; the steps of the computed neighbourhood
  inverse are reported beside it.
"""
import math

import numpy as np
import pytest

from oracle import learned_precond as lp
from oracle import mlp as omlp
from oracle import mom, precond, solve as osolve
from paper_2410_03060_amd import workloads as W
from parity_util import say

pytestmark = pytest.mark.gpu

NB = 7


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_03060_amd import binding
    binding.lib()
    return binding


def _np(t):
    return t.detach().cpu().numpy()


def _caller_rows(cl, size):
    """GPU row index (internal wire order) of every oracle row (caller order)."""
    row_ptr, col_idx, perm, _ = cl.pattern()
    iperm = np.empty_like(perm)
    iperm[perm] = np.arange(len(perm), dtype=perm.dtype)
    p = np.arange(len(perm))
    s = np.arange(size)
    c = np.arange(NB)
    return ((iperm[p][:, None, None] * size + s[None, :, None]) * NB + c[None, None, :]).reshape(-1)


def _cloud(seed=61, n=160):
    return W.random_cloud(seed, n, box_lam=2.5, d_c_lam=1.0)


@pytest.mark.parametrize("size", [3, 8])
def test_features_and_targets_match_oracle(B, size):
    cloud = _cloud()
    cl = B.build_cloud(cloud)
    Z, P = B.fill_Z(cl, B.C64)
    Mr = B.nbhd_raw_rows(cl, Z, size)
    rows = _caller_rows(cl, size)
    nb = precond.neighbourhoods(cloud, size)
    fg = _np(B.nbhd_mlp_features(cl, Mr, size))[rows].view(np.uint16)
    fo = lp.features(cloud, nb, size)
    g = omlp.from_bf16_bits(fg)
    o = omlp.bf16(fo)
    same = np.mean(g == o)             # equal BF16 values (+0 and -0 count as equal)
    bad = int(np.sum(np.abs(g - o) > 2.0 ** -7 * np.abs(o) + 1e-12))
    say(f"[nbhd mlp] size {size}: features identical {same:.6f}, beyond one ulp {bad}")
    assert same >= 0.99 and bad == 0
    # targets: the library's map from its raw rows against the oracle's map of the same rows
    row_ptr, col_idx, perm, _ = cl.pattern()
    V = _np(B.nbhd_blocks(cl, Mr, size, B.C64)).astype(np.complex128)
    raw = {}
    for i in range(cl.n):
        for e in range(int(row_ptr[i]), int(row_ptr[i + 1])):
            raw[(int(perm[i]), int(perm[col_idx[e]]))] = V[e]
    raw = {(p, int(q)): raw[(p, int(q))] for p in range(cloud.n) for q in nb[p]}
    Tg = _np(B.nbhd_mlp_targets(cl, Mr, P, size))[rows]
    Pg = _np(P).astype(np.complex128)
    dinv = np.empty_like(Pg)
    dinv[perm] = Pg                    # the library's inverse self blocks, caller order
    To = lp.targets(cloud, nb, size, raw, dinv)
    err = np.max(np.abs(Tg - To)) / np.max(np.abs(To))
    say(f"   targets: max err / max {err:.2e}")
    assert err <= 1e-6


def test_learned_preconditioner_matches_oracle_assembly(B):
    import torch
    size = 6
    cloud = _cloud(seed=62, n=120)
    cl = B.build_cloud(cloud)
    _, P = B.fill_Z(cl, B.C64)
    th = W.mlp_init(3)
    lay, _ = omlp.param_layout()
    rng = np.random.default_rng(4)
    for _, b, _, o in lay:
        th[b:b + o] = 0.1 * rng.standard_normal(o)
    theta = torch.from_numpy(th.astype(np.float32)).cuda()
    M = B.nbhd_mlp_precond(cl, theta, P, size)
    rows = _caller_rows(cl, size)
    nb = precond.neighbourhoods(cloud, size)
    X = omlp.bf16(lp.features(cloud, nb, size))
    Y, _ = omlp.forward(th.astype(np.float32).astype(np.float64), X, emulate_bf16=True)
    Mo = precond.symmetrise(lp.raw_from_outputs(cloud, nb, size, Y), cloud.n).tobsr(blocksize=(NB, NB))
    ref = {}
    for p in range(cloud.n):
        for e in range(Mo.indptr[p], Mo.indptr[p + 1]):
            ref[(p, int(Mo.indices[e]))] = Mo.data[e]
    row_ptr, col_idx, perm, _ = cl.pattern()
    V = _np(B.nbhd_blocks(cl, M, size, B.C64)).astype(np.complex128)
    scale = max(np.max(np.abs(v)) for v in ref.values())
    worst = 0.0
    for i in range(cl.n):
        for e in range(int(row_ptr[i]), int(row_ptr[i + 1])):
            k = (int(perm[i]), int(perm[col_idx[e]]))
            worst = max(worst, float(np.max(np.abs(V[e] - ref.get(k, 0.0)))))
    say(f"[nbhd mlp] learned blocks vs oracle: max err / max {worst / scale:.2e}")
    assert worst <= 2e-3 * scale


def test_trained_learned_preconditioner(B):
    import torch
    from paper_2410_03060_amd import learned
    size = 6
    train = [W.c5_train_cloud(j) for j in range(6)]
    samples = learned.nbhd_samples(train, size)
    res = learned.train(samples, W.mlp_init(0), epochs=6, batch=4096, seed=0)
    err = learned.relative_target_error(res.theta, samples)
    say(f"[nbhd mlp] trained on {samples.feat.shape[0]} rows: final loss {res.losses[-1]:.4e}, "
        f"relative error {err:.3f}")
    # held out: 2,000 wires at the same density (1.91 per cubic wavelength), d_c = 1 wavelength
    cloud = W._sphere_cloud(5999, 2000, 50.0 * (2000 / 1e6) ** (1.0 / 3.0), 1.0)
    inc = W.azimuth_incidences(4)
    cl = B.build_cloud(cloud)
    Z, P = B.fill_Z(cl, B.C64)
    o = dict(tol=1e-6, method=B.COCG, restart=2000, inner_tol=1e-5, max_cycles=60)
    Ml = B.nbhd_mlp_precond(cl, res.theta, P, size)
    Xl, il = B.solve(cl, Z, Ml, inc.k_hat, inc.e_hat, B.solve_opts(precond=B.PRECOND_NBHD, **o))
    Xb, ib = B.solve(cl, Z, P, inc.k_hat, inc.e_hat, B.solve_opts(precond=B.PRECOND_BLOCK, **o))
    Me = B.nbhd_precond(cl, Z, size)
    Xe, ie = B.solve(cl, Z, Me, inc.k_hat, inc.e_hat, B.solve_opts(precond=B.PRECOND_NBHD, **o))
    Zs, _ = mom.snfc_matrix(cloud)
    xo = osolve.sparse_solve(Zs, mom.excitation(cloud, inc.k_hat, inc.e_hat))
    cerr = float(np.max(np.linalg.norm(_np(Xl) - xo, axis=0) / np.linalg.norm(xo, axis=0)))
    say(f"[nbhd mlp] held-out N={cloud.n}: steps learned {il['iterations']}, block-Jacobi {ib['iterations']}, "
        f"computed neighbourhood inverse {ie['iterations']}; current err {cerr:.2e}")
    assert il["max_rel_residual"] <= 1e-6 and cerr <= 1e-4
    assert il["iterations"] < ib["iterations"]
