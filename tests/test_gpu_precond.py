"""GPU parity of the cluster block-Jacobi preconditioner against the FP64 oracle.

Tolerances:
  * internal wire order: identical to the oracle's cell order (index work);
  * cluster table: identical to runs of 8 wires per cloud (index work);
  * inverse blocks: relative Frobenius error per block <= kappa_k * e_fill,
    kappa_k the oracle's condition number of the cluster's diagonal submatrix
    and e_fill the per-block error bound of the fill it inverts (first-order
    perturbation of an inverse: |dM| / |M| <= kappa |dD| / |D|): 1e-10 for the
    FP64 path, 3e-5 for the FP32 path (plus 1e-6 for storing the FP64
    inverse in FP32); padding of short clusters is the identity exactly;
  * apply: against the library's own blocks <= 1e-12 (FP64) / 2e-6 (FP32)
    relative, and against the oracle within the block bound;
  * solves: currents <= 1e-10 (FP64 path) / <= 1e-4 (FP32 + FP64 refinement)
    of the oracle's sparse direct solution, as for block-Jacobi.
"""
import math

import numpy as np
import pytest

from oracle import mom, precond, solve as osolve
from paper_2410_03060_amd import workloads as W
from parity_util import current_err, say

pytestmark = pytest.mark.gpu


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


def _clouds():
    lam = W.WAVELENGTH
    empty = W.single_cloud(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0), lam, 1.5 * lam)
    return {
        "c1": W.c1().cloud,
        "c1_dense": W.c1(d_c=math.inf).cloud,
        "ragged_301": W.random_cloud(41, 301, box_lam=7.0, d_c_lam=1.5),
        "multi": W.concat_clouds([W.random_cloud(42, 203, box_lam=6.0, d_c_lam=1.5), empty,
                                  W.random_cloud(43, 5, box_lam=2.0, d_c_lam=1.5),
                                  W.random_cloud(44, 97, box_lam=5.0, d_c_lam=1.5)]),
    }


@pytest.mark.parametrize("name", ["c1", "c1_dense", "ragged_301", "multi"])
def test_internal_order_is_the_cell_order(B, name):
    cloud = _clouds()[name]
    say(f"[precond] internal order {name}: N={cloud.n} clouds={cloud.n_clouds}")
    cl = B.build_cloud(cloud)
    perm = cl.pattern()[2]
    assert np.array_equal(perm, precond.cell_order(cloud))


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("name", ["ragged_301", "multi"])
def test_cluster_blocks(B, name, prec):
    cloud = _clouds()[name]
    P = B.C128 if prec == "c128" else B.C64
    say(f"[precond] cluster blocks {name} {prec}: N={cloud.n}")
    cl = B.build_cloud(cloud)
    Z, _ = B.fill_Z(cl, P, with_pinv=False)
    M = B.cluster_precond(cl, Z, P)
    groups = precond.clusters(cloud, 8)
    assert B.cluster_count(cl) == len(groups)
    # table: runs of 8 wires per cloud, internal indices
    tab = _np(B.cluster_table(cl, M))
    exp = [(w0, min(8, int(cloud.cloud_off[k + 1]) - w0))
           for k in range(cloud.n_clouds)
           for w0 in range(int(cloud.cloud_off[k]), int(cloud.cloud_off[k + 1]), 8)]
    assert tab.tolist() == [list(e) for e in exp]
    Mg = _np(B.cluster_blocks(cl, M, P)).astype(np.complex128)
    Zs, _ = mom.snfc_matrix(cloud)
    Mo = precond.cluster_inverse(Zs, groups, 8)
    kap = precond.condition_numbers(Zs, groups)
    e_fill, e_store = (1e-10, 0.0) if prec == "c128" else (3e-5, 1e-6)
    err = np.linalg.norm(Mg - Mo, axis=(1, 2)) / np.linalg.norm(Mo, axis=(1, 2))
    bound = kap * e_fill + e_store
    worst = int(np.argmax(err / bound))
    say(f"  {len(groups)} clusters, kappa max {kap.max():.1f}, err max {err.max():.2e}, "
        f"worst err/bound {err[worst] / bound[worst]:.3f}")
    assert np.all(err <= bound)
    for k, g in enumerate(groups):   # identity padding of short clusters, exactly
        m = 7 * len(g)
        if m < 56:
            assert np.array_equal(Mg[k, m:, m:], np.eye(56 - m))
            assert not Mg[k, :m, m:].any() and not Mg[k, m:, :m].any()


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("s", [1, 5, 64, 70])
def test_cluster_apply(B, prec, s):
    import torch
    cloud = _clouds()["multi"]
    P = B.C128 if prec == "c128" else B.C64
    say(f"[precond] cluster apply {prec} s={s}: N={cloud.n}")
    cl = B.build_cloud(cloud)
    Z, _ = B.fill_Z(cl, P, with_pinv=False)
    M = B.cluster_precond(cl, Z, P)
    rng = np.random.default_rng(s)
    Xi = rng.standard_normal((7 * cloud.n, s)) + 1j * rng.standard_normal((7 * cloud.n, s))
    dt = torch.complex128 if prec == "c128" else torch.complex64
    Xd = torch.as_tensor(Xi, dtype=dt, device="cuda")
    Y = _np(B.cluster_apply(cl, M, Xd, P)).astype(np.complex128)
    Xr = _np(Xd).astype(np.complex128)
    # against the library's own blocks (kernel arithmetic only)
    Mg = _np(B.cluster_blocks(cl, M, P)).astype(np.complex128)
    tab = _np(B.cluster_table(cl, M))
    Yg = np.zeros_like(Xr)
    for k, (w0, nw) in enumerate(tab):
        r = slice(7 * w0, 7 * (w0 + nw))
        Yg[r] = Mg[k, :7 * nw, :7 * nw] @ Xr[r]
    tol = 1e-12 if prec == "c128" else 2e-6
    e1 = np.linalg.norm(Y - Yg) / np.linalg.norm(Yg)
    # against the oracle (caller order)
    perm = precond.cell_order(cloud)
    rows = (7 * perm[:, None] + np.arange(7)[None, :]).reshape(-1)
    Xc = np.empty_like(Xr)
    Xc[rows] = Xr
    Zs, _ = mom.snfc_matrix(cloud)
    groups = precond.clusters(cloud, 8)
    Yo = precond.cluster_apply(precond.cluster_inverse(Zs, groups, 8), groups, Xc)[rows]
    kap = precond.condition_numbers(Zs, groups).max()
    e2 = np.linalg.norm(Y - Yo) / np.linalg.norm(Yo)
    say(f"  vs own blocks {e1:.2e}, vs oracle {e2:.2e} (kappa max {kap:.1f})")
    assert e1 <= tol
    assert e2 <= kap * (1e-10 if prec == "c128" else 3e-5) + (0.0 if prec == "c128" else 1e-6)


def _oracle_x(cloud, inc):
    Zs, _ = mom.snfc_matrix(cloud)
    u = mom.excitation(cloud, inc.k_hat, inc.e_hat)
    return osolve.sparse_solve(Zs, u)


@pytest.mark.parametrize("method", ["cocg", "gmres", "gcr"])
@pytest.mark.parametrize("guess", [0, 2])
def test_c2_solve_with_cluster_preconditioner(B, method, guess):
    wl = W.c2()
    say(f"[precond] c2 complex64 + FP64 refinement, {method}, cluster preconditioner, use_x0={guess}")
    cl = B.build_cloud(wl.cloud)
    Z, Pb = B.fill_Z(cl, B.C64)
    M = B.cluster_precond(cl, Z, B.C64)
    meth = {"cocg": B.COCG, "gmres": B.GMRES, "gcr": B.GCR}[method]
    restarted = meth != B.COCG
    kw = dict(tol=1e-6, method=meth, restart=30 if restarted else 500,
              inner_tol=1e-4 if restarted else 1e-2, use_x0=guess)
    X, info = B.solve(cl, Z, M, wl.inc.k_hat, wl.inc.e_hat, B.solve_opts(precond=B.PRECOND_CLUSTER, **kw))
    _, info_b = B.solve(cl, Z, Pb, wl.inc.k_hat, wl.inc.e_hat, B.solve_opts(**kw))
    say(f"  cluster: cycles {info['cycles']} iters {info['iterations']} res {info['max_rel_residual']:.2e}; "
        f"block-Jacobi iters {info_b['iterations']}")
    assert info["max_rel_residual"] <= 1e-6
    e = current_err(_np(X), _oracle_x(wl.cloud, wl.inc))
    say(f"  current err {e.max():.3e}")
    assert e.max() <= 1e-4
    assert info["iterations"] < info_b["iterations"]


def test_complex128_cocg_with_cluster_preconditioner(B):
    wl = W.c1()
    say("[precond] c1 complex128 COCG, cluster preconditioner")
    cl = B.build_cloud(wl.cloud)
    Z, _ = B.fill_Z(cl, B.C128, with_pinv=False)
    M = B.cluster_precond(cl, Z, B.C128)
    X, info = B.solve(cl, Z, M, wl.inc.k_hat, wl.inc.e_hat,
                      B.solve_opts(tol=1e-12, method=B.COCG, restart=500, inner_tol=1e-12, prec=B.C128,
                                   precond=B.PRECOND_CLUSTER))
    say(f"  cycles {info['cycles']} iters {info['iterations']} res {info['max_rel_residual']:.2e}")
    e = current_err(_np(X), _oracle_x(wl.cloud, wl.inc))
    say(f"  current err {e.max():.3e}")
    assert e.max() <= 1e-10


@pytest.mark.parametrize("method", ["cocg", "gmres", "gcr"])
def test_multicloud_with_cluster_preconditioner(B, method):
    cloud = _clouds()["multi"]
    inc = W.azimuth_incidences(6)
    say(f"[precond] multi-cloud N={cloud.n} clouds={cloud.n_clouds} R=6 {method}")
    cl = B.build_cloud(cloud)
    Z, _ = B.fill_Z(cl, B.C64, with_pinv=False)
    M = B.cluster_precond(cl, Z, B.C64)
    meth = {"cocg": B.COCG, "gmres": B.GMRES, "gcr": B.GCR}[method]
    restarted = meth != B.COCG
    X, info = B.solve(cl, Z, M, inc.k_hat, inc.e_hat,
                      B.solve_opts(tol=1e-6, method=meth, restart=30 if restarted else 500,
                                   inner_tol=1e-4 if restarted else 1e-2, precond=B.PRECOND_CLUSTER))
    say(f"  cycles {info['cycles']} iters {info['iterations']} res {info['max_rel_residual']:.2e}")
    assert info["max_rel_residual"] <= 1e-6
    e = current_err(_np(X), _oracle_x(cloud, inc))
    say(f"  current err {e.max():.3e}")
    assert e.max() <= 1e-4


def test_cocg_compaction_with_cluster_preconditioner(B):
    """The stored z = M r is carried through column compaction."""
    cloud = W.concat_clouds([W.random_cloud(12, 1500, box_lam=10.0, d_c_lam=1.5),
                             W.random_cloud(14, 603, box_lam=6.0, d_c_lam=1.5)])
    inc = W.random_incidences(np.random.default_rng(13), 40)
    say(f"[precond] COCG compaction with clusters: N={cloud.n} R=40")
    cl = B.build_cloud(cloud)
    Z, _ = B.fill_Z(cl, B.C64, with_pinv=False)
    M = B.cluster_precond(cl, Z, B.C64)
    B.profile_enable(True)
    X, info = B.solve(cl, Z, M, inc.k_hat, inc.e_hat,
                      B.solve_opts(tol=1e-6, method=B.COCG, restart=500, inner_tol=1e-3, precond=B.PRECOND_CLUSTER))
    B.profile_enable(False)
    prof = B.profile_read()
    say(f"  cycles {info['cycles']} iters {info['iterations']} res {info['max_rel_residual']:.2e} "
        f"compactions {prof.get('cocg_compact', {}).get('launches', 0)}")
    assert "cocg_compact" in prof
    assert np.all(info["rel_res"] <= 1e-6)
    e = current_err(_np(X), _oracle_x(cloud, inc))
    say(f"  current err {e.max():.3e}")
    assert e.max() <= 1e-4


def test_other_buffers_are_rejected_as_cluster_preconditioner(B):
    """The host checks the first and last cluster entries before any launch:
    the block-Jacobi inverses passed where a cluster buffer is expected fail
    with CHAFF_EINVAL (the check reads 16 bytes of the valid buffer)."""
    import torch
    cloud = _clouds()["ragged_301"]
    say(f"[precond] wrong buffer rejected: N={cloud.n}")
    cl = B.build_cloud(cloud)
    Z, P = B.fill_Z(cl, B.C64)
    X = torch.zeros((7 * cloud.n, 2), dtype=torch.complex64, device="cuda")
    with pytest.raises(B.ChaffError) as e:
        B.cluster_apply(cl, P, X, B.C64)
    assert e.value.status == B.EINVAL
    inc = W.azimuth_incidences(2)
    with pytest.raises(B.ChaffError) as e:
        B.solve(cl, Z, P, inc.k_hat, inc.e_hat,
                B.solve_opts(tol=1e-6, method=B.COCG, restart=100, precond=B.PRECOND_CLUSTER))
    assert e.value.status == B.EINVAL
