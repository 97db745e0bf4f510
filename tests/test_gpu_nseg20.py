"""GPU parity of the whole path with the paper's own discretisation: 20
segments and 19 rooftop unknowns per wire (Sec. II-A), against the FP64
oracle evaluated with n_seg = 20.

Tolerances are those of the 8-segment path: pair sets identical; blocks
<= 1e-11 (complex128) and the row-aware FP32 bar (complex64); excitation
<= 1e-13; product <= 2e-5; currents <= 1e-10 (complex128) and <= 1e-4
(complex64 with FP64 refinement); RCS <= 1e-6 dB (complex128) and 0.1 dB
(complex64).
"""
import math

import numpy as np
import pytest

from oracle import mom, solve as osolve
from paper_2410_03060_amd import workloads as W
from parity_util import current_err, db_err, fp32_block_check, gpu_blocks_caller, gpu_pairs, rel_block_err, say

pytestmark = pytest.mark.gpu

NS = 20
NBW = NS - 1


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_03060_amd import binding
    binding.lib()
    return binding


def _cloud(seed=11, n=90, box=3.0, d_c=1.0):
    return W.random_cloud(seed, n, box_lam=box, d_c_lam=d_c, n_seg=NS)


def test_pairs_and_blocks_complex128(B):
    cloud = _cloud()
    k = 2 * math.pi / cloud.wavelength
    say(f"[nseg20] pairs and complex128 blocks: N={cloud.n}")
    cl = B.build_cloud(cloud)
    assert cl.nb == NBW
    I, J = gpu_pairs(cl)
    Io, Jo = mom.near_pairs(cloud.center, cloud.cloud_off, cloud.d_c)
    assert np.array_equal(I, Io) and np.array_equal(J, Jo)
    Z, P = B.fill_Z(cl, B.C128)
    assert tuple(Z.shape[1:]) == (NBW, NBW)
    rows, cols, Zg = gpu_blocks_caller(cl, Z)
    Zo = mom.cloud_blocks(cloud, n_seg=NS, rows=rows, cols=cols)
    err = rel_block_err(Zg, Zo)
    say(f"  max rel block err {err.max():.3e} over {len(err)} blocks ({int((rows != cols).sum())} mutual)")
    assert err.max() <= 1e-11
    _, _, _, diag = cl.pattern()
    Pg = P.cpu().numpy()
    worst = max(np.abs(Zg[diag[i]] @ Pg[i] - np.eye(NBW)).max() for i in range(cl.n))
    say(f"  self block x inverse: max |Z P - I| {worst:.2e}")
    assert worst < 1e-9


def test_blocks_complex64(B):
    cloud = _cloud(seed=12, n=120)
    say(f"[nseg20] complex64 blocks: N={cloud.n}")
    cl = B.build_cloud(cloud)
    Z, _ = B.fill_Z(cl, B.C64, with_pinv=False)
    rows, cols, Zg = gpu_blocks_caller(cl, Z)
    Zo = mom.cloud_blocks(cloud, n_seg=NS, rows=rows, cols=cols)
    figs, ok = fp32_block_check(rows, cols, Zg, Zo)
    self_err = rel_block_err(Zg[rows == cols].astype(np.complex128), Zo[rows == cols])
    say(f"  {figs}; self blocks max rel {self_err.max():.3e}")
    assert ok and self_err.max() <= 1e-5


def test_excitation_and_product(B):
    import torch
    cloud = _cloud(seed=13, n=150)
    inc = W.random_incidences(np.random.default_rng(3), 5)
    say(f"[nseg20] excitation and product: N={cloud.n}")
    cl = B.build_cloud(cloud)
    U = B.excitation(cl, inc.k_hat, inc.e_hat).cpu().numpy()
    Uo = mom.excitation(cloud, inc.k_hat, inc.e_hat, n_seg=NS)
    assert np.abs(U - Uo).max() <= 1e-13 * np.abs(Uo).max()
    Z, _ = B.fill_Z(cl, B.C64, with_pinv=False)
    Zs, _ = mom.snfc_matrix(cloud, n_seg=NS)
    _, _, perm, _ = cl.pattern()
    rows_int = (NBW * perm[:, None] + np.arange(NBW)[None, :]).reshape(-1)
    rng = np.random.default_rng(5)
    for s in (1, 3, 64):
        Xc = rng.standard_normal((cloud.n * NBW, s)) + 1j * rng.standard_normal((cloud.n * NBW, s))
        Yo = Zs @ Xc
        Xi = torch.as_tensor(Xc[rows_int], dtype=torch.complex64, device="cuda")
        for v in (0, 1, 3, 5, 6):
            Yg = B.spmm(cl, Z, Xi, B.C64, variant=v).cpu().numpy().astype(np.complex128)
            e = np.linalg.norm(Yg - Yo[rows_int]) / np.linalg.norm(Yo)
            assert e <= 2e-5, (s, v, e)
        say(f"  s={s}: product within 2e-5 for variants 0, 1, 3, 5, 6")


@pytest.mark.parametrize("method", ["gmres", "cocg", "gcr"])
def test_complex128_solve_and_rcs(B, method):
    cloud = _cloud(seed=14, n=100)
    inc = W.azimuth_incidences(3)
    say(f"[nseg20] complex128 {method}: N={cloud.n}, 3 RHS")
    cl = B.build_cloud(cloud)
    Z, P = B.fill_Z(cl, B.C128)
    m = {"gmres": B.GMRES, "cocg": B.COCG, "gcr": B.GCR}[method]
    X, info = B.solve(cl, Z, P, inc.k_hat, inc.e_hat,
                      B.solve_opts(tol=1e-12, prec=B.C128, method=m, restart=60 if method != "cocg" else 2000))
    Zs, _ = mom.snfc_matrix(cloud, n_seg=NS)
    xo = osolve.sparse_solve(Zs, mom.excitation(cloud, inc.k_hat, inc.e_hat, n_seg=NS))
    e = current_err(X.cpu().numpy(), xo)
    say(f"  iters {info['iterations']} current err {e.max():.2e}")
    assert e.max() <= 1e-10
    sm = B.rcs(cl, X, -inc.k_hat, inc.e_hat, monostatic=True)[0].cpu().numpy()
    smo = mom.monostatic_rcs(cloud, xo, inc.k_hat, inc.e_hat, n_seg=NS)
    assert np.abs(sm - smo).max() <= 1e-9 * smo.max()
    if method == "gmres":   # bistatic on a 5-degree grid, both polarisations
        T, Pp, rh, th, ph = W.bistatic_grid(5.0)
        sg = B.rcs(cl, X[:, :1].contiguous(), np.concatenate([rh, rh]), np.concatenate([th, ph]),
                   monostatic=False)[0, 0].cpu().numpy()
        so = np.concatenate([mom.rcs_from_currents(cloud, xo[:, 0], rh, th, n_seg=NS)[0],
                             mom.rcs_from_currents(cloud, xo[:, 0], rh, ph, n_seg=NS)[0]])
        e_db, e_lo = db_err(sg, so)
        say(f"  bistatic {rh.shape[0]} x 2: {e_db:.2e} dB, below floor {e_lo:.2e}")
        assert e_db <= 1e-6 and e_lo <= 1e-8


@pytest.mark.parametrize("method", ["cocg", "gcr"])
def test_complex64_refined_solve_paper_cloud(B, method):
    """A 4,000-chaff cut of the paper's 13 GHz cloud (uniform sphere at 119.37 chaffs/m^3,
    identical half-wave chaffs of diameter 20 um, d_c = 2 lambda), 16 azimuths."""
    cloud = W.paper_cloud(4000, seed=3)
    inc = W.azimuth_incidences(16)
    say(f"[nseg20] complex64 + FP64 refinement, {method}: paper cloud N={cloud.n}, 16 RHS")
    cl = B.build_cloud(cloud)
    Z, P = B.fill_Z(cl, B.C64)
    m = {"cocg": B.COCG, "gcr": B.GCR}[method]
    X, info = B.solve(cl, Z, P, inc.k_hat, inc.e_hat,
                      B.solve_opts(tol=1e-6, method=m, restart=2000 if method == "cocg" else 30, inner_tol=1e-5))
    say(f"  pairs {cl.n_pairs}, cycles {info['cycles']} iters {info['iterations']} res {info['max_rel_residual']:.2e}")
    assert info["max_rel_residual"] <= 1e-6
    Zs, _ = mom.snfc_matrix(cloud, n_seg=NS)
    xo = osolve.sparse_solve(Zs, mom.excitation(cloud, inc.k_hat, inc.e_hat, n_seg=NS))
    e = current_err(X.cpu().numpy(), xo)
    sm = B.rcs(cl, X, -inc.k_hat, inc.e_hat, monostatic=True)[0].cpu().numpy()
    smo = mom.monostatic_rcs(cloud, xo, inc.k_hat, inc.e_hat, n_seg=NS)
    e_db, _ = db_err(sm, smo)
    say(f"  current err {e.max():.2e}, monostatic {e_db:.2e} dB")
    assert e.max() <= 1e-4 and e_db <= 0.1


def test_eight_segment_only_parts_refuse_twenty(B):
    import torch
    cloud = _cloud(seed=15, n=40)
    cl = B.build_cloud(cloud)
    Z, P = B.fill_Z(cl, B.C64)
    with pytest.raises(B.ChaffError) as ei:
        B.cluster_precond(cl, Z, B.C64)
    assert ei.value.status == B.EINVAL
    inc = W.azimuth_incidences(1)
    with pytest.raises(B.ChaffError):
        B.mlp_features(cl, inc.k_hat, inc.e_hat)
    M = torch.zeros(1 << 16, dtype=torch.uint8, device="cuda")
    with pytest.raises(B.ChaffError):
        B.solve(cl, Z, M, inc.k_hat, inc.e_hat, B.solve_opts(tol=1e-6, method=B.COCG, precond=B.PRECOND_CLUSTER))
