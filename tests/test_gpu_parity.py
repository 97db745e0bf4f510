"""GPU (gfx950) parity of every step of the hot path against the FP64 oracle.

All calls go through the C ABI (libchaff.so via the ctypes binding).  Each
test prints the case it runs before touching the GPU.

Tolerances:
  * pair sets: identical (integer work, FP64 distance test on both sides);
  * blocks: FP64 path <= 1e-11 relative Frobenius per block; FP32 path
    ||dZ_b|| <= 1e-5 ||Z_b|| + 1e-7 ||Z_ii|| per block and <= 2e-6 per block
    row (see parity_util.fp32_block_check), self blocks <= 1e-5;
  * sparse product: <= 1e-5 relative (FP32 Z and FP32 vectors vs FP64 oracle);
  * currents: <= 1e-10 (FP64 path), <= 1e-4 (FP32 + FP64 refinement);
  * RCS: <= 0.1 dB on directions within 40 dB of the peak; below that,
    absolute error <= 1e-3 of the peak.
"""
import math

import numpy as np
import pytest

from oracle import mom, solve as osolve
from paper_2410_03060_amd import workloads as W
from parity_util import (current_err, db_err, fp32_block_check, gpu_blocks_caller, gpu_pairs,
                         oracle_bistatic, oracle_mono_per_cloud, rel_block_err, say)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_03060_amd import binding
    binding.lib()
    return binding


def _to_np(t):
    return t.detach().cpu().numpy()


# ----------------------------------------------------------------------------- K-a

@pytest.mark.parametrize("name", ["c1", "c2", "c1_dense", "ragged_37", "c3_small"])
def test_pair_set_identical(B, name):
    if name == "c1":
        cloud = W.c1().cloud
    elif name == "c1_dense":
        cloud = W.c1(d_c=math.inf).cloud
    elif name == "c2":
        cloud = W.c2().cloud
    elif name == "ragged_37":
        cloud = W.random_cloud(77, 37, box_lam=3.0, d_c_lam=0.9)
    else:
        cloud = W.c3(n_main=3000, n_side=3, n_angles=1).cloud
    say(f"[pairs] {name}: N={cloud.n} clouds={cloud.n_clouds} d_c={cloud.d_c}")
    cl = B.build_cloud(cloud)
    I, J = gpu_pairs(cl)
    Io, Jo = mom.near_pairs(cloud.center, cloud.cloud_off, cloud.d_c)
    assert np.array_equal(I, Io) and np.array_equal(J, Jo)
    assert cl.nnzb == cloud.n + Io.size
    # pattern invariants: ascending columns, diagonal present, Morton permutation is a permutation
    row_ptr, col_idx, perm, diag = cl.pattern()
    assert np.array_equal(np.sort(perm), np.arange(cloud.n))
    for i in range(cloud.n):
        cols = col_idx[row_ptr[i]:row_ptr[i + 1]]
        assert np.all(np.diff(cols) > 0)
        assert col_idx[diag[i]] == i


# ----------------------------------------------------------------------------- K-b

def test_blocks_fp64_c1(B):
    wl = W.c1()
    say("[blocks] c1 complex128, d_c = 2 lambda")
    cl = B.build_cloud(wl.cloud)
    Z, P = B.fill_Z(cl, B.C128)
    rows, cols, Zg = gpu_blocks_caller(cl, Z)
    Zo = mom.cloud_blocks(wl.cloud, rows=rows, cols=cols)
    err = rel_block_err(Zg, Zo)
    say(f"  max rel block err {err.max():.3e} over {len(err)} blocks")
    assert err.max() <= 1e-11
    # block-Jacobi inverses
    row_ptr, col_idx, perm, diag = cl.pattern()
    Pg = _to_np(P)
    for i in range(cl.n):
        eye = Zg[diag[i]] @ Pg[i]
        assert np.abs(eye - np.eye(7)).max() < 1e-10


def test_blocks_fp32_c2(B):
    wl = W.c2()
    say("[blocks] c2 complex64")
    cl = B.build_cloud(wl.cloud)
    Z, P = B.fill_Z(cl, B.C64)
    rows, cols, Zg = gpu_blocks_caller(cl, Z)
    Zo = mom.cloud_blocks(wl.cloud, rows=rows, cols=cols)
    figs, ok = fp32_block_check(rows, cols, Zg, Zo)
    self_err = rel_block_err(Zg[rows == cols].astype(np.complex128), Zo[rows == cols])
    say(f"  {figs}; self blocks max rel {self_err.max():.3e}")
    assert ok
    assert self_err.max() <= 1e-5
    # stored symmetric: block (i,j) == block (j,i)^T exactly
    key = {(int(r), int(c)): k for k, (r, c) in enumerate(zip(rows, cols))}
    for k, (r, c) in enumerate(zip(rows, cols)):
        assert np.array_equal(Zg[k], Zg[key[(int(c), int(r))]].T)


def test_blocks_fp32_dense_far_pairs(B):
    """d_c = inf on a 10-wavelength cube: FP32 phases of far pairs stay accurate."""
    wl = W.c1(d_c=math.inf)
    say("[blocks] c1 dense complex64")
    cl = B.build_cloud(wl.cloud)
    Z, _ = B.fill_Z(cl, B.C64, with_pinv=False)
    rows, cols, Zg = gpu_blocks_caller(cl, Z)
    Zo = mom.cloud_blocks(wl.cloud, rows=rows, cols=cols)
    figs, ok = fp32_block_check(rows, cols, Zg, Zo)
    say(f"  {figs}")
    assert ok


def test_per_wire_radii_blocks_and_solve(B):
    """Wires of different radii: reduced distance with a^2 = (a_p^2 + a_p'^2)/2
    between wires and each wire's own radius on itself, both precisions."""
    cloud = W.random_cloud(41, 160, box_lam=3.0, d_c_lam=1.0)
    cloud.radius = np.random.default_rng(42).uniform(0.3e-4, 3e-4, cloud.n) * W.WAVELENGTH
    inc = W.azimuth_incidences(3)
    say(f"[blocks] per-wire radii: N={cloud.n}, radii {cloud.radius.min():.2e}..{cloud.radius.max():.2e} m")
    cl = B.build_cloud(cloud)
    Z64, P64 = B.fill_Z(cl, B.C128)
    rows, cols, Zg = gpu_blocks_caller(cl, Z64)
    Zo = mom.cloud_blocks(cloud, rows=rows, cols=cols)
    err = rel_block_err(Zg, Zo)
    say(f"  complex128: max rel block err {err.max():.3e} over {len(err)} blocks")
    assert err.max() <= 1e-11
    Z32, P32 = B.fill_Z(cl, B.C64)
    rows, cols, Zg32 = gpu_blocks_caller(cl, Z32)
    figs, ok = fp32_block_check(rows, cols, Zg32, Zo)
    say(f"  complex64: {figs}")
    assert ok
    Zs, _ = mom.snfc_matrix(cloud)
    xo = osolve.sparse_solve(Zs, mom.excitation(cloud, inc.k_hat, inc.e_hat))
    X, info = B.solve(cl, Z64, P64, inc.k_hat, inc.e_hat, B.solve_opts(tol=1e-12, prec=B.C128, restart=60))
    e = current_err(_to_np(X), xo)
    say(f"  complex128 solve: iters {info['iterations']} current err {e.max():.3e}")
    assert e.max() <= 1e-10
    X, info = B.solve(cl, Z32, P32, inc.k_hat, inc.e_hat, B.solve_opts(tol=1e-6))
    e = current_err(_to_np(X), xo)
    say(f"  complex64 + refinement: iters {info['iterations']} current err {e.max():.3e}")
    assert info["max_rel_residual"] <= 1e-6 and e.max() <= 1e-4


# ----------------------------------------------------------------------------- K-e, K-c

def test_excitation_c2(B):
    wl = W.c2()
    inc = W.random_incidences(np.random.default_rng(3), 5)
    say("[excitation] c2, 5 random incidences")
    cl = B.build_cloud(wl.cloud)
    U = _to_np(B.excitation(cl, inc.k_hat, inc.e_hat))
    Uo = mom.excitation(wl.cloud, inc.k_hat, inc.e_hat)
    assert np.abs(U - Uo).max() <= 1e-13 * np.abs(Uo).max()


@pytest.mark.parametrize("s,variant", [(1, 0), (1, 1), (3, 1), (8, 1), (8, 2), (64, 1), (70, 1),
                                       (1, 5), (3, 5), (8, 5), (16, 5), (70, 5),
                                       (1, 6), (3, 6), (8, 6), (16, 6), (33, 6), (70, 6),
                                       (2, 7), (5, 7), (12, 6), (16, 7), (24, 7), (32, 7), (64, 7)])
def test_spmm_c2(B, s, variant):
    import torch
    wl = W.c2()
    say(f"[spmm] c2 complex64 s={s} variant={variant}")
    cl = B.build_cloud(wl.cloud)
    Z, _ = B.fill_Z(cl, B.C64, with_pinv=False)
    rng = np.random.default_rng(11)
    Xc = rng.standard_normal((cl.n * 7, s)) + 1j * rng.standard_normal((cl.n * 7, s))   # caller order
    row_ptr, col_idx, perm, diag = cl.pattern()
    rows_int = (perm[:, None] * 7 + np.arange(7)[None, :]).ravel()   # internal row -> caller row
    Xi = Xc[rows_int]
    Y = _to_np(B.spmm(cl, Z, torch.as_tensor(Xi.astype(np.complex64), device="cuda"), B.C64, variant))
    Zs, _ = mom.snfc_matrix(wl.cloud)
    Yo = (Zs @ Xc)[rows_int]
    err = np.linalg.norm(Y - Yo) / np.linalg.norm(Yo)
    say(f"  rel err {err:.3e}")
    assert err <= 1e-5


# ----------------------------------------------------------------------------- solve + rcs

_METHODS = {"gmres": "GMRES", "cocg": "COCG", "gcr": "GCR"}


def _method_opts(B, method):
    """Method constant and its cycle settings: restarted methods 30 steps to a
    1e-4 reduction per refinement cycle, COCG up to 500 steps to 1e-2."""
    meth = getattr(B, _METHODS[method])
    restarted = meth in (B.GMRES, B.GCR)
    return dict(method=meth, restart=30 if restarted else 500, inner_tol=1e-4 if restarted else 1e-2)


@pytest.mark.parametrize("method", ["gmres", "gcr"])
@pytest.mark.parametrize("dense", [False, True])
def test_c1_complex128_solve_and_bistatic_rcs(B, dense, method):
    wl = W.c1(d_c=math.inf if dense else 2.0)
    say(f"[solve] c1 complex128 dense={dense} {method}")
    cl = B.build_cloud(wl.cloud)
    Z, P = B.fill_Z(cl, B.C128)
    X, info = B.solve(cl, Z, P, wl.inc.k_hat, wl.inc.e_hat,
                      B.solve_opts(tol=1e-12, restart=60, max_cycles=20, prec=B.C128,
                                   method=getattr(B, _METHODS[method])))
    say(f"  cycles {info['cycles']} iters {info['iterations']} res {info['max_rel_residual']:.2e}")
    u = mom.excitation(wl.cloud, wl.inc.k_hat, wl.inc.e_hat)
    if dense:
        xo = osolve.dense_solve(mom.dense_Z(wl.cloud), u)
    else:
        Zs, _ = mom.snfc_matrix(wl.cloud)
        xo = osolve.sparse_solve(Zs, u)
    e = current_err(_to_np(X), xo)
    say(f"  current err {e.max():.3e}")
    assert e.max() <= 1e-10
    T, Pp, rh, th, ph = W.bistatic_grid(1.0)
    dirs = np.concatenate([rh, rh])
    pols = np.concatenate([th, ph])
    sig = _to_np(B.rcs(cl, X, dirs, pols, monostatic=False))[0, 0]
    so_t, so_p = oracle_bistatic(wl.cloud, xo, rh, th, ph)
    so = np.concatenate([so_t, so_p])
    e_db, e_lo = db_err(sig, so)
    say(f"  bistatic dB err {e_db:.2e}, below-floor {e_lo:.2e}")
    assert e_db <= 1e-6 and e_lo <= 1e-8
    # monostatic through the same path
    sm = _to_np(B.rcs(cl, X, -wl.inc.k_hat, wl.inc.e_hat, monostatic=True))[0]
    smo = mom.monostatic_rcs(wl.cloud, xo, wl.inc.k_hat, wl.inc.e_hat)
    assert abs(sm[0] - smo[0]) <= 1e-9 * smo[0]


@pytest.mark.parametrize("method", ["gmres", "cocg", "gcr"])
def test_c2_fp32_refined_solve(B, method):
    wl = W.c2()
    say(f"[solve] c2 complex64 + FP64 refinement to 1e-6, {method}")
    cl = B.build_cloud(wl.cloud)
    Z, P = B.fill_Z(cl, B.C64)
    X, info = B.solve(cl, Z, P, wl.inc.k_hat, wl.inc.e_hat, B.solve_opts(tol=1e-6, **_method_opts(B, method)))
    say(f"  cycles {info['cycles']} iters {info['iterations']} res {info['max_rel_residual']:.2e}")
    assert info["max_rel_residual"] <= 1e-6
    Zs, _ = mom.snfc_matrix(wl.cloud)
    u = mom.excitation(wl.cloud, wl.inc.k_hat, wl.inc.e_hat)
    xo = osolve.sparse_solve(Zs, u)
    e = current_err(_to_np(X), xo)
    say(f"  current err {e.max():.3e}")
    assert e.max() <= 1e-4
    sm = _to_np(B.rcs(cl, X, -wl.inc.k_hat, wl.inc.e_hat, monostatic=True))[0]
    smo = mom.monostatic_rcs(wl.cloud, xo, wl.inc.k_hat, wl.inc.e_hat)
    e_db, _ = db_err(sm, smo)
    say(f"  monostatic dB err {e_db:.2e}")
    assert e_db <= 0.1


@pytest.mark.parametrize("method", ["gmres", "cocg", "gcr"])
def test_multicloud_multirhs_one_launch(B, method):
    """Three uneven clouds (one empty) x 6 azimuth RHS in one build/fill/solve/rcs."""
    lam = W.WAVELENGTH
    parts = [W.random_cloud(5, 400, box_lam=12.0, d_c_lam=2.0),
             W.random_cloud(6, 0, box_lam=5.0, d_c_lam=2.0) if False else None,
             W.random_cloud(7, 150, box_lam=6.0, d_c_lam=2.0),
             W.random_cloud(8, 233, box_lam=9.0, d_c_lam=2.0)]
    parts = [p for p in parts if p is not None]
    # an empty cloud in the middle
    empty = W.single_cloud(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0), lam, 2.0 * lam)
    cloud = W.concat_clouds([parts[0], empty, parts[1], parts[2]])
    inc = W.azimuth_incidences(6)
    say(f"[solve] multi-cloud N={cloud.n} clouds={cloud.n_clouds} R=6")
    cl = B.build_cloud(cloud)
    Z, P = B.fill_Z(cl, B.C64)
    X, info = B.solve(cl, Z, P, inc.k_hat, inc.e_hat, B.solve_opts(tol=1e-6, **_method_opts(B, method)))
    say(f"  cycles {info['cycles']} iters {info['iterations']} res {info['max_rel_residual']:.2e}")
    assert info["max_rel_residual"] <= 1e-6
    Zs, _ = mom.snfc_matrix(cloud)
    u = mom.excitation(cloud, inc.k_hat, inc.e_hat)
    xo = osolve.sparse_solve(Zs, u)
    e = current_err(_to_np(X), xo)
    say(f"  current err {e.max():.3e}")
    assert e.max() <= 1e-4
    sig = _to_np(B.rcs(cl, X, -inc.k_hat, inc.e_hat, monostatic=True))
    so = oracle_mono_per_cloud(cloud, xo, inc.k_hat, inc.e_hat)
    assert np.all(sig[1] == 0.0)
    for c in (0, 2, 3):
        e_db, _ = db_err(sig[c], so[c])
        assert e_db <= 0.1


def test_gcr_and_gmres_minimise_over_the_same_space(B):
    """Right-preconditioned GCR(m) and GMRES(m) minimise the residual over the
    same Krylov space, so in FP64 they need the same number of steps and reach
    the same currents (four RHS, one cycle each)."""
    wl = W.c2(n=600)
    inc = W.azimuth_incidences(4)
    say(f"[solve] GCR against GMRES, N={wl.cloud.n} R=4, complex128")
    cl = B.build_cloud(wl.cloud)
    Z, P = B.fill_Z(cl, B.C128)
    out = {}
    for name in ("GMRES", "GCR"):
        X, info = B.solve(cl, Z, P, inc.k_hat, inc.e_hat,
                          B.solve_opts(tol=1e-10, restart=120, max_cycles=4, prec=B.C128, method=getattr(B, name)))
        out[name] = (_to_np(X), info)
        say(f"  {name}: cycles {info['cycles']} iters {info['iterations']} res {info['max_rel_residual']:.2e}")
    assert abs(out["GCR"][1]["iterations"] - out["GMRES"][1]["iterations"]) <= 2
    assert current_err(out["GCR"][0], out["GMRES"][0]).max() <= 1e-8


def test_degenerate_single_wire_and_no_pairs(B):
    lam = W.WAVELENGTH
    one = W.single_cloud([[0.0, 0.0, 0.0]], [[0.0, 0.0, 1.0]], [0.48 * lam], lam, 2 * lam)
    say("[edge] single wire")
    cl = B.build_cloud(one)
    assert cl.nnzb == 1 and cl.n_pairs == 0
    Z, P = B.fill_Z(cl, B.C64)
    kh = np.array([[1.0, 0.0, 0.0]])
    e = np.array([[0.0, 0.0, 1.0]])
    X, info = B.solve(cl, Z, P, kh, e, B.solve_opts(tol=1e-7))
    s = _to_np(B.rcs(cl, X, -kh, e, monostatic=True))[0, 0] / lam ** 2
    so = mom.monostatic_rcs(one, osolve.dense_solve(mom.dense_Z(one), mom.excitation(one, kh, e)), kh, e)[0]
    assert abs(10 * math.log10(s * lam ** 2 / so)) < 1e-3
    # tiny d_c: no pairs at all, block diagonal system
    far = W.random_cloud(3, 50, box_lam=20.0, d_c_lam=1e-3)
    say("[edge] no pairs")
    cl = B.build_cloud(far)
    assert cl.nnzb == 50 and cl.n_pairs == 0


def test_determinism_bitwise(B):
    wl = W.c2()
    say("[determinism] c2 twice")
    outs = []
    for _ in range(2):
        cl = B.build_cloud(wl.cloud)
        Z, P = B.fill_Z(cl, B.C64)
        X, _ = B.solve(cl, Z, P, wl.inc.k_hat, wl.inc.e_hat, B.solve_opts(tol=1e-6))
        outs.append((cl.pattern()[1], _to_np(Z), _to_np(X)))
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("method", ["cocg", "gmres"])
def test_non_finite_solution_is_reported_as_breakdown(B, method):
    """A NaN entry in Z makes the FP64 residual of the systems that touch it
    non-finite: the solve ends with CHAFF_ENOCONV and a relative residual of
    +inf, never with convergence."""
    import torch
    cloud = W.random_cloud(43, 60, box_lam=2.0, d_c_lam=1.0)
    inc = W.azimuth_incidences(3)
    say(f"[breakdown] {method}: NaN entry in one block, 60 wires, 3 RHS")
    cl = B.build_cloud(cloud)
    Z, P = B.fill_Z(cl, B.C64)
    Z[0, 0, 0] = complex(float("nan"), 0.0)
    torch.cuda.synchronize()
    opts = B.solve_opts(tol=1e-6, method=B.COCG if method == "cocg" else B.GMRES, restart=50, max_cycles=3)
    with pytest.raises(B.ChaffError) as err:
        B.solve(cl, Z, P, inc.k_hat, inc.e_hat, opts)
    assert err.value.status == B.ENOCONV and "breakdown" in str(err.value)
    _, info = B.solve(cl, Z, P, inc.k_hat, inc.e_hat, opts, raise_on_noconv=False)
    assert math.isinf(info["max_rel_residual"])
    B.destroy(cl)


def test_tangent_validation_on_device(B):
    bad = W.random_cloud(9, 20, box_lam=3.0, d_c_lam=1.0)
    bad.tangent[3] *= 1.01
    say("[edge] non-unit tangent rejected")
    with pytest.raises(B.ChaffError) as ei:
        B.build_cloud(bad)
    assert ei.value.status == B.EINVAL


def test_autotune_records_and_uses_the_fastest_variant(B):
    import torch
    wl = W.c2()
    say("[autotune] c2, s=8")
    cl = B.build_cloud(wl.cloud)
    Z, _ = B.fill_Z(cl, B.C64, with_pinv=False)
    best, ms = B.autotune(cl, Z, 8, B.C64)
    assert 0 <= best <= 7 and ms > 0
    table = B.tune_report()
    ent = [e for e in table if e["n"] == cl.n and e["nnzb"] == cl.nnzb and e["s"] == 8 and e["prec"] == B.C64]
    assert len(ent) == 1 and ent[0]["best"] == best
    assert min(ent[0]["ms"]) == pytest.approx(ent[0]["ms"][best])
    X = torch.randn(cl.n * 7, 8, dtype=torch.complex64, device="cuda")
    y_tuned = _to_np(B.spmm(cl, Z, X, B.C64, -1))
    y_best = _to_np(B.spmm(cl, Z, X, B.C64, best))
    assert np.array_equal(y_tuned, y_best)
    # a solve on the tuned table still meets the bar
    X2, info = B.solve(cl, *B.fill_Z(cl, B.C64), wl.inc.k_hat, wl.inc.e_hat, B.solve_opts(tol=1e-6))
    assert info["max_rel_residual"] <= 1e-6


@pytest.mark.parametrize("n_clouds", [1, 2])
def test_cocg_column_compaction(B, n_clouds):
    """Incidences that converge at different speeds: once few columns are left
    above their checkpoint the COCG cycle packs them into a narrower block;
    every column must still reach the oracle's solution."""
    parts = [W.random_cloud(12, 1500, box_lam=10.0, d_c_lam=1.5)]
    if n_clouds == 2:
        parts.append(W.random_cloud(14, 600, box_lam=6.0, d_c_lam=1.5))
    cloud = W.concat_clouds(parts) if n_clouds > 1 else parts[0]
    inc = W.random_incidences(np.random.default_rng(13), 24)
    say(f"[solve] COCG column compaction: N={cloud.n} clouds={n_clouds} R=24")
    cl = B.build_cloud(cloud)
    Z, P = B.fill_Z(cl, B.C64)
    B.profile_enable(True)
    X, info = B.solve(cl, Z, P, inc.k_hat, inc.e_hat,
                      B.solve_opts(tol=1e-6, method=B.COCG, restart=500, inner_tol=1e-3))
    B.profile_enable(False)
    prof = B.profile_read()
    say(f"  cycles {info['cycles']} iters {info['iterations']} res {info['max_rel_residual']:.2e} "
        f"compactions {prof.get('cocg_compact', {}).get('launches', 0)}")
    assert "cocg_compact" in prof
    assert np.all(info["rel_res"] <= 1e-6)
    Zs, _ = mom.snfc_matrix(cloud)
    u = mom.excitation(cloud, inc.k_hat, inc.e_hat)
    xo = osolve.sparse_solve(Zs, u)
    e = current_err(_to_np(X), xo)
    say(f"  current err {e.max():.3e}")
    assert e.max() <= 1e-4


@pytest.mark.parametrize("R", [40, 64, 70])
def test_cocg_wide_rhs(B, R):
    """More than 32 right-hand sides: the COCG product runs 64-column tiles
    (ragged last tile for 40 and 70)."""
    cloud = W.random_cloud(31, 900, box_lam=8.0, d_c_lam=1.5)
    inc = W.random_incidences(np.random.default_rng(32), R)
    say(f"[solve] COCG R={R} N={cloud.n}")
    cl = B.build_cloud(cloud)
    Z, P = B.fill_Z(cl, B.C64)
    X, info = B.solve(cl, Z, P, inc.k_hat, inc.e_hat,
                      B.solve_opts(tol=1e-6, method=B.COCG, restart=500, inner_tol=1e-3))
    say(f"  cycles {info['cycles']} iters {info['iterations']} res {info['max_rel_residual']:.2e}")
    assert np.all(info["rel_res"] <= 1e-6)
    Zs, _ = mom.snfc_matrix(cloud)
    u = mom.excitation(cloud, inc.k_hat, inc.e_hat)
    xo = osolve.sparse_solve(Zs, u)
    e = current_err(_to_np(X), xo)
    say(f"  current err {e.max():.3e}")
    assert e.max() <= 1e-4
