"""Pins for two readings of the thin-wire kernel that the other pins leave open.

1. Different radii (reading of Sec. II-A's thin-wire approximation): between
   wires of radii a_p and a_p' the reduced distance is
   R = sqrt(|r - r'|^2 + (a_p^2 + a_p'^2)/2).  The oracle's mutual block is
   checked against brute-force adaptive quadrature of the defining double
   integral (eqs. 5-8 with rooftop bases), written out here from the basis
   definitions alone; the check is sensitive to the mixing rule (a plausible
   other rule moves the block far beyond the tolerance), and the block pair
   computed from both sides is transposed exactly (Galerkin symmetry).

2. FP32 block accuracy: a faithful complex-FP32 evaluation of the same
   segment-pair quadrature (geometry formed in FP64 and rounded once, samples
   and sums in FP32, phase in revolutions), written in this test, reaches a
   relative error above 1e-5 on blocks whose value nearly cancels: their
   far-field transverse factor (t . t') - (R.t)(R.t') is small.  The error of
   those blocks measured against their block row stays at the FP32 rounding
   level.  This is why the FP32 parity bar is row-aware: ||dZ_b|| <=
   1e-5 ||Z_b|| + 1e-7 ||Z_ii|| per block and <= 2e-6 per block row.
"""
import math

import numpy as np
import pytest

from oracle import mom
from paper_2410_03060_amd import workloads as W

LAM = W.WAVELENGTH
K = 2.0 * math.pi / LAM


# --------------------------------------------------------------------------- different radii

def _two_thick_wires(a0, a1):
    """Two skew wires passing 0.02 lambda apart, radii a0 and a1 (thick, so that
    the reduced distance is dominated by the radii near the crossing)."""
    t = np.array([[1.0, 0.0, 0.0], [0.6, 0.8, 0.0]])
    c = np.array([[0.0, 0.0, 0.0], [0.03 * LAM, -0.01 * LAM, 0.02 * LAM]])
    L = np.array([0.5, 0.45]) * LAM
    return W.single_cloud(c, t, L, LAM, math.inf, np.array([a0, a1]))


def _brute_entry(cl, m, n, a2):
    """Z_mn between wire 0 (test basis m) and wire 1 (source basis n) by adaptive
    quadrature of int int [(t.t') L_m L_n - (1/k^2) L_m' L_n'] G(R) ds' ds,
    G = exp(-jkR)/(4 pi R), R^2 = |r - r'|^2 + a2, rooftops of peak 1."""
    from scipy.integrate import dblquad
    c, t, L = cl.center, cl.tangent, cl.length
    n_seg = 8
    D = L / n_seg
    s_m = -0.5 * L[0] + (m + 1) * D[0]
    s_n = -0.5 * L[1] + (n + 1) * D[1]
    tt = float(t[0] @ t[1])

    def lam(s, sv, d):
        return 1.0 - abs(s - sv) / d

    def dlam(s, sv, d):
        return (1.0 if s < sv else -1.0) / d

    def f(sp, s, part):
        r = c[0] + s * t[0] - c[1] - sp * t[1]
        R = math.sqrt(float(r @ r) + a2)
        g = np.exp(-1j * K * R) / (4 * math.pi * R)
        v = (tt * lam(s, s_m, D[0]) * lam(sp, s_n, D[1])
             - dlam(s, s_m, D[0]) * dlam(sp, s_n, D[1]) / K ** 2) * g
        return v.real if part == 0 else v.imag

    tot = 0.0 + 0.0j
    for s0, s1 in ((s_m - D[0], s_m), (s_m, s_m + D[0])):
        for p0, p1 in ((s_n - D[1], s_n), (s_n, s_n + D[1])):
            re = dblquad(lambda sp, s: f(sp, s, 0), s0, s1, p0, p1, epsabs=0, epsrel=1e-11)[0]
            im = dblquad(lambda sp, s: f(sp, s, 1), s0, s1, p0, p1, epsabs=0, epsrel=1e-11)[0]
            tot += re + 1j * im
    return tot


def test_mixed_radius_block_against_brute_force_quadrature():
    a0, a1 = 0.01 * LAM, 0.03 * LAM
    cl = _two_thick_wires(a0, a1)
    # converged tensor Gauss rule of the oracle (16 nodes per segment; the nearest
    # singularity sits one reduced radius off the segment, so this is exact to ~1e-12)
    Zo = mom.mutual_blocks(cl.center, cl.tangent, cl.length, cl.radius, [0], [1], K, q=16)[0]
    a2 = 0.5 * (a0 * a0 + a1 * a1)
    scale = np.abs(Zo).max()
    for m, n in ((0, 0), (3, 3), (3, 4), (6, 1)):
        zb = _brute_entry(cl, m, n, a2)
        assert abs(zb - Zo[m, n]) <= 1e-8 * scale, (m, n, zb, Zo[m, n])
    # sensitivity: the arithmetic mean of the radii (another plausible rule) or
    # the test wire's own radius gives blocks far outside that tolerance
    for a_other in (0.5 * (a0 + a1), a0):
        cl2 = _two_thick_wires(a_other, a_other)
        Z2 = mom.mutual_blocks(cl2.center, cl2.tangent, cl2.length, cl2.radius, [0], [1], K, q=16)[0]
        assert np.abs(Z2 - Zo).max() > 1e-3 * scale


def test_mixed_radius_galerkin_symmetry_and_equal_radius_limit():
    cl = _two_thick_wires(0.01 * LAM, 0.03 * LAM)
    Z01 = mom.mutual_blocks(cl.center, cl.tangent, cl.length, cl.radius, [0], [1], K)[0]
    Z10 = mom.mutual_blocks(cl.center, cl.tangent, cl.length, cl.radius, [1], [0], K)[0]
    assert np.abs(Z01 - Z10.T).max() <= 1e-13 * np.abs(Z01).max()
    # equal radii: the rule is the common radius (the thin-wire kernel of every other pin)
    a = 0.02 * LAM
    cl_eq = _two_thick_wires(a, a)
    a_eq = math.sqrt(0.5 * (a * a + a * a))
    assert a_eq == pytest.approx(a, rel=1e-15)


def test_mixed_radius_cloud_matrix_is_symmetric():
    """A cloud with per-wire radii: the assembled S-NFC matrix is complex symmetric."""
    cl = W.random_cloud(5, 12, box_lam=1.5, d_c_lam=0.8)
    cl.radius = np.random.default_rng(6).uniform(0.5e-4, 3e-4, cl.n) * LAM
    Zs, _ = mom.snfc_matrix(cl)
    Zd = Zs.toarray()
    assert np.abs(Zd - Zd.T).max() <= 1e-13 * np.abs(Zd).max()


# --------------------------------------------------------------------------- FP32 block accuracy

def _mutual_fp32(cloud, I, J, q=4, n_seg=8):
    """Mutual blocks evaluated in complex FP32 (written here, not in the oracle).

    Per segment pair (alpha, beta): the offset b = s0_i t_i - (c_j - c_i) - s0_j t_j
    and the segment vectors D t are formed in FP64 and rounded once to FP32;
    every Green sample, weight product and moment sum is FP32; the phase
    k R is taken in revolutions R/lambda and reduced to [0, 1) before the
    trigonometric functions.  Assembly into rooftop blocks also in FP32.
    """
    f32 = np.float32
    xi, g = mom.gauss01(q)
    xq, wq = xi.astype(f32), g.astype(f32)
    c, t, L, a = cloud.center, cloud.tangent, cloud.length, cloud.radius
    I, J = np.asarray(I), np.asarray(J)
    Di, Dj = L[I] / n_seg, L[J] / n_seg
    al = np.arange(n_seg)
    s0i = -0.5 * L[I][:, None] + al[None, :] * Di[:, None]            # [B,S] FP64
    s0j = -0.5 * L[J][:, None] + al[None, :] * Dj[:, None]
    sep = c[J] - c[I]
    b = (s0i[:, :, None, None] * t[I][:, None, None, :] - sep[:, None, None, :]
         - s0j[:, None, :, None] * t[J][:, None, None, :]).astype(f32)  # [B,S,S,3]
    ui = (Di[:, None] * t[I]).astype(f32)
    uj = (Dj[:, None] * t[J]).astype(f32)
    a2 = (0.5 * (a[I] ** 2 + a[J] ** 2)).astype(f32)
    inv_lam = f32(1.0 / cloud.wavelength)
    # d[B,S,S,k,l,3] = (b - x_l uj) + x_k ui
    p = b[:, :, :, None, :] - xq[None, None, None, :, None] * uj[:, None, None, None, :]
    d = p[:, :, :, None, :, :] + xq[None, None, None, :, None, None] * ui[:, None, None, None, None, :]
    r2 = np.sum(d * d, axis=-1, dtype=f32) + a2[:, None, None, None, None]
    ir = (f32(1) / np.sqrt(r2)).astype(f32)
    rev = (r2 * ir * inv_lam).astype(f32)
    fr = (rev - np.floor(rev)).astype(f32)
    ang = (f32(2 * math.pi) * fr).astype(f32)
    gre = (np.cos(ang) * ir).astype(f32)
    gim = (-np.sin(ang) * ir).astype(f32)
    G = (gre + 1j * gim).astype(np.complex64)                         # [B,S,S,k,l]
    phi = np.stack([xq, f32(1) - xq]).astype(f32)                     # phi_+, phi_-
    wa = (wq[None, :] * phi).astype(f32)                              # [2,Q]
    A = np.einsum("ak,bl,nsukl->nabsu", wa, wa, G).astype(np.complex64)
    sc = (Di * Dj / (4.0 * math.pi)).astype(f32)
    A = (A * sc[:, None, None, None, None]).astype(np.complex64)
    Bs = A.sum(axis=(1, 2)).astype(np.complex64)
    tt = np.sum(t[I] * t[J], axis=-1).astype(f32)[:, None, None]
    sz = (1.0 / (K * K * Di * Dj)).astype(f32)[:, None, None]
    nb = n_seg - 1
    Z = np.zeros((len(I), nb, nb), dtype=np.complex64)
    for ia, sa, da in ((0, 1.0, 0), (1, -1.0, 1)):
        for ib, sb, db in ((0, 1.0, 0), (1, -1.0, 1)):
            Z += tt * A[:, ia, ib, da:da + nb, db:db + nb]
            Z -= f32(sa * sb) * sz * Bs[:, da:da + nb, db:db + nb]
    return Z


def test_fp32_evaluation_error_level_on_c2_blocks():
    cloud = W.c2().cloud
    I, J = mom.near_pairs(cloud.center, cloud.cloud_off, cloud.d_c)
    up = I < J
    I, J = I[up], J[up]
    Zo = mom.mutual_blocks(cloud.center, cloud.tangent, cloud.length, cloud.radius, I, J, K)
    Z32 = _mutual_fp32(cloud, I, J).astype(np.complex128)
    err = np.linalg.norm((Z32 - Zo).reshape(len(I), -1), axis=1)
    nrm = np.linalg.norm(Zo.reshape(len(I), -1), axis=1)
    rel = err / nrm
    # transverse (far-field) factor of each pair
    sep = cloud.center[J] - cloud.center[I]
    Rh = sep / np.linalg.norm(sep, axis=1, keepdims=True)
    ti, tj = cloud.tangent[I], cloud.tangent[J]
    tf = np.abs(np.sum(ti * tj, 1) - np.sum(Rh * ti, 1) * np.sum(Rh * tj, 1))
    # the self blocks of the rows, for the row-aware bar
    Zii = mom.self_blocks(cloud.length[I], cloud.radius[I], K)
    nd = np.linalg.norm(Zii.reshape(len(I), -1), axis=1)
    high = rel > 1e-5
    print(f"\nFP32 evaluation on {len(I)} c2 pairs: rel err median {np.median(rel):.2e}, max {rel.max():.2e}; "
          f"{int(high.sum())} above 1e-5 with transverse factor <= {tf[high].max() if high.any() else 0:.3f} "
          f"(median over all pairs {np.median(tf):.3f}); max err / ||Z_ii|| {np.max(err / nd):.2e}")
    # a faithful FP32 evaluation does not meet a flat 1e-5 per-block bar (the
    # complex64 fill measured 6.1e-5 on these blocks) ...
    assert rel.max() > 3e-5
    # ... because its absolute error is ordinary FP32 rounding of the samples,
    # nearly the same on every block, so the relative error grows as the
    # block's norm shrinks ...
    assert err.max() <= 4.0 * np.median(err)
    assert np.corrcoef(np.log(rel), np.log(nrm))[0, 1] < -0.8
    assert np.all(nrm[high] < np.median(nrm))
    # ... and the worst blocks are those that nearly cancel (small transverse factor)
    worst = rel > 3e-5
    assert np.all(tf[worst] < 0.2) and np.median(tf[worst]) < 0.06 and np.median(tf) > 0.25
    # the row-aware bar of the FP32 parity tests holds with margin
    assert np.all(err <= 1e-5 * nrm + 1e-7 * nd)
    assert np.max(err / nd) <= 2e-7
