"""Thin-wire EFIE Galerkin MoM in complex128 (oracle; test infrastructure only).

Formulation (Sec. II-A of the paper, time convention exp(+j w t)):

* each wire p (centre c_p, unit tangent t_p, length L_p, radius a_p) is cut
  into ``n_seg`` equal segments of length D_p = L_p/n_seg; one rooftop
  (triangle) basis sits on every interior vertex, so a wire carries
  n_seg - 1 unknowns (eq. 2 and its footnote).  Global index n = p*(n_seg-1)+q.
* Z = Z1 + Z2 with (eqs. 5-8)
      Z1_mn =           int int (t_m . t_n) L_m(r) L_n(r') G dr' dr
      Z2_mn = -(1/k^2)  int int (dL_m/ds)(dL_n/ds') G dr' dr
  and G = exp(-j k R)/(4 pi R).
* thin-wire (reduced) kernel: R = sqrt(|r - r'|^2 + a^2) with r, r' on the
  wire axes; for two wires of different radii a^2 = (a_p^2 + a_p'^2)/2, which
  keeps Z symmetric.
* quadrature: tensor Gauss-Legendre per segment pair, ``q_mutual`` nodes for
  different wires, ``q_self`` nodes on the same wire; on the same wire for
  segment offsets |alpha - beta| <= 1 the static part 1/(4 pi R) is integrated
  in closed form and only (exp(-jkR) - 1)/(4 pi R) is sampled (the "analytic
  singularity extraction" of Sec. II-A).
* excitation (eq. 4): u_m = int L_m (t_m . e) exp(-j k k_hat . r) ds, evaluated
  exactly (triangle Fourier transform); the paper's v = -(j/(w mu0)) u, and
  the physical current is -(j/(w mu0)) x where Z x = u.
* S-NFC (eq. 9): block (p, p') is kept iff the centroid distance is <= d_c,
  tested in FP64 as ((dx*dx + dy*dy) + dz*dz) <= d_c*d_c without fused
  multiply-add; the diagonal blocks are always kept.
* RCS: with w_n(r_hat, e) = int L_n (t_n . e) exp(+j k r_hat . r) ds and
  S = w^T x, sigma = |S|^2/(4 pi) [m^2] for a unit-amplitude incident wave
  (mu0, eta0 and c0 cancel; only the wavelength enters).
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import polynomial as npoly

FOUR_PI = 4.0 * math.pi


def gauss01(q: int):
    """Gauss-Legendre nodes and weights on [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(q)
    return 0.5 * (x + 1.0), 0.5 * w


def n_unknowns_per_wire(n_seg: int) -> int:
    return n_seg - 1


# ----------------------------------------------------------------------------
# closed-form static self integrals (same wire, collinear segments)
# ----------------------------------------------------------------------------

def _line_weights():
    """Monomial weights integrated along the lines xi - xi' = t (Jacobian 1).

    m_mn(t) = int over {xi - xi' = t} of xi^m xi'^n, for t in [0,1] and [-1,0].
    Returned as numpy polynomial coefficient arrays in t: {(m,n): (pos, neg)}.
    """
    P = npoly.Polynomial
    t = P([0.0, 1.0])
    pos = {(0, 0): 1 - t, (1, 0): (1 - t * t) / 2, (0, 1): (1 - t) ** 2 / 2,
           (1, 1): (1 - t) ** 2 * (2 + t) / 6}
    neg = {(0, 0): 1 + t, (1, 0): (1 + t) ** 2 / 2, (0, 1): (1 - t * t) / 2,
           (1, 1): (1 + t) ** 2 * (2 - t) / 6}
    return pos, neg


def _ab_weights():
    """Line weights of phi_a(xi) phi_b(xi') with phi_+ = xi, phi_- = 1 - xi.

    Index 0 is '+' (rising half of a rooftop), 1 is '-' (falling half).
    """
    pos, neg = _line_weights()
    out = {}
    for side, m in (("pos", pos), ("neg", neg)):
        out[(0, 0, side)] = m[(1, 1)]
        out[(0, 1, side)] = m[(1, 0)] - m[(1, 1)]
        out[(1, 0, side)] = m[(0, 1)] - m[(1, 1)]
        out[(1, 1, side)] = m[(0, 0)] - m[(1, 0)] - m[(0, 1)] + m[(1, 1)]
    return out


def _antiderivs(v: float, b: float) -> np.ndarray:
    """I_n(v) with d/dv I_n = v^n / sqrt(v^2 + b^2), n = 0..3."""
    s = math.sqrt(v * v + b * b)
    ash = math.asinh(v / b)
    return np.array([ash, s, 0.5 * (v * s - b * b * ash),
                     (v * v + b * b) * s / 3.0 - b * b * s])


def static_self_integral(d: int, b: float) -> np.ndarray:
    """K[a,b] = int_0^1 int_0^1 phi_a(xi) phi_b(xi') / sqrt((d + xi - xi')^2 + b^2).

    ``d`` is the segment offset alpha - beta, ``b`` = radius / segment length.
    Exact: reduce to one variable t = xi - xi' with the polynomial line
    weights, substitute v = d + t and integrate v^n/sqrt(v^2+b^2) in closed
    form.
    """
    W = _ab_weights()
    K = np.zeros((2, 2))
    shift = npoly.Polynomial([-float(d), 1.0])  # t = v - d
    for a in range(2):
        for bb in range(2):
            tot = 0.0
            for side, (t0, t1) in (("pos", (0.0, 1.0)), ("neg", (-1.0, 0.0))):
                Pv = W[(a, bb, side)](shift)  # polynomial in v
                coef = np.zeros(4)
                coef[:len(Pv.coef)] = Pv.coef
                Ihi = _antiderivs(d + t1, b)
                Ilo = _antiderivs(d + t0, b)
                tot += float(np.dot(coef, Ihi - Ilo))
            K[a, bb] = tot
    return K


# ----------------------------------------------------------------------------
# impedance blocks
# ----------------------------------------------------------------------------

def _assemble(A: np.ndarray, Bsum: np.ndarray, tt, Di, Dj, k: float) -> np.ndarray:
    """Rooftop assembly of segment-pair integrals into basis blocks.

    A[..., a, b, alpha, beta] = D_i D_j int int phi_a phi_b G (segment pair),
    Bsum = sum_ab A.  Basis q (0-based) sits on vertex q+1: rising ('+',
    slope +1/D) on segment q and falling ('-', slope -1/D) on segment q+1.
    """
    S = A.shape[-1]
    nb = S - 1
    Z = np.zeros(A.shape[:-4] + (nb, nb), dtype=np.complex128)
    tt = np.asarray(tt)[..., None, None]
    scal = (1.0 / (k * k)) / (np.asarray(Di) * np.asarray(Dj))
    scal = np.asarray(scal)[..., None, None]
    for a, sa, da in ((0, 1.0, 0), (1, -1.0, 1)):
        for b, sb, db in ((0, 1.0, 0), (1, -1.0, 1)):
            Z += tt * A[..., a, b, da:da + nb, db:db + nb]
            Z -= scal * (sa * sb) * Bsum[..., da:da + nb, db:db + nb]
    return Z


def _axis_offsets(L, n_seg, xi):
    """s[..., alpha, k] = -L/2 + (alpha + xi_k) * L/n_seg."""
    L = np.asarray(L, dtype=np.float64)
    D = L / n_seg
    alpha = np.arange(n_seg, dtype=np.float64)
    return (-0.5 * L)[..., None, None] + (alpha[:, None] + xi[None, :]) * D[..., None, None]


def mutual_blocks(center, tangent, length, radius, I, J, k: float,
                  n_seg: int = 8, q: int = 4) -> np.ndarray:
    """Z blocks between wires I[b] (test) and J[b] (source), I != J. -> [B, nb, nb]."""
    I = np.asarray(I)
    J = np.asarray(J)
    xi, g = gauss01(q)
    Di = length[I] / n_seg
    Dj = length[J] / n_seg
    si = _axis_offsets(length[I], n_seg, xi)            # [B,S,Q]
    sj = _axis_offsets(length[J], n_seg, xi)
    ti = tangent[I]
    tj = tangent[J]
    sep = center[J] - center[I]                          # FP64 centroid separation
    # r - r' as seen from wire I: (s_i t_i) - (sep + s_j t_j)
    diff = (si[:, :, :, None, None, None] * ti[:, None, None, None, None, :]
            - sj[:, None, None, :, :, None] * tj[:, None, None, None, None, :]
            - sep[:, None, None, None, None, :])         # [B,S,Q,S,Q,3]
    a2 = 0.5 * (radius[I] ** 2 + radius[J] ** 2)
    R = np.sqrt(np.sum(diff * diff, axis=-1) + a2[:, None, None, None, None])
    G = np.exp(-1j * k * R) / (FOUR_PI * R)
    phi = np.stack([xi, 1.0 - xi])                       # [2,Q]: phi_+, phi_-
    wa = g[None, :] * phi                                # [2,Q]
    A = np.einsum("ak,bl,nskul->nabsu", wa, wa, G)       # [B,2,2,S,S]
    A *= (Di * Dj)[:, None, None, None, None]
    Bsum = A.sum(axis=(1, 2))
    tt = np.sum(ti * tj, axis=-1)
    return _assemble(A, Bsum, tt, Di, Dj, k)


def self_blocks(length, radius, k: float, n_seg: int = 8, q: int = 8) -> np.ndarray:
    """Self blocks of wires with the given lengths/radii -> [B, nb, nb].

    Same-wire segment pairs with |alpha - beta| >= 2: Gauss q x q on G.
    |alpha - beta| <= 1: Gauss q x q on (exp(-jkR) - 1)/(4 pi R) plus the
    closed-form integral of 1/(4 pi R).
    """
    length = np.atleast_1d(np.asarray(length, dtype=np.float64))
    radius = np.broadcast_to(np.asarray(radius, dtype=np.float64), length.shape)
    xi, g = gauss01(q)
    D = length / n_seg
    s = _axis_offsets(length, n_seg, xi)                 # [B,S,Q]
    u = s[:, :, :, None, None] - s[:, None, None, :, :]  # [B,S,Q,S,Q]
    R = np.sqrt(u * u + (radius ** 2)[:, None, None, None, None])
    alpha = np.arange(n_seg)
    off = np.abs(alpha[:, None] - alpha[None, :])        # [S,S]
    near = (off <= 1)[None, :, None, :, None]
    G = np.where(near, np.expm1(-1j * k * R), np.exp(-1j * k * R)) / (FOUR_PI * R)
    phi = np.stack([xi, 1.0 - xi])
    wa = g[None, :] * phi
    A = np.einsum("ak,bl,nskul->nabsu", wa, wa, G)
    A *= (D * D)[:, None, None, None, None]
    # closed-form static part on touching/identical segments
    for n in range(length.shape[0]):
        bb = radius[n] / D[n]
        Kd = {d: static_self_integral(d, bb) for d in (-1, 0, 1)}
        for al in range(n_seg):
            for be in range(n_seg):
                d = al - be
                if abs(d) <= 1:
                    A[n, :, :, al, be] += D[n] / FOUR_PI * Kd[d]
    Bsum = A.sum(axis=(1, 2))
    return _assemble(A, Bsum, np.ones(length.shape[0]), D, D, k)


# ----------------------------------------------------------------------------
# S-NFC near set (eq. 9) and matrices
# ----------------------------------------------------------------------------

def _d2(ci: np.ndarray, cj: np.ndarray) -> np.ndarray:
    dx = cj[..., 0] - ci[..., 0]
    dy = cj[..., 1] - ci[..., 1]
    dz = cj[..., 2] - ci[..., 2]
    return (dx * dx + dy * dy) + dz * dz   # numpy never fuses: each op rounded


def near_pairs(center: np.ndarray, cloud_off, d_c: float, method: str = "auto"):
    """All ordered pairs (i, j), i != j, of the same cloud with centroid distance <= d_c.

    Returns (I, J) int64 arrays sorted by (I, J).  Brute force for small
    clouds; for large clouds a k-d tree proposes candidates and the same
    exact FP64 test decides.
    """
    dc2 = d_c * d_c
    Is, Js = [], []
    for c in range(len(cloud_off) - 1):
        lo, hi = int(cloud_off[c]), int(cloud_off[c + 1])
        n = hi - lo
        use_tree = (method == "tree") or (method == "auto" and n > 6000 and math.isfinite(d_c))
        if not use_tree:
            step = max(1, 4_000_000 // max(n, 1))
            for r0 in range(lo, hi, step):
                r1 = min(hi, r0 + step)
                d2 = _d2(center[r0:r1, None, :], center[None, lo:hi, :])
                ii, jj = np.nonzero(d2 <= dc2)
                ii = ii + r0
                jj = jj + lo
                keep = ii != jj
                Is.append(ii[keep])
                Js.append(jj[keep])
        else:
            from scipy.spatial import cKDTree
            tree = cKDTree(center[lo:hi])
            pr = tree.query_pairs(d_c * (1.0 + 1e-9) + 1e-12, output_type="ndarray")
            if pr.size:
                a = pr[:, 0] + lo
                b = pr[:, 1] + lo
                ok = _d2(center[a], center[b]) <= dc2
                a, b = a[ok], b[ok]
                Is += [a, b]
                Js += [b, a]
    if Is:
        I = np.concatenate(Is).astype(np.int64)
        J = np.concatenate(Js).astype(np.int64)
    else:
        I = np.zeros(0, np.int64)
        J = np.zeros(0, np.int64)
    order = np.lexsort((J, I))
    return I[order], J[order]


def bsr_pattern(n: int, I: np.ndarray, J: np.ndarray):
    """Row pointers / column indices of the block pattern incl. the diagonal."""
    rows = np.concatenate([I, np.arange(n)])
    cols = np.concatenate([J, np.arange(n)])
    order = np.lexsort((cols, rows))
    rows = rows[order]
    cols = cols[order]
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(indptr, rows + 1, 1)
    indptr = np.cumsum(indptr)
    return indptr, cols.astype(np.int64), rows.astype(np.int64)


def cloud_blocks(cloud, n_seg: int = 8, q_mutual: int = 4, q_self: int = 8,
                 rows=None, cols=None, batch: int = 512):
    """Blocks Z[rows[b], cols[b]] (p == p' uses the self rule)."""
    k = 2.0 * math.pi / cloud.wavelength
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    nb = n_seg - 1
    out = np.zeros((rows.shape[0], nb, nb), dtype=np.complex128)
    diag = rows == cols
    idx = np.nonzero(diag)[0]
    for s in range(0, idx.size, batch):
        e = idx[s:s + batch]
        out[e] = self_blocks(cloud.length[rows[e]], cloud.radius[rows[e]], k, n_seg, q_self)
    idx = np.nonzero(~diag)[0]
    for s in range(0, idx.size, batch):
        e = idx[s:s + batch]
        out[e] = mutual_blocks(cloud.center, cloud.tangent, cloud.length, cloud.radius,
                               rows[e], cols[e], k, n_seg, q_mutual)
    return out


def dense_Z(cloud, n_seg: int = 8, q_mutual: int = 4, q_self: int = 8) -> np.ndarray:
    """Full "entire coupling" matrix (every block of every cloud pair computed).

    Blocks between different clouds are zero (independent clouds).
    """
    n = cloud.n
    nb = n_seg - 1
    cid = np.repeat(np.arange(cloud.n_clouds), np.diff(cloud.cloud_off))
    I, J = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    I = I.ravel()
    J = J.ravel()
    same = cid[I] == cid[J]
    blocks = np.zeros((n * n, nb, nb), dtype=np.complex128)
    blocks[same] = cloud_blocks(cloud, n_seg, q_mutual, q_self, I[same], J[same])
    Z = blocks.reshape(n, n, nb, nb).transpose(0, 2, 1, 3).reshape(n * nb, n * nb)
    return Z


def snfc_matrix(cloud, n_seg: int = 8, q_mutual: int = 4, q_self: int = 8, pairs=None):
    """S-NFC block-sparse matrix (scipy BSR, caller wire order) and its pattern."""
    import scipy.sparse as sp
    n = cloud.n
    nb = n_seg - 1
    if pairs is None:
        pairs = near_pairs(cloud.center, cloud.cloud_off, cloud.d_c)
    I, J = pairs
    indptr, indices, rows = bsr_pattern(n, I, J)
    data = cloud_blocks(cloud, n_seg, q_mutual, q_self, rows, indices)
    Z = sp.bsr_matrix((data, indices, indptr), shape=(n * nb, n * nb), blocksize=(nb, nb))
    return Z, (indptr, indices, rows)


# ----------------------------------------------------------------------------
# excitation and far field
# ----------------------------------------------------------------------------

def _triangle_ft(cloud, dirs: np.ndarray, pol: np.ndarray, sign: float, n_seg: int):
    """F[p*nb+q, m] = int L_{p,q}(s) (t_p . pol_m) exp(sign j k dir_m . (c_p + s t_p)) ds.

    Closed form of the triangle transform: for a rooftop of half-width D
    centred at s_q, int L(s) exp(j b s) ds = exp(j b s_q) D sinc^2(b D / 2)
    with sinc x = sin x / x.
    """
    k = 2.0 * math.pi / cloud.wavelength
    nb = n_seg - 1
    D = cloud.length / n_seg                                  # [N]
    sq = -0.5 * cloud.length[:, None] + D[:, None] * np.arange(1, n_seg)[None, :]  # [N,nb]
    tp = cloud.tangent @ pol.T                                # [N,M]
    beta = k * (cloud.tangent @ dirs.T)                       # [N,M]
    ph0 = k * (cloud.center @ dirs.T)                         # [N,M]
    env = D[:, None] * np.sinc(beta * D[:, None] / (2.0 * math.pi)) ** 2
    F = (tp * env)[:, None, :] * np.exp(sign * 1j * (ph0[:, None, :]
                                                     + beta[:, None, :] * sq[:, :, None]))
    return F.reshape(cloud.n * nb, dirs.shape[0])


def excitation(cloud, k_hat: np.ndarray, e_hat: np.ndarray, n_seg: int = 8) -> np.ndarray:
    """u [N*nb, R]: tested incident field of eq. (4) without the -(j/(w mu0)) factor."""
    return _triangle_ft(cloud, np.atleast_2d(k_hat), np.atleast_2d(e_hat), -1.0, n_seg)


def farfield_weights(cloud, r_hat: np.ndarray, e_hat: np.ndarray, n_seg: int = 8) -> np.ndarray:
    """w [N*nb, M]: radiation functional for observation direction r_hat, polarisation e_hat."""
    return _triangle_ft(cloud, np.atleast_2d(r_hat), np.atleast_2d(e_hat), +1.0, n_seg)


def rcs_from_currents(cloud, x: np.ndarray, r_hat: np.ndarray, e_hat: np.ndarray,
                      n_seg: int = 8, cloud_index: int | None = None) -> np.ndarray:
    """sigma [R, M] = |w(r_hat_m, e_m)^T x_r|^2 / (4 pi) in m^2.

    With ``cloud_index`` the sum runs over that cloud's wires only.
    """
    x = np.asarray(x).reshape(cloud.n * (n_seg - 1), -1)
    w = farfield_weights(cloud, r_hat, e_hat, n_seg)
    if cloud_index is not None:
        nb = n_seg - 1
        lo, hi = cloud.cloud_off[cloud_index] * nb, cloud.cloud_off[cloud_index + 1] * nb
        w = w[lo:hi]
        x = x[lo:hi]
    S = x.T @ w                                               # [R,M]
    return np.abs(S) ** 2 / FOUR_PI


def monostatic_rcs(cloud, x: np.ndarray, k_hat: np.ndarray, e_hat: np.ndarray,
                   n_seg: int = 8) -> np.ndarray:
    """Backscatter sigma_r for RHS r: observation -k_hat[r], polarisation e_hat[r]."""
    k_hat = np.atleast_2d(k_hat)
    e_hat = np.atleast_2d(e_hat)
    x = np.asarray(x).reshape(cloud.n * (n_seg - 1), -1)
    w = farfield_weights(cloud, -k_hat, e_hat, n_seg)
    S = np.sum(w * x, axis=0)
    return np.abs(S) ** 2 / FOUR_PI
