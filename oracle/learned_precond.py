"""Learned neighbourhood-inverse preconditioner (oracle; test infrastructure only).

The network of ``oracle.mlp`` (192 inputs, three SiLU layers of 128, 14
outputs) used as a block preconditioner: instead of computing each wire's row
of the inverse of its neighbourhood submatrix (``oracle.precond``), the
network predicts that row from the neighbourhood's geometry, one 7-entry
column of one 7 x 7 block per sample; the predicted rows are then symmetrised
exactly as the computed ones (M_pq = (R_p[p,q] + R_q[q,p]^T) / 2).  The
preconditioner changes only how fast the solver converges, never the
solution of the S-NFC system.

Canonical frame.  Every wire gets a canonical tangent tau_p = sigma_p t_p,
sigma_p = +1 when the first nonzero of (t_z, t_y, t_x) is positive, else -1
(no incidence enters a preconditioner).  With S_p = sigma_p P_p (P_p the
identity, or the reversal q -> 6 - q of the rooftops when sigma_p = -1), a
wire's rooftop coefficients in the canonical frame are S_p x_p, blocks of Z
become S_p Z_pq S_q and so do blocks of any inverse: the canonical raw row
block is S_p R_p[p,q] S_q.

Samples.  Row (p, s, c), row index (p K + s) 7 + c in caller wire order: slot
s of p's neighbourhood N(p) (q = N(p)[s]), column c of the canonical block.
Slots beyond |N(p)| are empty rows (features and targets zero; ignored).

Features (FP64, rounded to BF16 once), with d_xy = c_y - c_x, k = 2 pi/lambda,
E(x) = exp(-j k x):
  [c]           = 1                       (one-hot column, 0..6)
  [7 + s]       = 1                       (one-hot slot, 7..14)
  [15], [16]    = 10 (L_p/lambda - 1/2), 10 (L_q/lambda - 1/2)
  [17..22]      = |d_pq|/d_c, tau_p.d_pq/d_c, tau_q.d_pq/d_c, tau_p.tau_q,
                  Re, Im E(|d_pq|)
  [23]          = |N(p)| / 8
  member t of N(p) (slot order), at 24 + 15 t:
                  1, 10 (L_t/lambda - 1/2),
                  |d_pt|/d_c, tau_p.d_pt/d_c, tau_t.d_pt/d_c, tau_p.tau_t, Re, Im E(|d_pt|),
                  |d_qt|/d_c, tau_q.d_qt/d_c, tau_t.d_qt/d_c, tau_q.tau_t, Re, Im E(|d_qt|),
                  1 if t and q are a near pair (eq. 9) or t = q, else 0
  (144 used, 48 zero.)

Targets: y[2i] + j y[2i+1] = G * (S_p (R_p[p,q] - delta_pq Z_pp^-1) S_q)[i, c],
G = TARGET_SCALE: the network predicts what the neighbourhood changes in the
row against the block-diagonal preconditioner of Sec. II-B (the diagonal raw
block is Z_pp^-1 plus a correction, the other raw blocks are corrections
only), so that a network with zero output gives exactly the block-diagonal
preconditioner.  (The raw diagonal blocks are 10-100 times larger than
their corrections and than the other blocks.)
"""
from __future__ import annotations

import math

import numpy as np

from .mlp import self_inverse
from .mom import _d2
from .precond import symmetrise  # noqa: F401  (the same symmetrisation as the computed rows)

N_FEAT = 192
N_OUT = 14
NB = 7
K_MAX = 8
F_HEAD = 24
F_MEMBER = 15
TARGET_SCALE = 0.05


def canonical_sign(tangent: np.ndarray) -> np.ndarray:
    """sigma [N]: +1 when the first nonzero of (t_z, t_y, t_x) is positive, else -1."""
    t = np.asarray(tangent, dtype=np.float64)
    pos = (t[:, 2] > 0) | ((t[:, 2] == 0) & ((t[:, 1] > 0) | ((t[:, 1] == 0) & (t[:, 0] > 0))))
    return np.where(pos, 1.0, -1.0)


def _S(sig: float) -> np.ndarray:
    """S = sigma P: the canonical-frame map of one wire's rooftop coefficients."""
    return np.eye(NB) if sig > 0 else -np.eye(NB)[::-1]


def features(cloud, nbhd, size: int) -> np.ndarray:
    """F [N*size*7, 192] in FP64 (unrounded)."""
    n = cloud.n
    lam = cloud.wavelength
    k = 2.0 * math.pi / lam
    dc = cloud.d_c
    if not math.isfinite(dc):
        raise ValueError("the learned preconditioner needs a finite d_c")
    c = np.asarray(cloud.center, dtype=np.float64)
    sig = canonical_sign(cloud.tangent)
    tau = sig[:, None] * cloud.tangent
    L = cloud.length
    out = np.zeros((n, size, NB, N_FEAT))

    def rel(x, y):   # the six pair features of (x, y), d = c_y - c_x
        d = c[y] - c[x]
        dist = math.sqrt(_d2(c[x], c[y]))
        e = np.exp(-1j * k * dist)
        return [dist / dc, float(tau[x] @ d) / dc, float(tau[y] @ d) / dc, float(tau[x] @ tau[y]), e.real, e.imag]

    dc2 = dc * dc
    for p in range(n):
        g = [int(v) for v in nbhd[p]]
        m = len(g)
        for s in range(min(m, size)):
            q = g[s]
            f = np.zeros(N_FEAT)
            f[7 + s] = 1.0
            f[15] = 10.0 * (L[p] / lam - 0.5)
            f[16] = 10.0 * (L[q] / lam - 0.5)
            f[17:23] = rel(p, q)
            f[23] = m / 8.0
            for t, w in enumerate(g):
                b = F_HEAD + F_MEMBER * t
                f[b] = 1.0
                f[b + 1] = 10.0 * (L[w] / lam - 0.5)
                f[b + 2:b + 8] = rel(p, w)
                f[b + 8:b + 14] = rel(q, w)
                f[b + 14] = 1.0 if (w == q or _d2(c[q], c[w]) <= dc2) else 0.0
            for cc in range(NB):
                out[p, s, cc] = f
                out[p, s, cc, cc] = 1.0
    return out.reshape(n * size * NB, N_FEAT)


def targets(cloud, nbhd, size: int, raw: dict, dinv=None) -> np.ndarray:
    """Y [N*size*7, 14] from raw row blocks {(p, q): R_p[p,q]} (caller order);
    dinv [N, 7, 7] = Z_pp^-1 (computed here when not given)."""
    n = cloud.n
    dinv = self_inverse(cloud) if dinv is None else dinv
    sig = canonical_sign(cloud.tangent)
    y = np.zeros((n, size, NB, N_OUT))
    for p in range(n):
        for s, q in enumerate(nbhd[p][:size]):
            q = int(q)
            dep = raw[(p, q)] - (dinv[p] if q == p else 0.0)
            blk = _S(sig[p]) @ dep @ _S(sig[q]) * TARGET_SCALE
            y[p, s, :, 0::2] = blk.real.T     # row c of y = column c of the block
            y[p, s, :, 1::2] = blk.imag.T
    return y.reshape(n * size * NB, N_OUT)


def raw_from_outputs(cloud, nbhd, size: int, y: np.ndarray, dinv=None) -> dict:
    """{(p, q): R_p[p,q]} from network outputs Y [N*size*7, 14]; inverse of ``targets``."""
    n = cloud.n
    dinv = self_inverse(cloud) if dinv is None else dinv
    sig = canonical_sign(cloud.tangent)
    yr = np.asarray(y, dtype=np.float64).reshape(n, size, NB, N_OUT)
    out = {}
    for p in range(n):
        for s, q in enumerate(nbhd[p][:size]):
            q = int(q)
            blk = (yr[p, s, :, 0::2] + 1j * yr[p, s, :, 1::2]).T / TARGET_SCALE   # [i, c]
            out[(p, q)] = _S(sig[p]) @ blk @ _S(sig[q]) + (dinv[p] if q == p else 0.0)
    return out
