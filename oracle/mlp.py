"""Learned initial guess for the Krylov solve (oracle; test infrastructure only).

The paper solves every incidence from scratch.  The learned part predicts,
for each wire and incidence, the wire's 7 rooftop currents from its local
neighbourhood, and the prediction is handed to the solver as its initial
iterate.  Nothing here changes the solution of the S-NFC system: the solver
still drives the true residual to the same tolerance.

This module is the plain definition of every step, in FP64 NumPy:

* ``knn``        -- the (up to) 16 nearest other wires of the same cloud
                    within d_c, ascending in (squared distance, caller index),
                    squared distance formed exactly as in the near-set test
                    of eq. (9);
* ``features``   -- 192 rotation- and translation-invariant numbers per
                    (wire, incidence), in the wire's canonical frame;
* ``targets`` / ``currents_from_outputs`` -- the map between solved currents
                    and the 14 network outputs: the departure of the currents
                    from the wire's isolated (block-Jacobi) response
                    b_p = Z_pp^{-1} u_p, in the canonical frame, incident
                    phase at the wire centre removed, fixed scale;
* ``forward`` / ``loss_and_grad`` -- the 192-128-128-128-14 SiLU network,
                    optionally with the BF16 rounding points of the GPU
                    method emulated (BF16 weights and layer inputs, exact
                    accumulation, FP32 biases);
* ``adam``       -- one Adam update.

Canonical frame.  With s_p = +1 if t_p . e >= 0 else -1 the wire's canonical
tangent is tau_p = s_p t_p.  Reversing a wire's tangent reverses the order of
its rooftops (q -> 6 - q) and negates their coefficients, so the canonical
currents are x~_{p,q} = s_p x_{p, q'} with q' = q (s_p = 1) or 6 - q.

Per (wire p, incidence with propagation k_hat, polarisation e), k = 2 pi/lambda,
Delta_p = L_p/8, beta_p = k (k_hat . tau_p), s_q = -L_p/2 + (q+1) Delta_p:

  own[0]            = 10 (L_p/lambda - 1/2)
  own[1]            = n_p / 16          (n_p = other wires within d_c)
  own[2+2q], [3+2q] = Re, Im of (tau_p . e) sinc^2(beta_p Delta_p / 2)
                       exp(-j beta_p s_q)            (q = 0..6; sinc x = sin x/x)

and for neighbour slot j (j-th nearest p', d = c_p' - c_p), at 16 + 11 j:

  |d|/d_c, (tau_p . d)/d_c, (tau_p' . d)/d_c, tau_p . tau_p',
  Re, Im of (tau_p' . e) exp(-j k (k_hat . d)), 10 (L_p'/lambda - 1/2),
  k_hat . tau_p', Re, Im of exp(-j k |d|) (the retardation of the coupling
  between the two centres), 1
  (all zero for an empty slot).

Own features 2..15 are the excitation of eq. (4) in the canonical frame,
divided by Delta_p and with the incident phase at c_p removed.

Targets: y[2q] + j y[2q+1] = (x~_{p,q} - b~_{p,q}) exp(+j k k_hat . c_p) / 0.5,
where b~ is the canonical form of b_p = Z_pp^{-1} u_p (the currents the wire
would carry alone) -- the network predicts only what the neighbours change.

Rounding to BF16 (``bf16``): FP64 -> FP32 (nearest even) -> BF16 (nearest
even on the FP32 bit pattern).

Sample (row) order everywhere: row = p * R + r, caller wire order p.
"""
from __future__ import annotations

import math

import numpy as np

from .mom import _d2, excitation, near_pairs, self_blocks

K_NB = 16
F_OWN = 16
F_NB = 11
N_FEAT = F_OWN + K_NB * F_NB       # 192
HIDDEN = 128
N_OUT = 14
X_SCALE = 0.5
LAYERS = ((N_FEAT, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, N_OUT))


# ----------------------------------------------------------------------------
# parameters: W1 [192][128], b1 [128], W2, b2, W3, b3, W4 [128][14], b4 [14]
# (each W stored input-major: W[i][o] at offset + i*n_out + o)
# ----------------------------------------------------------------------------

def param_layout():
    """[(w_off, b_off, n_in, n_out)] per layer and the total count."""
    out, off = [], 0
    for n_in, n_out in LAYERS:
        out.append((off, off + n_in * n_out, n_in, n_out))
        off += n_in * n_out + n_out
    return out, off


def unpack(theta: np.ndarray):
    lay, n = param_layout()
    assert theta.shape == (n,)
    return [(theta[w:w + i * o].reshape(i, o), theta[b:b + o]) for w, b, i, o in lay]


# ----------------------------------------------------------------------------
# BF16 rounding
# ----------------------------------------------------------------------------

def bf16(x: np.ndarray) -> np.ndarray:
    """Round to BF16 (via FP32, both steps nearest-even); returned as float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(f)
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def bf16_bits(x: np.ndarray) -> np.ndarray:
    """uint16 bit patterns of bf16(x)."""
    return (bf16(x).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)


def from_bf16_bits(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint32) << 16).view(np.float32).astype(np.float64)


# ----------------------------------------------------------------------------
# neighbourhoods and features
# ----------------------------------------------------------------------------

def knn(cloud, k: int = K_NB):
    """nbr [N, k] (caller indices, -1 = empty) and n_p [N] (all within d_c)."""
    if not math.isfinite(cloud.d_c):
        raise ValueError("the learned guess needs a finite d_c")
    I, J = near_pairs(cloud.center, cloud.cloud_off, cloud.d_c)
    n = cloud.n
    d2 = _d2(cloud.center[I], cloud.center[J])
    order = np.lexsort((J, d2, I))              # by row, then distance, then index
    I, J = I[order], J[order]
    count = np.bincount(I, minlength=n)
    start = np.concatenate([[0], np.cumsum(count)])
    nbr = np.full((n, k), -1, dtype=np.int64)
    for p in range(n):
        m = min(k, count[p])
        nbr[p, :m] = J[start[p]:start[p] + m]
    return nbr, count


def canonical_sign(tangent: np.ndarray, e_hat: np.ndarray) -> np.ndarray:
    """s [N, R] = +1 where t_p . e_r >= 0, else -1."""
    return np.where(tangent @ np.atleast_2d(e_hat).T >= 0.0, 1.0, -1.0)


def _sinc(x):
    return np.sinc(x / math.pi)


def features(cloud, k_hat: np.ndarray, e_hat: np.ndarray, nbrs=None) -> np.ndarray:
    """F [N*R, 192] in FP64 (unrounded), row = p*R + r."""
    k_hat = np.atleast_2d(k_hat)
    e_hat = np.atleast_2d(e_hat)
    R = k_hat.shape[0]
    n = cloud.n
    lam = cloud.wavelength
    k = 2.0 * math.pi / lam
    nbr, count = knn(cloud) if nbrs is None else nbrs
    s = canonical_sign(cloud.tangent, e_hat)                  # [N,R]
    tau = s[:, :, None] * cloud.tangent[:, None, :]          # [N,R,3]
    L = cloud.length
    D = L / 8.0
    out = np.zeros((n, R, N_FEAT))
    te = np.einsum("nrc,rc->nr", tau, e_hat)                  # tau_p . e
    kt = np.einsum("nrc,rc->nr", tau, k_hat)                  # k_hat . tau_p
    beta = k * kt
    env = _sinc(beta * D[:, None] / 2.0) ** 2
    out[:, :, 0] = (10.0 * (L / lam - 0.5))[:, None]
    out[:, :, 1] = (count / 16.0)[:, None]
    for q in range(7):
        sq = -0.5 * L + (q + 1) * D
        z = te * env * np.exp(-1j * beta * sq[:, None])
        out[:, :, 2 + 2 * q] = z.real
        out[:, :, 3 + 2 * q] = z.imag
    for j in range(K_NB):
        pj = nbr[:, j]
        has = pj >= 0
        if not np.any(has):
            continue
        p = np.nonzero(has)[0]
        q = pj[has]
        d = cloud.center[q] - cloud.center[p]                 # [m,3]
        dist = np.sqrt(_d2(cloud.center[p], cloud.center[q]))
        tp = tau[p]                                           # [m,R,3]
        tq = tau[q]
        base = F_OWN + F_NB * j
        out[p, :, base + 0] = (dist / cloud.d_c)[:, None]
        out[p, :, base + 1] = np.einsum("mrc,mc->mr", tp, d) / cloud.d_c
        out[p, :, base + 2] = np.einsum("mrc,mc->mr", tq, d) / cloud.d_c
        out[p, :, base + 3] = np.einsum("mrc,mrc->mr", tp, tq)
        drive = np.einsum("mrc,rc->mr", tq, e_hat) * np.exp(-1j * k * (d @ k_hat.T))
        out[p, :, base + 4] = drive.real
        out[p, :, base + 5] = drive.imag
        out[p, :, base + 6] = (10.0 * (L[q] / lam - 0.5))[:, None]
        out[p, :, base + 7] = np.einsum("mrc,rc->mr", tq, k_hat)
        ret = np.exp(-1j * k * dist)
        out[p, :, base + 8] = ret.real[:, None]
        out[p, :, base + 9] = ret.imag[:, None]
        out[p, :, base + 10] = 1.0
    return out.reshape(n * R, N_FEAT)


def self_inverse(cloud) -> np.ndarray:
    """Z_pp^{-1} [N, 7, 7] (the block-Jacobi preconditioner of Sec. II-B)."""
    k = 2.0 * math.pi / cloud.wavelength
    return np.linalg.inv(self_blocks(cloud.length, cloud.radius, k))


def isolated_response(cloud, k_hat: np.ndarray, e_hat: np.ndarray, dinv=None) -> np.ndarray:
    """b [N, 7, R] = Z_pp^{-1} u_p exp(+j k k_hat . c_p) (raw rooftop order)."""
    k_hat = np.atleast_2d(k_hat)
    e_hat = np.atleast_2d(e_hat)
    n, R = cloud.n, k_hat.shape[0]
    k = 2.0 * math.pi / cloud.wavelength
    dinv = self_inverse(cloud) if dinv is None else dinv
    u = excitation(cloud, k_hat, e_hat).reshape(n, 7, R)
    ph = np.exp(1j * k * (cloud.center @ k_hat.T))            # [N,R]
    return np.einsum("nij,njr->nir", dinv, u) * ph[:, None, :]


def targets(cloud, k_hat: np.ndarray, e_hat: np.ndarray, x: np.ndarray, dinv=None) -> np.ndarray:
    """Y [N*R, 14] from currents x [N*7, R] (caller order)."""
    k_hat = np.atleast_2d(k_hat)
    e_hat = np.atleast_2d(e_hat)
    n, R = cloud.n, k_hat.shape[0]
    k = 2.0 * math.pi / cloud.wavelength
    ph = np.exp(1j * k * (cloud.center @ k_hat.T))            # [N,R]
    d = np.asarray(x).reshape(n, 7, R) * ph[:, None, :] - isolated_response(cloud, k_hat, e_hat, dinv)
    s = canonical_sign(cloud.tangent, e_hat)                  # [N,R]
    dc = np.where((s > 0)[:, None, :], d, d[:, ::-1, :])      # canonical order
    dc = s[:, None, :] * dc / X_SCALE                         # [N,7,R]
    y = np.empty((n, R, N_OUT))
    y[:, :, 0::2] = dc.real.transpose(0, 2, 1)
    y[:, :, 1::2] = dc.imag.transpose(0, 2, 1)
    return y.reshape(n * R, N_OUT)


def currents_from_outputs(cloud, k_hat: np.ndarray, e_hat: np.ndarray, y: np.ndarray, dinv=None) -> np.ndarray:
    """x [N*7, R] (caller order) from network outputs Y [N*R, 14]; inverse of ``targets``."""
    k_hat = np.atleast_2d(k_hat)
    e_hat = np.atleast_2d(e_hat)
    n, R = cloud.n, k_hat.shape[0]
    k = 2.0 * math.pi / cloud.wavelength
    yr = np.asarray(y, dtype=np.float64).reshape(n, R, N_OUT)
    dc = (yr[:, :, 0::2] + 1j * yr[:, :, 1::2]).transpose(0, 2, 1)   # [N,7,R] canonical
    s = canonical_sign(cloud.tangent, e_hat)
    dc = X_SCALE * s[:, None, :] * dc
    d = np.where((s > 0)[:, None, :], dc, dc[:, ::-1, :])
    ph = np.exp(-1j * k * (cloud.center @ k_hat.T))
    x = (d + isolated_response(cloud, k_hat, e_hat, dinv)) * ph[:, None, :]
    return x.reshape(n * 7, R)


# ----------------------------------------------------------------------------
# network: SiLU(x W1 + b1) -> SiLU(. W2 + b2) -> SiLU(. W3 + b3) -> . W4 + b4
# ----------------------------------------------------------------------------

def _sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def silu(z):
    return z * _sigmoid(z)


def silu_prime(z):
    s = _sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def _f32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def forward(theta: np.ndarray, X: np.ndarray, emulate_bf16: bool = False):
    """Outputs Y [B, 14] and the cache for ``backward``.

    ``emulate_bf16``: weights and every layer input rounded to BF16, biases
    to FP32, products accumulated exactly (FP64).
    """
    layers = unpack(np.asarray(theta, dtype=np.float64))
    a = np.asarray(X, dtype=np.float64)
    cache = []
    for li, (W, b) in enumerate(layers):
        if emulate_bf16:
            a_in, W, b = bf16(a), bf16(W), _f32(b)
        else:
            a_in = a
        z = a_in @ W + b
        cache.append((a_in, W, z))
        a = silu(z) if li < len(layers) - 1 else z
    return a, cache


def loss_and_grad(theta: np.ndarray, X: np.ndarray, T: np.ndarray, emulate_bf16: bool = False):
    """Mean squared error over B rows x 14 outputs and its gradient [P].

    ``emulate_bf16`` also rounds the back-propagated quantities where the GPU
    method feeds them to BF16 products: 2 (y - t) and every dL/dz of a hidden
    layer (the 1/(14 B) factor is applied to the final sums).
    """
    Y, cache = forward(theta, X, emulate_bf16)
    T = np.asarray(T, dtype=np.float64)
    B = Y.shape[0]
    diff = Y - T
    loss = float(np.sum(diff * diff) / (B * N_OUT))
    scale = 1.0 / (B * N_OUT)
    lay, n = param_layout()
    g = np.zeros(n)
    dz = 2.0 * diff
    for li in range(len(cache) - 1, -1, -1):
        a_in, W, z = cache[li]
        if emulate_bf16:
            dz = bf16(dz)
        w_off, b_off, n_in, n_out = lay[li]
        g[w_off:w_off + n_in * n_out] = (a_in.T @ dz).ravel() * scale
        g[b_off:b_off + n_out] = dz.sum(axis=0) * scale
        if li > 0:
            da = dz @ W.T
            dz = da * silu_prime(cache[li - 1][2])
    return loss, g


def adam(theta, m, v, g, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
         eps: float = 1e-8):
    """One Adam step (t counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def guess(cloud, k_hat, e_hat, theta, emulate_bf16: bool = True, dinv=None):
    """Initial currents x0 [N*7, R]: isolated response plus the network's correction."""
    X = features(cloud, k_hat, e_hat)
    if emulate_bf16:
        X = bf16(X)
    Y, _ = forward(theta, X, emulate_bf16)
    return currents_from_outputs(cloud, k_hat, e_hat, Y, dinv)
