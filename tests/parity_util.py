"""Helpers shared by the GPU parity tests (not collected by pytest).

They map the GPU's internal (Morton) order back to the caller's wire order
and compute the oracle's side of each comparison.  Nothing here feeds a GPU
result into an oracle computation.
"""
import math
import sys

import numpy as np

from oracle import mom

NB = 7


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_pairs(cl):
    """Ordered off-diagonal pairs (caller indices) of the GPU pattern, sorted."""
    row_ptr, col_idx, perm, diag = cl.pattern()
    n = cl.n
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    I = perm[rows].astype(np.int64)
    J = perm[col_idx].astype(np.int64)
    off = I != J
    I, J = I[off], J[off]
    o = np.lexsort((J, I))
    return I[o], J[o]


def gpu_blocks_caller(cl, Z):
    """(rows, cols, blocks) of the GPU matrix in caller wire indices."""
    row_ptr, col_idx, perm, diag = cl.pattern()
    rows = np.repeat(np.arange(cl.n), np.diff(row_ptr))
    return perm[rows].astype(np.int64), perm[col_idx].astype(np.int64), Z.cpu().numpy()


def rel_block_err(A, B):
    """Per-block relative Frobenius error ||A-B|| / ||B||."""
    num = np.linalg.norm((A - B).reshape(A.shape[0], -1), axis=1)
    den = np.linalg.norm(B.reshape(B.shape[0], -1), axis=1)
    return num / den


def db_err(sig_gpu, sig_orc, floor=1e-4):
    """R12: |10 log10(gpu/orc)| on entries >= floor * max; returns (max dB err, max rel err below floor)."""
    sig_gpu = np.asarray(sig_gpu, dtype=np.float64).ravel()
    sig_orc = np.asarray(sig_orc, dtype=np.float64).ravel()
    top = sig_orc.max()
    keep = sig_orc >= floor * top
    e_db = np.abs(10 * np.log10(sig_gpu[keep] / sig_orc[keep])).max() if keep.any() else 0.0
    e_lo = (np.abs(sig_gpu[~keep] - sig_orc[~keep]).max() / top) if (~keep).any() else 0.0
    return float(e_db), float(e_lo)


def oracle_bistatic(cloud, x, rh, th, ph, chunk=8192):
    """Oracle sigma for theta- and phi-polarised observation over a direction grid."""
    out_t, out_p = [], []
    for s in range(0, rh.shape[0], chunk):
        out_t.append(mom.rcs_from_currents(cloud, x, rh[s:s + chunk], th[s:s + chunk])[0])
        out_p.append(mom.rcs_from_currents(cloud, x, rh[s:s + chunk], ph[s:s + chunk])[0])
    return np.concatenate(out_t), np.concatenate(out_p)


def oracle_mono_per_cloud(cloud, x, k_hat, e_hat):
    """[n_clouds, R] monostatic sigma, each cloud summed over its own wires."""
    out = np.zeros((cloud.n_clouds, k_hat.shape[0]))
    w = mom.farfield_weights(cloud, -k_hat, e_hat)
    for c in range(cloud.n_clouds):
        lo, hi = cloud.cloud_off[c] * NB, cloud.cloud_off[c + 1] * NB
        S = np.sum(w[lo:hi] * x[lo:hi], axis=0)
        out[c] = np.abs(S) ** 2 / (4 * math.pi)
    return out


def current_err(xg, xo):
    """Per-RHS relative L2 current error."""
    xg = np.asarray(xg).reshape(xo.shape)
    return np.linalg.norm(xg - xo, axis=0) / np.linalg.norm(xo, axis=0)


def fp32_block_check(rows, cols, Zg, Zo, rel=1e-5, floor=1e-7, row_rel=2e-6):
    """FP32 block criterion.

    Every block: ||dZ|| <= rel*||Z_b|| + floor*||Z_ii|| (i its row's self block);
    every block row: ||dZ_row|| <= row_rel*||Z_row||.  Blocks whose value
    nearly cancels (transverse factor ~ 0) carry FP32 rounding amplified
    relative to their own size, but not relative to their row.
    Returns a dict of the observed figures.
    """
    Zg = Zg.astype(np.complex128)
    d = np.linalg.norm((Zg - Zo).reshape(len(rows), -1), axis=1)
    nb = np.linalg.norm(Zo.reshape(len(rows), -1), axis=1)
    diag = {int(r): k for k, (r, c) in enumerate(zip(rows, cols)) if r == c}
    nd = np.array([nb[diag[int(r)]] for r in rows])
    ok = d <= rel * nb + floor * nd
    n = int(max(rows.max(), cols.max())) + 1
    rd = np.zeros(n)
    rn = np.zeros(n)
    np.add.at(rd, rows, d ** 2)
    np.add.at(rn, rows, nb ** 2)
    have = rn > 0   # rows present in the comparison (all of them, or a sample)
    row_err = np.sqrt(rd[have]) / np.sqrt(rn[have])
    out = {"max_rel": float((d / nb).max()), "median_rel": float(np.median(d / nb)),
           "max_abs_over_diag": float((d / nd).max()), "max_row_rel": float(row_err.max()),
           "n_fail": int((~ok).sum())}
    return out, bool(ok.all() and row_err.max() <= row_rel)
