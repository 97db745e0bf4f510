#!/usr/bin/env python3
"""Write the oracle's solutions of the two largest workloads (test fixture).

    python tests/golden/make_fullsize_golden.py c4_eval [--procs 8]
    python tests/golden/make_fullsize_golden.py c5 [--procs 8] [--incidences 4]

Only the FP64 oracle (``oracle/``) and the seeded input generator
(``paper_2410_03060_amd.workloads``, which holds none of the method's
arithmetic) are used; nothing here touches the GPU library.

For each workload the S-NFC system (Galerkin blocks of eqs. 5-8 on the near
set of eq. 9) is assembled in complex128 by ``oracle.mom``, and the chosen
incidences (eq. 4 excitations) are solved with the oracle's FP64 GMRES to a
tight relative residual.  The preconditioner is the oracle's cluster inverse
(``oracle.precond``: exact inverse of the diagonal submatrix of each group of
8 nearby wires), which changes only the iteration count, never the solution.
The blocks are filled in parallel worker processes, each running the oracle's
``cloud_blocks`` on a contiguous range of stored blocks; incidences are solved
in parallel, one process per incidence.

Stored per incidence (``fullsize_<config>.npz`` beside this script):
  incidences   indices into the workload's incidence list
  sigma        monostatic RCS [m^2] of the whole cloud (far-field functional)
  xnorm        ||x||_2 of all currents
  rel_res      the true FP64 relative residual ||u - Z x|| / ||u|| reached
  iterations   GMRES inner iterations
  wires        2,000 seeded caller wire indices (rng 11)
  currents     their currents x [2000*7, n_inc] (complex128, wire-major)
"""
from __future__ import annotations

import argparse
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import mom, precond, solve  # noqa: E402
from paper_2410_03060_amd import workloads as W  # noqa: E402

NB = 7
HERE = os.path.dirname(os.path.abspath(__file__))
N_SAMPLE_WIRES = 2000

# state shared with forked workers (set before the pools start)
_G: dict = {}


def log(*a):
    print(f"[golden {time.strftime('%H:%M:%S')}]", *a, flush=True)


def _fill_chunk(rng_):
    b0, b1 = rng_
    out = np.ndarray((_G["nblocks"], NB, NB), dtype=np.complex128, buffer=_G["shm"].buf)
    out[b0:b1] = mom.cloud_blocks(_G["cloud"], rows=_G["rows"][b0:b1], cols=_G["cols"][b0:b1])
    return b1 - b0


def assemble(cloud, procs: int):
    """S-NFC matrix (scipy BSR, caller order) with blocks filled by worker processes."""
    import scipy.sparse as sp
    from multiprocessing import shared_memory
    t0 = time.time()
    I, J = mom.near_pairs(cloud.center, cloud.cloud_off, cloud.d_c)
    indptr, indices, rows = mom.bsr_pattern(cloud.n, I, J)
    nblocks = indices.size
    log(f"near set: {I.size} ordered pairs, {nblocks} blocks ({time.time() - t0:.1f} s)")
    shm = shared_memory.SharedMemory(create=True, size=nblocks * NB * NB * 16)
    _G.update(cloud=cloud, rows=rows, cols=indices, nblocks=nblocks, shm=shm)
    step = 4096
    chunks = [(b, min(b + step, nblocks)) for b in range(0, nblocks, step)]
    t0 = time.time()
    done = 0
    with mp.get_context("fork").Pool(procs) as pool:
        for k, n in enumerate(pool.imap_unordered(_fill_chunk, chunks)):
            done += n
            if k % 200 == 0:
                log(f"fill {done}/{nblocks} blocks ({time.time() - t0:.0f} s)")
    data = np.ndarray((nblocks, NB, NB), dtype=np.complex128, buffer=shm.buf).copy()
    shm.close()
    shm.unlink()
    log(f"fill done ({time.time() - t0:.0f} s)")
    Z = sp.bsr_matrix((data, indices, indptr), shape=(cloud.n * NB, cloud.n * NB), blocksize=(NB, NB))
    return Z


def _solve_one(r):
    Z, u, apply_m, rtol, restart = _G["Z"], _G["u"], _G["apply_m"], _G["rtol"], _G["restart"]
    st: dict = {}
    t0 = time.time()
    x = solve.gmres_solve(Z, u[:, r], NB, rtol=rtol, restart=restart, maxiter=2000, apply_m=apply_m,
                          stats=st)
    rr = float(solve.relative_residual(Z, x[:, None], u[:, r:r + 1])[0])
    log(f"incidence column {r}: {st['iterations'][0]} iterations, true residual {rr:.2e} "
        f"({time.time() - t0:.0f} s)")
    return r, x, rr, st["iterations"][0]


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("config", choices=["c4_eval", "c5"])
    ap.add_argument("--procs", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--incidences", type=int, default=None,
                    help="number of incidences solved (c4_eval: all 8; c5: a seeded 4 of 64)")
    ap.add_argument("--rtol", type=float, default=1e-10)
    ap.add_argument("--restart", type=int, default=60)
    a = ap.parse_args(argv)

    wl = getattr(W, a.config)()
    cloud = wl.cloud
    R = wl.inc.k_hat.shape[0]
    if a.config == "c4_eval":
        inc = np.arange(R) if a.incidences is None else np.arange(a.incidences)
    else:
        n_inc = 4 if a.incidences is None else a.incidences
        inc = np.sort(np.random.default_rng(13).choice(R, n_inc, replace=False))
    log(f"{a.config}: N={cloud.n}, incidences {inc.tolist()}, rtol {a.rtol}, {a.procs} processes")

    Z = assemble(cloud, a.procs)
    t0 = time.time()
    groups = precond.clusters(cloud, 8)
    Minv = precond.cluster_inverse(Z, groups, 8)
    log(f"cluster inverse of {len(groups)} groups ({time.time() - t0:.0f} s)")

    kh, eh = wl.inc.k_hat[inc], wl.inc.e_hat[inc]
    u = mom.excitation(cloud, kh, eh)
    _G.update(Z=Z, u=u, apply_m=lambda v: precond.cluster_apply(Minv, groups, v), rtol=a.rtol,
              restart=a.restart)
    x = np.zeros_like(u)
    rel = np.zeros(len(inc))
    its = np.zeros(len(inc), dtype=np.int64)
    with mp.get_context("fork").Pool(min(a.procs, len(inc))) as pool:
        for r, xr, rr, it in pool.imap_unordered(_solve_one, range(len(inc))):
            x[:, r], rel[r], its[r] = xr, rr, it
    assert np.all(rel <= a.rtol * 1.01), rel

    sigma = mom.monostatic_rcs(cloud, x, kh, eh)
    wires = np.sort(np.random.default_rng(11).choice(cloud.n, min(N_SAMPLE_WIRES, cloud.n), replace=False))
    rows = (NB * wires[:, None] + np.arange(NB)[None, :]).reshape(-1)
    out = os.path.join(HERE, f"fullsize_{a.config}.npz")
    np.savez_compressed(out, config=a.config, incidences=inc, sigma=sigma, xnorm=np.linalg.norm(x, axis=0),
                        rel_res=rel, iterations=its, wires=wires, currents=x[rows], rtol=a.rtol)
    log(f"wrote {out}: sigma/lambda^2 {np.round(sigma / cloud.wavelength ** 2, 3).tolist()}, "
        f"iterations {its.tolist()}, residuals {rel.tolist()}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
