"""Statistically averaged monostatic RCS of random chaff clouds.

The paper's statistical results (Sec. III-B: averaged monostatic RCS against
the mean spacing d_mean, compared with Marcus's 0.15 N_c asymptote; Sec. III-C:
the frequency response of a 1,000-chaff cloud, entire coupling against S-NFC
with d_c = 2 lambda; Sec. IV: a million identical or two-length chaffs over
frequency) average sigma_VV over many independent random clouds.  Here every
trial is one cloud of a multi-cloud input, so a whole batch of trials goes
through each stage of the library (neighbour search, fill, block-Jacobi
preconditioned Krylov solve with FP64 refinement, far field) in one launch.

The entire-coupling reference ("LU" in the paper) is the same solve with
d_c = infinity: every pair of wires of a trial is coupled, and the library
fills each trial's dense block matrix.  S-NFC and entire coupling see the same
trial geometries (same seeds), so their difference measures the
sparsification, not the sampling.

Averages are taken over trials and incidences of sigma in square metres and
reported in units of lambda^2 (and in dB); the relative error between two
averages follows Sec. III-C: log10(|sigma_ref - sigma| / |sigma_ref|).
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import workloads as W

# Sec. III-B: 100 trials of 1,000 half-wave chaffs per mean spacing
E2_TRIALS, E2_WIRES = 100, 1000
E2_SPACINGS = (0.5, 0.75, 1.0, 1.5, 2.0)         # d_mean / lambda (block-Jacobi COCG stalls below 0.5)
E2_CUTOFFS = (1.0, 2.0, 3.0, 4.0, math.inf)       # d_c / lambda
# Sec. III-C: 1,000 chaffs of length l1 in a sphere of radius 10 m, 100 trials per frequency
E3_TRIALS, E3_WIRES, E3_LENGTH, E3_RADIUS = 100, 1000, 0.01153, 10.0
E3_FREQS = tuple(round(0.6 + 0.1 * i, 1) for i in range(21))   # f / f1, f1 = c / (2 l1)
E3_CUTOFFS = (2.0, math.inf)
# Sec. IV: 10^6 chaffs in a sphere of radius 10 m, lengths l1 (identical) or l1 and l2 (two lengths)
E6_WIRES, E6_RADIUS, E6_L1, E6_L2 = 1_000_000, 10.0, 0.01125, 0.008817


def _max_nnzb(cloud: W.Cloud):
    """Dense trials need every (i, j) pair of each cloud; sparse ones use the library's estimate."""
    if math.isfinite(cloud.d_c):
        return None
    sizes = np.diff(cloud.cloud_off).astype(np.int64)
    return int(np.sum(sizes * sizes))


def solve_trials(cloud: W.Cloud, inc: W.Incidence, prec: str = "c64", tol: float = 1e-6,
                 max_cycles: int = 8, device: str = "cuda"):
    """Monostatic sigma [trials, R] (m^2) of every cloud of ``cloud`` and the solve
    statistics: one multi-cloud launch per stage, COCG with block-Jacobi (at
    most ``max_cycles`` refinement cycles of up to 5,000 steps; a trial that
    does not reach ``tol`` is reported as not converged, not dropped)."""
    import torch
    from . import binding as B
    p = B.C64 if prec == "c64" else B.C128
    t0 = time.perf_counter()
    cl = B.build_cloud(cloud, device=device, max_nnzb=_max_nnzb(cloud))
    try:
        Z, P = B.fill_Z(cl, p)
        opts = B.solve_opts(tol=tol, inner_tol=1e-5, restart=5000, max_cycles=max_cycles, prec=p,
                            method=B.COCG)
        X, info = B.solve(cl, Z, P, inc.k_hat, inc.e_hat, opts, raise_on_noconv=False)
        sig = B.rcs(cl, X, -inc.k_hat, inc.e_hat, monostatic=True)
        out = sig.cpu().numpy()
        torch.cuda.synchronize()
        stats = {"iterations": int(info["iterations"]), "cycles": int(info["cycles"]),
                 "max_rel_residual": float(info["max_rel_residual"]), "converged": info["status"] == B.OK,
                 "nnzb": int(cl.nnzb), "seconds": time.perf_counter() - t0}
        del Z, P, X, sig
        return out, stats
    finally:
        B.destroy(cl)


def average(sigma: np.ndarray, wavelength: float) -> dict:
    """Mean of sigma over trials and incidences, in lambda^2 and dB, with its
    standard error (trials x incidences taken as independent samples)."""
    s = np.asarray(sigma, dtype=np.float64).reshape(-1) / wavelength ** 2
    mean = float(s.mean())
    se = float(s.std(ddof=1) / math.sqrt(s.size)) if s.size > 1 else float("nan")
    return {"sigma_lambda2": mean, "sigma_db": 10.0 * math.log10(mean), "stderr_lambda2": se,
            "samples": int(s.size)}


def log_rel_error(ref: float, val: float) -> float:
    """log10(|ref - val| / |ref|) of two averaged values (Sec. III-C); -inf if equal."""
    d = abs(ref - val)
    return -math.inf if d == 0 else math.log10(d / abs(ref))


def run_point(seed0: int, trials: int, n: int, sphere_radius: float, length, wavelength: float,
              cutoffs, batch: int, prec: str = "c64", incidences: int = 1) -> list[dict]:
    """One abscissa of an ensemble experiment: the same trials at every d_c
    (in wavelengths; infinity = entire coupling), in batches of ``batch``
    trials per launch, each trial lit by ``incidences`` V-polarised waves
    from equally spaced azimuths (one: from +x) solved in lockstep.  Returns
    one record per d_c."""
    inc = W.azimuth_incidences(incidences)
    recs = []
    for dc in cutoffs:
        sig, st = [], {"iterations": 0, "seconds": 0.0, "max_rel_residual": 0.0, "converged": True, "nnzb": 0}
        for b0 in range(0, trials, batch):
            nb = min(batch, trials - b0)
            print(f"[ensemble] d_c {dc} lambda: trials {b0}..{b0 + nb - 1} of {trials} ({n} wires each)",
                  file=sys.stderr, flush=True)
            cloud = W.ensemble(seed0 + b0, nb, n, sphere_radius, length, wavelength, dc * wavelength)
            s, info = solve_trials(cloud, inc, prec)
            sig.append(s)
            st["iterations"] = max(st["iterations"], info["iterations"])
            st["seconds"] += info["seconds"]
            st["max_rel_residual"] = max(st["max_rel_residual"], info["max_rel_residual"])
            st["converged"] &= info["converged"]
            st["nnzb"] += info["nnzb"]
        sigma = np.concatenate(sig, axis=0)
        rec = {"d_c_lambda": dc if math.isfinite(dc) else "inf", "trials": trials, "wires": n,
               **average(sigma, wavelength), "per_wire": float(sigma.mean() / wavelength ** 2 / n), **st,
               "trials_per_s": trials / st["seconds"]}
        recs.append(rec)
    dense = [r for r in recs if r["d_c_lambda"] == "inf"]
    if dense:
        ref = dense[0]["sigma_lambda2"]
        for r in recs:
            if r is not dense[0]:
                r["log10_rel_err_vs_dense"] = log_rel_error(ref, r["sigma_lambda2"])
    return recs


def e2(trials=E2_TRIALS, n=E2_WIRES, spacings=E2_SPACINGS, cutoffs=E2_CUTOFFS, batch=None, prec="c64",
       incidences=1):
    """Sec. III-B: averaged monostatic sigma_VV of half-wave chaffs against d_mean."""
    lam = W.WAVELENGTH
    for i, dm in enumerate(spacings):
        a = W.sphere_radius_for_spacing(n, dm * lam)
        for r in run_point(20000 + 1000 * i, trials, n, a, 0.5 * lam, lam, cutoffs, batch or trials, prec,
                           incidences):
            yield {"experiment": "e2", "d_mean_lambda": dm, "marcus_per_wire": 0.15, **r}


def e3(trials=E3_TRIALS, n=E3_WIRES, freqs=E3_FREQS, cutoffs=E3_CUTOFFS, batch=None, prec="c64",
       incidences=1):
    """Sec. III-C: averaged monostatic sigma_VV of 1,000 chaffs of length l1 over f / f1."""
    f1 = W.C0 / (2.0 * E3_LENGTH)
    for i, fr in enumerate(freqs):
        lam = W.C0 / (fr * f1)
        for r in run_point(30000 + 1000 * i, trials, n, E3_RADIUS, E3_LENGTH, lam, cutoffs, batch or trials,
                           prec, incidences):
            yield {"experiment": "e3", "f_over_f1": fr, "f_ghz": fr * f1 / 1e9, **r}


def e6(freqs=(1.0,), n=E6_WIRES, two_lengths=False, trials=1, prec="c64", incidences=64):
    """Sec. IV: 10^6 identical (l1) or two-length (l1, l2) chaffs, S-NFC with
    d_c = 2 lambda; one trial is averaged over ``incidences`` azimuths."""
    f1 = W.C0 / (2.0 * E6_L1)
    lengths = (E6_L1, E6_L2) if two_lengths else E6_L1
    for i, fr in enumerate(freqs):
        lam = W.C0 / (fr * f1)
        for r in run_point(60000 + 1000 * i, trials, n, E6_RADIUS, lengths, lam, (2.0,), trials, prec,
                           incidences):
            yield {"experiment": "e6", "two_lengths": bool(two_lengths), "f_over_f1": fr,
                   "f_ghz": fr * f1 / 1e9, **r}


def _floats(s):
    return tuple(math.inf if v.strip() == "inf" else float(v) for v in s.split(","))


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description="averaged monostatic RCS of random chaff ensembles")
    ap.add_argument("--experiment", choices=("e2", "e3", "e6"), default="e2")
    ap.add_argument("--trials", type=int, default=None)
    ap.add_argument("--wires", type=int, default=None)
    ap.add_argument("--points", type=_floats, default=None,
                    help="d_mean / lambda (e2) or f / f1 (e3, e6), comma-separated")
    ap.add_argument("--cutoffs", type=_floats, default=None, help="d_c / lambda, comma-separated; inf = dense")
    ap.add_argument("--batch", type=int, default=25, help="trials per launch")
    ap.add_argument("--two-lengths", action="store_true", help="e6: half of the wires of length l2")
    ap.add_argument("--prec", choices=("c64", "c128"), default="c64")
    ap.add_argument("--incidences", type=int, default=None,
                    help="V-polarised azimuth incidences per trial (default 1; e6: 64)")
    a = ap.parse_args(argv)
    kw = {"prec": a.prec}
    if a.incidences is not None:
        kw["incidences"] = a.incidences
    if a.trials is not None:
        kw["trials"] = a.trials
    if a.wires is not None:
        kw["n"] = a.wires
    if a.experiment == "e2":
        gen = e2(spacings=a.points or E2_SPACINGS, cutoffs=a.cutoffs or E2_CUTOFFS, batch=a.batch, **kw)
    elif a.experiment == "e3":
        gen = e3(freqs=a.points or E3_FREQS, cutoffs=a.cutoffs or E3_CUTOFFS, batch=a.batch, **kw)
    else:
        gen = e6(freqs=a.points or (1.0,), two_lengths=a.two_lengths, **kw)
    for rec in gen:
        print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
