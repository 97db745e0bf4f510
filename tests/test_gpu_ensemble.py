"""GPU parity of the ensemble driver (averaged monostatic RCS, Sec. III-B, III-C).

Every trial of a multi-cloud batch is checked against the oracle solving that
trial alone: S-NFC (sparse direct solve of the oracle's S-NFC matrix) and
entire coupling (dense solve of the oracle's full matrix), monostatic sigma_VV
of the V-polarised incidence.  The bars: 1e-4 dB for complex64 with FP64
refinement to a 1e-6 residual, 1e-6 dB for complex128 to 1e-10.  The
driver's averages and its log10 relative error against entire coupling
(Sec. III-C) are then recomputed from the oracle's per-trial values.
"""
import math

import numpy as np
import pytest

from oracle import mom, solve
from paper_2410_03060_amd import ensemble as E
from paper_2410_03060_amd import workloads as W
from parity_util import say

pytestmark = pytest.mark.gpu

LAM = W.WAVELENGTH


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_03060_amd import binding
    binding.lib()
    return binding


def _oracle_sigma(seed0, trials, n, a, length, lam, d_c, inc):
    out = []
    for t in range(trials):
        tr = W.ensemble_trial(seed0 + t, n, a, length, lam, d_c)
        u = mom.excitation(tr, inc.k_hat, inc.e_hat)
        if math.isfinite(d_c):
            x = solve.sparse_solve(mom.snfc_matrix(tr)[0], u)
        else:
            x = solve.dense_solve(mom.dense_Z(tr), u)
        out.append(mom.monostatic_rcs(tr, x, inc.k_hat, inc.e_hat))
    return np.array(out)


@pytest.mark.parametrize("prec,tol,bar_db", [("c64", 1e-6, 1e-4), ("c128", 1e-10, 1e-6)])
@pytest.mark.parametrize("dc_lam", [1.0, math.inf])
def test_ensemble_sigma_per_trial_matches_the_oracle(B, prec, tol, bar_db, dc_lam):
    n, trials, seed0 = 40, 3, 11
    a = W.sphere_radius_for_spacing(n, 0.5 * LAM)
    inc = W.azimuth_incidences(3)          # sigma [trials, incidences]
    say(f"[ensemble] {trials} trials x {n} half-wave wires, 3 incidences, d_mean 0.5 lambda, "
        f"d_c {dc_lam} lambda, {prec}")
    cloud = W.ensemble(seed0, trials, n, a, 0.5 * LAM, LAM, dc_lam * LAM)
    sig, st = E.solve_trials(cloud, inc, prec, tol=tol)
    assert st["converged"] and st["max_rel_residual"] <= tol
    so = _oracle_sigma(seed0, trials, n, a, 0.5 * LAM, LAM, dc_lam * LAM, inc)
    assert sig.shape == so.shape == (trials, 3)
    db = np.abs(10 * np.log10(sig / so))
    say(f"  iterations {st['iterations']}, sigma error max {db.max():.2e} dB")
    assert db.max() <= bar_db


def test_run_point_averages_and_relative_error(B):
    """Two cutoffs on the same trials, split over two launches (batch of 2 of 3
    trials): the averages and the relative error against entire coupling are
    those of the oracle's per-trial values."""
    n, trials, seed0 = 30, 3, 50
    a = W.sphere_radius_for_spacing(n, 0.4 * LAM)
    recs = E.run_point(seed0, trials, n, a, 0.5 * LAM, LAM, (1.0, math.inf), batch=2)
    assert [r["d_c_lambda"] for r in recs] == [1.0, "inf"]
    inc = W.v_incidence()
    ref = {dc: _oracle_sigma(seed0, trials, n, a, 0.5 * LAM, LAM, dc * LAM, inc) for dc in (1.0, math.inf)}
    for r, dc in zip(recs, (1.0, math.inf)):
        mean = float(ref[dc].mean() / LAM ** 2)
        assert r["sigma_lambda2"] == pytest.approx(mean, rel=5e-5)
        assert r["samples"] == trials and r["converged"]
    want = E.log_rel_error(float(ref[math.inf].mean()), float(ref[1.0].mean()))
    say(f"  d_c = lambda against entire coupling: log10 rel err {recs[0]['log10_rel_err_vs_dense']:.3f} "
        f"(oracle {want:.3f})")
    assert recs[0]["log10_rel_err_vs_dense"] == pytest.approx(want, abs=0.01)
    assert "log10_rel_err_vs_dense" not in recs[1]


def _orientation_average(L, lam, n_ct=16, n_phi=32):
    """The oracle's orientation-averaged monostatic sigma / lambda^2 of one wire
    (Gauss rule in cos theta, midpoint rule in phi; V-polarised incidence)."""
    kh = np.array([[-1.0, 0.0, 0.0]])
    e = np.array([[0.0, 0.0, -1.0]])
    one = W.single_cloud(np.zeros((1, 3)), np.array([[0.0, 0.0, 1.0]]), np.array([L]), lam)
    Zd = mom.dense_Z(one)                      # the matrix of one wire does not depend on its direction
    ct, wt = np.polynomial.legendre.leggauss(n_ct)
    acc = 0.0
    for c, w in zip(ct, wt):
        s = math.sqrt(1.0 - c * c)
        for ph in (np.arange(n_phi) + 0.5) * 2.0 * math.pi / n_phi:
            cl = W.single_cloud(np.zeros((1, 3)), np.array([[s * math.cos(ph), s * math.sin(ph), c]]),
                                np.array([L]), lam)
            x = solve.dense_solve(Zd, mom.excitation(cl, kh, e))
            acc += w / 2.0 / n_phi * mom.monostatic_rcs(cl, x, kh, e)[0]
    return acc / lam ** 2


def test_sparse_ensemble_tends_to_the_isolated_wire_average(B):
    """d_mean = 20 lambda: the trial-averaged sigma of 1,000 half-wave wires is
    N times the oracle's orientation-averaged sigma of one wire, within three
    standard errors of the 100-trial mean (incoherent limit of Sec. III-B)."""
    n, trials = 1000, 100
    a = W.sphere_radius_for_spacing(n, 20.0 * LAM)
    rec = E.run_point(20005, trials, n, a, 0.5 * LAM, LAM, (2.0,), batch=50)[0]
    single = _orientation_average(0.5 * LAM, LAM)
    say(f"  per wire {rec['per_wire']:.4f} +- {rec['stderr_lambda2'] / n:.4f}, isolated wire {single:.4f}")
    assert rec["converged"]
    assert abs(rec["per_wire"] - single) <= 3.0 * rec["stderr_lambda2"] / n


def test_snfc_matches_entire_coupling_over_frequency(B):
    """Sec. III-C: 1,000 chaffs of length l1 in a 10 m sphere; S-NFC with
    d_c = 2 lambda and entire coupling on the same 20 trials agree to
    log10 relative error below -2 at f1 and 2 f1, and the average peaks there
    (above its value at 1.5 f1)."""
    recs = {r["f_over_f1"]: r for r in E.e3(trials=20, freqs=(1.0, 1.5, 2.0), batch=20) if r["d_c_lambda"] == 2.0}
    for fr in (1.0, 2.0):
        say(f"  f/f1 {fr}: sigma {recs[fr]['sigma_lambda2']:.2f} lambda^2, "
            f"log10 rel err {recs[fr]['log10_rel_err_vs_dense']:.2f}")
        assert recs[fr]["converged"] and recs[fr]["log10_rel_err_vs_dense"] < -2.0
        assert recs[fr]["sigma_lambda2"] > 2.0 * recs[1.5]["sigma_lambda2"]
