"""Pins of the oracle with the paper's own discretisation (Sec. II-A: 20
segments, 19 rooftop unknowns per chaff, chaff diameter 20 um).

The oracle's functions take the segment count as a parameter; these pins tie
the 20-segment evaluation to facts outside the oracle: the textbook resonant
half-wave dipole, exact Galerkin symmetry, reciprocity of the far field, and
the refinement limit of the 8-segment model.
"""
import json
import math
import os

import numpy as np

from oracle import mom, solve
from paper_2410_03060_amd import workloads as W

NS = 20
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_claims.json")


def _mono(cloud, k_hat, e_hat, n_seg):
    x = solve.dense_solve(mom.dense_Z(cloud, n_seg=n_seg), mom.excitation(cloud, k_hat, e_hat, n_seg))
    return mom.monostatic_rcs(cloud, x, k_hat, e_hat, n_seg)


def test_resonant_halfwave_chaff_at_13_ghz():
    """One 20-um-diameter chaff at 13 GHz, broadside, polarisation along it: the
    backscatter peaks near 0.86 lambda^2 (half-wave dipole) slightly below L = lambda/2."""
    with open(GOLDEN) as f:
        ref = json.load(f)["halfwave_dipole_peak_monostatic_rcs_lambda2"]["value"]
    lam = W.C0 / W.PAPER_FREQ
    kh = np.array([[1.0, 0.0, 0.0]])
    e = np.array([[0.0, 0.0, 1.0]])
    Ls = np.arange(0.42, 0.5201, 0.005)
    sig = np.array([_mono(W.single_cloud([[0, 0, 0]], [[0, 0, 1.0]], [L * lam], lam, math.inf, [W.WIRE_RADIUS], NS),
                          kh, e, NS)[0] / lam ** 2 for L in Ls])
    i = int(np.argmax(sig))
    assert abs(10 * math.log10(sig[i] / ref)) < 0.5
    assert 0.45 <= Ls[i] <= 0.50


def test_galerkin_symmetry_and_reciprocity_20_segments():
    cl = W.random_cloud(21, 5, box_lam=1.2, n_seg=NS)
    Z = mom.dense_Z(cl, n_seg=NS)
    assert Z.shape == (5 * 19, 5 * 19)
    assert np.abs(Z - Z.T).max() <= 1e-13 * np.abs(Z).max()
    inc = W.random_incidences(np.random.default_rng(4), 2)
    ki, ei = inc.k_hat[:1], inc.e_hat[:1]
    rs, es = -inc.k_hat[1:], inc.e_hat[1:]
    S1 = (mom.farfield_weights(cl, rs, es, NS).T @ solve.dense_solve(Z, mom.excitation(cl, ki, ei, NS)))[0, 0]
    S2 = (mom.farfield_weights(cl, -ki, ei, NS).T @ solve.dense_solve(Z, mom.excitation(cl, -rs, es, NS)))[0, 0]
    assert abs(S1 - S2) <= 1e-10 * abs(S1)


def test_twenty_segments_sit_between_eight_and_the_refined_limit():
    """Segment refinement of one coupled pair: the 20-segment monostatic RCS is closer to
    the 64-segment value than the 8-segment one is."""
    cl8 = W.random_cloud(22, 2, box_lam=0.8)
    kh = np.array([[0.3, -0.8, 0.52]])
    kh /= np.linalg.norm(kh)
    e = np.cross(kh, [[0.0, 0.0, 1.0]])
    e /= np.linalg.norm(e)
    s = {}
    for ns in (8, 20, 64):
        cl = W.single_cloud(cl8.center, cl8.tangent, cl8.length, cl8.wavelength, math.inf, cl8.radius, ns)
        s[ns] = _mono(cl, kh, e, ns)[0]
    assert abs(s[20] - s[64]) < abs(s[8] - s[64])
