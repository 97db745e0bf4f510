"""Host side of the ensemble experiments: the trial recipe and the statistics.

The mean-spacing definition is pinned to the value the paper prints for its
deterministic cloud (Sec. III-A: 1,000 chaffs in a sphere of radius 0.2 m at
15 GHz give d_mean / lambda of about 1.61); the frequency grid to the resonance
the paper reports for l1 = 11.53 mm (Sec. III-C: peaks at f1 = c / (2 l1) and
2 f1).
"""
import math

import numpy as np
import pytest

from paper_2410_03060_amd import ensemble as E
from paper_2410_03060_amd import workloads as W


def test_mean_spacing_matches_the_paper_for_its_deterministic_cloud():
    lam15 = W.C0 / 15e9
    assert W.spacing_of_sphere(1000, 0.2) / lam15 == pytest.approx(1.61, abs=0.005)


def test_sphere_radius_and_spacing_are_inverse():
    for n, dm in [(1000, 0.05), (7, 1.3), (10**6, 0.16)]:
        assert W.spacing_of_sphere(n, W.sphere_radius_for_spacing(n, dm)) == pytest.approx(dm, rel=1e-14)
    # 1,000 wires at d_mean = lambda: (4/3) pi a^3 = 1000 lambda^3
    a = W.sphere_radius_for_spacing(1000, 1.0)
    assert 4.0 / 3.0 * math.pi * a ** 3 == pytest.approx(1000.0, rel=1e-13)


def test_e3_resonance_is_13_ghz():
    f1 = W.C0 / (2 * E.E3_LENGTH)
    assert f1 / 1e9 == pytest.approx(13.01, abs=0.01)
    assert 1.0 in E.E3_FREQS and 2.0 in E.E3_FREQS


def test_trials_are_inside_their_sphere_and_reproducible():
    a, lam = 0.7, 0.1
    cl = W.ensemble(5, 4, 300, a, 0.05, lam, 2 * lam)
    assert cl.n_clouds == 4 and cl.n == 1200
    assert np.all(np.linalg.norm(cl.center, axis=1) <= a)
    assert np.allclose(np.linalg.norm(cl.tangent, axis=1), 1.0, rtol=0, atol=1e-14)
    assert np.all(cl.length == 0.05) and np.all(cl.radius == W.WIRE_RADIUS)
    assert cl.d_c == 2 * lam and cl.wavelength == lam
    # trial t does not depend on how many trials are drawn
    few = W.ensemble(5, 2, 300, a, 0.05, lam, 2 * lam)
    assert np.array_equal(few.center, cl.center[:600]) and np.array_equal(few.tangent, cl.tangent[:600])
    later = W.ensemble(7, 2, 300, a, 0.05, lam, 2 * lam)
    assert np.array_equal(later.center, cl.center[600:])
    # a uniform ball: the fraction inside half the radius is close to 1/8
    inner = np.mean(np.linalg.norm(cl.center, axis=1) <= a / 2)
    assert abs(inner - 0.125) < 0.03


def test_two_length_trials_alternate_lengths():
    cl = W.ensemble_trial(3, 10, 1.0, (E.E6_L1, E.E6_L2), 0.02, 0.04)
    assert cl.length.tolist() == [E.E6_L1, E.E6_L2] * 5


def test_average_and_relative_error():
    lam = 0.5
    sig = np.array([[1.0], [3.0], [2.0], [2.0]]) * lam ** 2
    r = E.average(sig, lam)
    assert r["sigma_lambda2"] == pytest.approx(2.0, rel=1e-15)
    assert r["sigma_db"] == pytest.approx(10 * math.log10(2.0), rel=1e-15)
    assert r["stderr_lambda2"] == pytest.approx(math.sqrt(2.0 / 3.0) / 2.0, rel=1e-14)
    assert r["samples"] == 4
    assert E.log_rel_error(100.0, 99.0) == pytest.approx(-2.0, abs=1e-12)
    assert E.log_rel_error(5.0, 5.0) == -math.inf


def test_dense_trials_reserve_every_pair():
    cl = W.concat_clouds([W.random_cloud(1, 5), W.random_cloud(2, 7)])
    assert E._max_nnzb(cl) == 25 + 49
    sparse = W.random_cloud(1, 5, d_c_lam=1.0)
    assert E._max_nnzb(sparse) is None
