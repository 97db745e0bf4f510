"""chaff_rcs_noalloc (far field without a workspace) against chaff_rcs.

The no-allocation entry point runs the same kernels on the library's fixed
per-GPU scratch array, so its sigma must equal chaff_rcs's exactly, on two
calls in a row (the second with a smaller cloud and fewer incidences, the
scratch keeping the first call's contents), monostatic and bistatic; a request
larger than the fixed scratch is refused on the host.
"""
import numpy as np
import pytest

from paper_2410_03060_amd import workloads as W
from parity_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_03060_amd import binding
    binding.lib()
    return binding


def _case(B, n, R, seed):
    wl = W.c2(n=n, seed=seed)
    inc = W.azimuth_incidences(R)
    cl = B.build_cloud(wl.cloud)
    Z, P = B.fill_Z(cl, B.C64)
    X, info = B.solve(cl, Z, P, inc.k_hat, inc.e_hat, B.solve_opts(tol=1e-6))
    return cl, X, inc


def test_rcs_noalloc_equals_rcs_on_two_calls(B):
    for n, R, seed in ((900, 12, 2), (250, 3, 5)):
        say(f"[rcs_noalloc] N={n} R={R} seed={seed}")
        cl, X, inc = _case(B, n, R, seed)
        s_ref = B.rcs(cl, X, -inc.k_hat, inc.e_hat, monostatic=True).cpu().numpy()
        s_new = B.rcs_noalloc(cl, X, -inc.k_hat, inc.e_hat, monostatic=True).cpu().numpy()
        assert np.array_equal(s_ref, s_new), (s_ref, s_new)
        T, Pp, rh, th, ph = W.bistatic_grid(10.0)
        b_ref = B.rcs(cl, X, rh, th, monostatic=False).cpu().numpy()
        b_new = B.rcs_noalloc(cl, X, rh, th, monostatic=False).cpu().numpy()
        assert np.array_equal(b_ref, b_new)
        say(f"  monostatic and {rh.shape[0]}-direction bistatic sigma identical")


def test_rcs_noalloc_refuses_more_than_its_scratch(B):
    cl, X, inc = _case(B, 300, 4, 7)
    M = 600_000   # 2 chunks x 4 RHS x M x 16 B > 64 MiB
    rng = np.random.default_rng(0)
    d = rng.standard_normal((M, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    e = np.cross(d, np.array([0.0, 0.0, 1.0]))
    e /= np.linalg.norm(e, axis=1, keepdims=True)
    with pytest.raises(B.ChaffError) as ei:
        B.rcs_noalloc(cl, X, d, e, monostatic=False)
    assert ei.value.status == -2 and "exceeds the fixed" in str(ei.value)
