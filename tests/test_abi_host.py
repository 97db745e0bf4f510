"""Host-side checks of the C ABI: symbols, argument validation, workspace sizing.

None of these launch a kernel: validation happens on the host before any HIP
call, so they run on machines without a GPU.
"""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chaff.h")


@pytest.fixture(scope="module")
def B():
    from paper_2410_03060_amd import binding
    try:
        binding.lib()
    except ImportError as e:  # the build step has not run
        pytest.skip(str(e))
    return binding


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(chaff_[A-Za-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("chaff_build_cloud", "chaff_fill_Z", "chaff_solve", "chaff_rcs", "chaff_destroy",
                 "chaff_last_error"):
        assert want in names


def test_library_exports_every_declared_symbol(B):
    L = B.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert set(B.EXPORTS) == set(declared_functions())


def _params(B, **kw):
    p = dict(n_wires=10, n_clouds=1, n_seg=8, wavelength=0.1, d_c=0.2, quad_mutual=4, quad_self=8,
             max_nnzb=100)
    p.update(kw)
    return B.Params(**p)


def _build(B, p, off=None, ws_bytes=1 << 30, geom=True):
    n = p.n_wires
    if off is None:
        off = [0, max(n, 0)]
    arr = (C.c_int64 * len(off))(*off)
    fake = C.c_void_p(0x1000) if geom else None   # never dereferenced: validation fails first
    nn = C.c_int64(0)
    h = C.c_void_p()
    st = B.lib().chaff_build_cloud(C.byref(p), arr, fake, fake, fake, fake, C.c_void_p(0x1000),
                                   ws_bytes, C.byref(nn), None, C.byref(h))
    return st, B.last_error(), nn.value


@pytest.mark.parametrize("kw,msg", [
    (dict(n_wires=0), "n_wires"),
    (dict(n_clouds=0), "n_clouds"),
    (dict(n_seg=12), "n_seg"),
    (dict(n_seg=7), "n_seg"),
    (dict(wavelength=0.0), "wavelength"),
    (dict(wavelength=float("nan")), "wavelength"),
    (dict(d_c=-1.0), "d_c"),
    (dict(d_c=float("nan")), "d_c"),
    (dict(quad_mutual=0), "quad_mutual"),
    (dict(quad_mutual=9), "quad_mutual"),
    (dict(quad_self=1), "quad_self"),
    (dict(max_nnzb=5), "max_nnzb"),
])
def test_build_rejects_bad_params(B, kw, msg):
    p = _params(B, **kw)
    off = [0, max(p.n_wires, 0)] if p.n_clouds == 1 else [0] * (max(p.n_clouds, 0) + 1)
    st, err, _ = _build(B, p, off)
    assert st == B.EINVAL
    assert msg in err


def test_build_rejects_bad_cloud_offsets(B):
    p = _params(B, n_clouds=2)
    for off, msg in (([1, 5, 10], "cloud_off[0]"), ([0, 6, 5], "non-decreasing"), ([0, 4, 9], "n_wires")):
        st, err, _ = _build(B, p, off)
        assert st == B.EINVAL and msg in err


def test_build_rejects_null_geometry_and_small_workspace(B):
    st, err, _ = _build(B, _params(B), geom=False)
    assert st == B.EINVAL and "geometry" in err
    st, err, _ = _build(B, _params(B), ws_bytes=16)
    assert st == B.EWORKSPACE and "workspace" in err


def test_build_workspace_grows_with_size(B):
    L = B.lib()
    a = L.chaff_build_workspace_bytes(1000, 1, 24000)
    b = L.chaff_build_workspace_bytes(2000, 1, 48000)
    c = L.chaff_build_workspace_bytes(2000, 1, 96000)
    assert 0 < a < b < c
    assert L.chaff_build_workspace_bytes(0, 1, 10) == 0
    assert L.chaff_build_workspace_bytes(10, 1, 5) == 0
    # the pattern itself: 4 bytes per block index at least
    assert c - b >= 4 * 48000


def test_calls_on_null_handle_fail_cleanly(B):
    L = B.lib()
    assert L.chaff_fill_Z(None, B.C64, C.c_void_p(0x1000), None, None) == B.EINVAL
    o = B.solve_opts()
    assert L.chaff_solve(None, C.byref(o), None, None, None, None, 1, None, None, 0, None, None,
                         None) == B.EINVAL
    assert L.chaff_rcs(None, None, 1, None, None, 1, 1, None, None, 0, None) == B.EINVAL
    assert L.chaff_spmm(None, B.C64, None, None, None, 1, -1, None) == B.EINVAL
    assert L.chaff_solve_workspace_bytes(None, C.byref(o), 1) == 0
    L.chaff_destroy(None)   # no-op


def test_version_string(B):
    assert B.version().startswith("chaff-gfx950")


def test_mlp_entry_points_validate_before_any_launch(B):
    L = B.lib()
    P = C.c_void_p(0x1000)          # never dereferenced: every call below fails validation
    a = L.chaff_mlp_workspace_bytes(1000, 1)
    b = L.chaff_mlp_workspace_bytes(100000, 1)
    f = L.chaff_mlp_workspace_bytes(100000, 0)
    assert 0 < a < b and 0 < f < b
    assert L.chaff_mlp_workspace_bytes(0, 1) == 0
    # Adam: bad step / hyper-parameters
    assert L.chaff_mlp_adam(P, P, P, P, 0, 1e-3, 0.9, 0.999, 1e-8, None) == B.EINVAL
    assert "step" in B.last_error()
    assert L.chaff_mlp_adam(P, P, P, P, 1, 1e-3, 1.0, 0.999, 1e-8, None) == B.EINVAL
    assert L.chaff_mlp_adam(None, P, P, P, 1, 1e-3, 0.9, 0.999, 1e-8, None) == B.EINVAL
    # misaligned features, too small a workspace, empty batch
    assert L.chaff_mlp_forward(P, C.c_void_p(0x1002), 10, P, P, 1 << 30, None) == B.EINVAL
    assert "aligned" in B.last_error()
    assert L.chaff_mlp_forward(P, P, 10, P, P, 16, None) == B.EWORKSPACE
    assert L.chaff_mlp_grad(P, P, P, None, 0, P, None, P, 1 << 30, None) == B.EINVAL
    assert L.chaff_mlp_train_step(P, P, P, 1, 1e-3, 0.9, 0.999, 1e-8, P, P, None, 100, None, P, 16,
                                  None) == B.EWORKSPACE
    # cloud-based calls need a handle
    assert L.chaff_mlp_features(None, P, P, 1, 0, 1, P, None) == B.EINVAL
    assert L.chaff_mlp_targets(None, B.C64, P, P, P, 1, P, P, None) == B.EINVAL
    assert L.chaff_mlp_guess(None, B.C64, P, P, P, P, 1, P, P, 1 << 30, None) == B.EINVAL
    assert L.chaff_mlp_guess_workspace_bytes(None, 1) == 0


def test_solve_rejects_bad_initial_guess_mode(B):
    L = B.lib()
    o = B.solve_opts(use_x0=3)
    assert L.chaff_solve_workspace_bytes(C.c_void_p(0x1000), C.byref(o), 1) == 0
    assert "use_x0" in B.last_error()


def test_solve_rejects_bad_preconditioner_and_reserved_field(B):
    L = B.lib()
    o = B.solve_opts(precond=3)
    assert L.chaff_solve_workspace_bytes(C.c_void_p(0x1000), C.byref(o), 1) == 0
    assert "precond" in B.last_error()
    o = B.solve_opts()
    o.reserved = 1
    assert L.chaff_solve_workspace_bytes(C.c_void_p(0x1000), C.byref(o), 1) == 0
    assert "reserved" in B.last_error()


def test_solve_rejects_unknown_method_and_long_gcr_cycles(B):
    L = B.lib()
    o = B.solve_opts(method=4)
    assert L.chaff_solve_workspace_bytes(C.c_void_p(0x1000), C.byref(o), 1) == 0
    assert "method" in B.last_error()
    o = B.solve_opts(method=B.GCR, restart=201)
    assert L.chaff_solve_workspace_bytes(C.c_void_p(0x1000), C.byref(o), 1) == 0
    assert "restart" in B.last_error()


def test_cluster_entry_points_validate_before_any_launch(B):
    L = B.lib()
    H = C.c_void_p(0x1000)          # never dereferenced: every call below fails validation
    P = C.c_void_p(0x1000)
    assert L.chaff_cluster_count(None) == -1
    assert L.chaff_cluster_precond_bytes(None, B.C64) == 0
    assert L.chaff_cluster_precond(None, B.C64, P, P, None) == B.EINVAL
    assert L.chaff_cluster_precond(H, 7, P, P, None) == B.EINVAL
    assert L.chaff_cluster_precond(H, B.C64, P, C.c_void_p(0x1010), None) == B.EINVAL
    assert "aligned" in B.last_error()
    assert L.chaff_cluster_apply(H, B.C64, P, P, P, 0, None) == B.EINVAL
    assert L.chaff_cluster_apply(H, B.C64, None, P, P, 1, None) == B.EINVAL


def test_tuning_table_round_trip_through_json(B, tmp_path):
    """chaff_tune_load merges a JSON table; chaff_tune_save writes it back with the same entries."""
    import json
    src = tmp_path / "tune_in.json"
    rows = [{"nb": 7, "n": 1000, "nnzb": 5000, "s": 8, "prec": 0, "best": 6,
             "ms": [0.5, 0.4, 0.45, 0.41, 0.43, 0.6, 0.3, 0.31]},
            {"nb": 19, "n": 500, "nnzb": 520, "s": 1, "prec": 1, "best": 0,
             "ms": [0.1, 0.2, 0.2, 0.2, 0.2, 0.3, 0.0, 0.0]}]
    src.write_text(json.dumps(rows))
    assert B.tune_load(str(src)) == 2
    table = {(e["nb"], e["n"], e["nnzb"], e["s"], e["prec"]): e for e in B.tune_report()}
    for r in rows:
        e = table[(r["nb"], r["n"], r["nnzb"], r["s"], r["prec"])]
        assert e["best"] == r["best"] and np.allclose(e["ms"], r["ms"])
    out = tmp_path / "tune_out.json"
    B.tune_save(str(out))
    back = {(e["nb"], e["n"], e["nnzb"], e["s"], e["prec"]): e["best"] for e in json.loads(out.read_text())}
    assert back[(7, 1000, 5000, 8, 0)] == 6 and back[(19, 500, 520, 1, 1)] == 0


def test_tuning_table_rejects_other_files(B, tmp_path):
    bad = tmp_path / "bad.json"
    bad.write_text('[{"nb": 7, "n": 10}]')
    with pytest.raises(B.ChaffError) as ei:
        B.tune_load(str(bad))
    assert ei.value.status == B.EINVAL
    with pytest.raises(B.ChaffError):
        B.tune_load(str(tmp_path / "missing.json"))


def test_nbhd_entry_points_validate_before_any_launch(B):
    L = B.lib()
    H = C.c_void_p(0x1000)          # never dereferenced: every call below fails validation
    P = C.c_void_p(0x1000)
    assert L.chaff_nbhd_precond_bytes(None, B.C64, 4) == 0
    assert L.chaff_nbhd_precond_bytes(H, B.C64, 0) == 0
    assert L.chaff_nbhd_precond_bytes(H, B.C64, 9) == 0
    assert L.chaff_nbhd_precond(None, B.C64, 4, P, P, None) == B.EINVAL
    assert L.chaff_nbhd_precond(H, 7, 4, P, P, None) == B.EINVAL
    assert L.chaff_nbhd_precond(H, B.C64, 0, P, P, None) == B.EINVAL
    assert "size" in B.last_error()
    assert L.chaff_nbhd_precond(H, B.C64, 9, P, P, None) == B.EINVAL
    assert L.chaff_nbhd_precond(H, B.C64, 4, P, C.c_void_p(0x1010), None) == B.EINVAL
    assert "aligned" in B.last_error()
