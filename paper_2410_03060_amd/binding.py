"""ctypes binding of libchaff (include/chaff.h): argument marshalling only.

Every step of the hot path runs in the gfx950 kernels of libchaff.so; this
module only allocates device memory with PyTorch, passes raw pointers and the
current HIP stream, and turns status codes into exceptions.  There is no CPU
fallback: if the library is missing the import of a binding function fails.

Function names follow the C ABI: ``build_cloud``, ``fill_Z``, ``solve``,
``rcs``, ``excitation``, ``spmm``, ``destroy``, ``last_error``.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime libchaff binds to)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libchaff.so")

OK, EINVAL, EWORKSPACE, EHIP, ESINGULAR, ENOCONV = 0, -1, -2, -3, -4, -5
C64, C128 = 0, 1
NB = 7
NSEG = 8


class ChaffError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"chaff status {status}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("n_wires", C.c_int64), ("n_clouds", C.c_int32), ("n_seg", C.c_int32),
                ("wavelength", C.c_double), ("d_c", C.c_double),
                ("quad_mutual", C.c_int32), ("quad_self", C.c_int32), ("max_nnzb", C.c_int64)]


class CloudInfo(C.Structure):
    _fields_ = [("n_wires", C.c_int64), ("nnzb", C.c_int64), ("n_pairs", C.c_int64),
                ("n_clouds", C.c_int32), ("n_seg", C.c_int32),
                ("wavelength", C.c_double), ("d_c", C.c_double),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("perm", C.c_void_p),
                ("diag_pos", C.c_void_p)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("inner_tol", C.c_double), ("restart", C.c_int32),
                ("max_cycles", C.c_int32), ("use_x0", C.c_int32), ("prec", C.c_int32),
                ("spmm_variant", C.c_int32), ("method", C.c_int32), ("precond", C.c_int32),
                ("reserved", C.c_int32)]


class KernelTime(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("launches", C.c_int64), ("total_ms", C.c_double),
                ("min_ms", C.c_double), ("max_ms", C.c_double), ("bytes", C.c_double),
                ("flops", C.c_double)]


class SolveStats(C.Structure):
    _fields_ = [("cycles", C.c_int32), ("iterations", C.c_int32),
                ("max_rel_residual", C.c_double), ("seconds", C.c_double)]


_lib = None

EXPORTS = {
    "chaff_build_workspace_bytes": (C.c_size_t, [C.c_int64, C.c_int32, C.c_int64]),
    "chaff_build_cloud": (C.c_int, [C.POINTER(Params), C.POINTER(C.c_int64), C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                    C.POINTER(C.c_int64), C.c_void_p, C.POINTER(C.c_void_p)]),
    "chaff_get_info": (C.c_int, [C.c_void_p, C.POINTER(CloudInfo)]),
    "chaff_fill_Z": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "chaff_solve_workspace_bytes": (C.c_size_t, [C.c_void_p, C.POINTER(SolveOpts), C.c_int64]),
    "chaff_solve": (C.c_int, [C.c_void_p, C.POINTER(SolveOpts), C.c_void_p, C.c_void_p, C.c_void_p,
                              C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_size_t,
                              C.POINTER(SolveStats), C.c_void_p, C.c_void_p]),
    "chaff_excitation": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "chaff_spmm": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                             C.c_int32, C.c_void_p]),
    "chaff_rcs_workspace_bytes": (C.c_size_t, [C.c_void_p, C.c_int64, C.c_int64, C.c_int32]),
    "chaff_rcs": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_int64,
                            C.c_int32, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "chaff_rcs_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_int64,
                                    C.c_int32, C.c_void_p, C.c_void_p]),
    "chaff_destroy": (None, [C.c_void_p]),
    "chaff_autotune": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                 C.POINTER(C.c_int32), C.POINTER(C.c_double), C.c_void_p]),
    "chaff_tune_report": (C.c_int32, [C.c_char_p, C.c_int32]),
    "chaff_tune_save": (C.c_int, [C.c_char_p]),
    "chaff_tune_load": (C.c_int, [C.c_char_p, C.POINTER(C.c_int32)]),
    "chaff_profile_enable": (C.c_int, [C.c_int32]),
    "chaff_profile_read": (C.c_int32, [C.c_void_p, C.c_int32]),
    "chaff_mlp_features": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_int64,
                                     C.c_void_p, C.c_void_p]),
    "chaff_mlp_targets": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                    C.c_void_p, C.c_void_p, C.c_void_p]),
    "chaff_mlp_workspace_bytes": (C.c_size_t, [C.c_int64, C.c_int32]),
    "chaff_mlp_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_size_t,
                                    C.c_void_p]),
    "chaff_mlp_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "chaff_mlp_adam": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_float,
                                 C.c_float, C.c_float, C.c_float, C.c_void_p]),
    "chaff_mlp_train_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_float, C.c_float,
                                       C.c_float, C.c_float, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                       C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "chaff_mlp_guess_workspace_bytes": (C.c_size_t, [C.c_void_p, C.c_int64]),
    "chaff_mlp_guess": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_int64, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "chaff_cluster_count": (C.c_int64, [C.c_void_p]),
    "chaff_cluster_precond_bytes": (C.c_size_t, [C.c_void_p, C.c_int]),
    "chaff_cluster_precond": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "chaff_nbhd_precond_bytes": (C.c_size_t, [C.c_void_p, C.c_int, C.c_int32]),
    "chaff_nbhd_precond": (C.c_int, [C.c_void_p, C.c_int, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "chaff_nbhd_raw_rows": (C.c_int, [C.c_void_p, C.c_int, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "chaff_nbhd_mlp_features": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p]),
    "chaff_nbhd_mlp_targets": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "chaff_nbhd_mlp_workspace_bytes": (C.c_size_t, [C.c_void_p, C.c_int32]),
    "chaff_nbhd_mlp_precond": (C.c_int, [C.c_void_p, C.c_int, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_void_p, C.c_size_t, C.c_void_p]),
    "chaff_cluster_apply": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                      C.c_void_p]),
    "chaff_last_error": (C.c_char_p, []),
    "chaff_version": (C.c_char_p, []),
}


def lib():
    """Load libchaff.so (built in-tree by paper_2410_03060_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2410_03060_amd.build` (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().chaff_last_error().decode()


def _check(st: int):
    if st != OK:
        raise ChaffError(st, last_error())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _dev_f64(a, device):
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=torch.float64).contiguous()
    return torch.as_tensor(np.array(a, dtype=np.float64, order="C", copy=True), device=device)


def _2d(a):
    if isinstance(a, torch.Tensor):
        return a.reshape(-1, 3)
    return np.atleast_2d(a)


# --------------------------------------------------------------------------- handle

@dataclass
class Cloud:
    handle: C.c_void_p
    ws: torch.Tensor          # build workspace (holds the pattern; keep alive)
    n: int
    n_clouds: int
    nnzb: int
    n_pairs: int
    wavelength: float
    d_c: float
    device: torch.device
    nseg: int = NSEG

    @property
    def nb(self) -> int:
        """Rooftop unknowns per wire (n_seg - 1)."""
        return self.nseg - 1

    def info(self) -> CloudInfo:
        inf = CloudInfo()
        _check(lib().chaff_get_info(self.handle, C.byref(inf)))
        return inf

    def pattern(self):
        """(row_ptr, col_idx, perm, diag_pos) as host numpy arrays (internal order)."""
        inf = self.info()

        def grab(ptr, count, dtype):
            t = torch.empty(count, dtype=dtype, device=self.device)
            nbytes = count * t.element_size()
            if nbytes:
                _copy_ptr(t, ptr, nbytes)
            return t.cpu().numpy()

        return (grab(inf.row_ptr, self.n + 1, torch.int64), grab(inf.col_idx, self.nnzb, torch.int32),
                grab(inf.perm, self.n, torch.int32), grab(inf.diag_pos, self.n, torch.int64))

    def __del__(self):
        try:
            if self.handle:
                lib().chaff_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


def _copy_ptr(dst: torch.Tensor, src_ptr: int, nbytes: int):
    """Device-to-device copy from a raw library pointer into a tensor (HIP runtime)."""
    hip = _hip()
    st = torch.cuda.current_stream().cuda_stream
    rc = hip.hipMemcpyAsync(C.c_void_p(dst.data_ptr()), C.c_void_p(src_ptr), C.c_size_t(nbytes),
                            C.c_int(3), C.c_void_p(st))
    if rc != 0:
        raise RuntimeError(f"hipMemcpyAsync failed ({rc})")


_hiprt = None


def _hip():
    global _hiprt
    if _hiprt is None:
        _hiprt = C.CDLL("libamdhip64.so.7", mode=C.RTLD_GLOBAL)
        _hiprt.hipMemcpyAsync.restype = C.c_int
        _hiprt.hipMemcpyAsync.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p]
    return _hiprt


@dataclass
class DeviceGeometry:
    """Wire geometry already resident in device memory (float64 tensors)."""
    center: torch.Tensor
    tangent: torch.Tensor
    length: torch.Tensor
    radius: torch.Tensor
    cloud_off: np.ndarray
    wavelength: float
    d_c: float
    n_seg: int = NSEG

    @property
    def n(self) -> int:
        return int(self.center.shape[0])

    @property
    def n_clouds(self) -> int:
        return int(len(self.cloud_off) - 1)


def upload(cloud, device="cuda") -> DeviceGeometry:
    device = torch.device(device)
    return DeviceGeometry(_dev_f64(cloud.center, device), _dev_f64(cloud.tangent, device),
                          _dev_f64(cloud.length, device), _dev_f64(cloud.radius, device),
                          np.asarray(cloud.cloud_off, dtype=np.int64), float(cloud.wavelength),
                          float(cloud.d_c), int(getattr(cloud, "n_seg", NSEG)))


def build_cloud(cloud, device="cuda", max_nnzb: int | None = None, quad_mutual: int = 4,
                quad_self: int = 8) -> Cloud:
    """Neighbour search and internal layout for a (multi-)cloud (chaff_build_cloud).

    ``cloud`` is a host workload (numpy arrays, uploaded here) or a
    DeviceGeometry already in device memory.  Its ``n_seg`` (8, or 20 for the
    paper's 19 unknowns per wire) sets the discretisation.
    """
    if not isinstance(cloud, DeviceGeometry):
        cloud = upload(cloud, device)
    device = cloud.center.device
    n = cloud.n
    nc = cloud.n_clouds
    c, t, L, a = cloud.center, cloud.tangent, cloud.length, cloud.radius
    off = (C.c_int64 * (nc + 1))(*[int(v) for v in cloud.cloud_off])
    if max_nnzb is None:
        max_nnzb = n * n if not math.isfinite(cloud.d_c) else min(n * n, 24 * n + 64)
    for _ in range(2):
        p = Params(n, nc, int(cloud.n_seg), float(cloud.wavelength), float(cloud.d_c), quad_mutual, quad_self,
                   int(max_nnzb))
        need = lib().chaff_build_workspace_bytes(n, nc, int(max_nnzb))
        if need == 0:
            raise ChaffError(EINVAL, "bad sizes for the build workspace")
        ws = torch.empty(need, dtype=torch.uint8, device=device)
        nnzb = C.c_int64(0)
        h = C.c_void_p()
        st = lib().chaff_build_cloud(C.byref(p), off, _ptr(c), _ptr(t), _ptr(L), _ptr(a), _ptr(ws),
                                     need, C.byref(nnzb), _stream(), C.byref(h))
        if st == EWORKSPACE and nnzb.value > max_nnzb:
            max_nnzb = int(nnzb.value)
            continue
        _check(st)
        out = Cloud(h, ws, n, nc, int(nnzb.value), 0, float(cloud.wavelength), float(cloud.d_c), device,
                    int(cloud.n_seg))
        out.n_pairs = int(out.info().n_pairs)
        return out
    raise ChaffError(EWORKSPACE, last_error())


def fill_Z(cl: Cloud, prec: int = C64, with_pinv: bool = True):
    """Impedance blocks [nnzb,nb,nb] and inverse self blocks [N,nb,nb] (chaff_fill_Z)."""
    dt = torch.complex64 if prec == C64 else torch.complex128
    Z = torch.empty((cl.nnzb, cl.nb, cl.nb), dtype=dt, device=cl.device)
    P = torch.empty((cl.n, cl.nb, cl.nb), dtype=dt, device=cl.device) if with_pinv else None
    _check(lib().chaff_fill_Z(cl.handle, prec, _ptr(Z), _ptr(P), _stream()))
    return Z, P


GMRES, COCG, COCG_RR, GCR = 0, 1, 2, 3
PRECOND_BLOCK, PRECOND_CLUSTER, PRECOND_NBHD = 0, 1, 2
CLUSTER_WIRES, CLUSTER_ROWS = 8, 56
NBHD_MAX, NBHD_HEADER = 8, 256


def solve_opts(tol=1e-6, inner_tol=1e-4, restart=30, max_cycles=50, use_x0=0, prec=C64,
               spmm_variant=-1, method=GMRES, precond=PRECOND_BLOCK) -> SolveOpts:
    return SolveOpts(tol, inner_tol, restart, max_cycles, int(use_x0), prec, spmm_variant, method,
                     int(precond), 0)


def cluster_count(cl: Cloud) -> int:
    return int(lib().chaff_cluster_count(cl.handle))


def cluster_precond(cl: Cloud, Z, prec: int = C64):
    """Cluster block-Jacobi preconditioner buffer (chaff_cluster_precond): uint8 [bytes]."""
    nbytes = lib().chaff_cluster_precond_bytes(cl.handle, prec)
    if nbytes == 0:
        raise ChaffError(EINVAL, last_error() or "bad cluster preconditioner arguments")
    M = torch.empty(nbytes, dtype=torch.uint8, device=cl.device)
    _check(lib().chaff_cluster_precond(cl.handle, prec, _ptr(Z), _ptr(M), _stream()))
    return M


def cluster_table(cl: Cloud, M):
    """[n_clusters, 2] int32 view (first internal wire, wires) of a preconditioner buffer."""
    n = cluster_count(cl)
    return M[:n * 8].view(torch.int32).view(n, 2)


def cluster_blocks(cl: Cloud, M, prec: int = C64):
    """[n_clusters, 56, 56] complex view of the inverse blocks of a preconditioner buffer."""
    n = cluster_count(cl)
    off = (n * 8 + 255) // 256 * 256
    dt = torch.complex64 if prec == C64 else torch.complex128
    esz = 8 if prec == C64 else 16
    return M[off:off + n * CLUSTER_ROWS * CLUSTER_ROWS * esz].view(dt).view(n, CLUSTER_ROWS, CLUSTER_ROWS)


def nbhd_precond(cl: Cloud, Z, size: int, prec: int = C64):
    """Neighbourhood-inverse preconditioner buffer (chaff_nbhd_precond): uint8 [bytes]."""
    nbytes = lib().chaff_nbhd_precond_bytes(cl.handle, prec, int(size))
    if nbytes == 0:
        raise ChaffError(EINVAL, last_error() or "bad neighbourhood preconditioner arguments")
    M = torch.empty(nbytes, dtype=torch.uint8, device=cl.device)
    _check(lib().chaff_nbhd_precond(cl.handle, prec, int(size), _ptr(Z), _ptr(M), _stream()))
    return M


def nbhd_raw_rows(cl: Cloud, Z, size: int, prec: int = C64):
    """Unsymmetrised neighbourhood rows (chaff_nbhd_raw_rows): uint8 buffer, the targets' source."""
    nbytes = lib().chaff_nbhd_precond_bytes(cl.handle, prec, int(size))
    if nbytes == 0:
        raise ChaffError(EINVAL, last_error() or "bad neighbourhood preconditioner arguments")
    M = torch.empty(nbytes, dtype=torch.uint8, device=cl.device)
    _check(lib().chaff_nbhd_raw_rows(cl.handle, prec, int(size), _ptr(Z), _ptr(M), _stream()))
    return M


def nbhd_mlp_features(cl: Cloud, M, size: int, row0: int = 0, n_rows: int | None = None):
    """BF16 features [rows, 192] (int16 bit patterns) of the samples (wire, slot, column) of M."""
    total = cl.n * size * 7
    n_rows = total - row0 if n_rows is None else n_rows
    F = torch.empty((n_rows, MLP_NFEAT), dtype=torch.int16, device=cl.device)
    _check(lib().chaff_nbhd_mlp_features(cl.handle, _ptr(M), row0, n_rows, _ptr(F), _stream()))
    return F


def nbhd_mlp_targets(cl: Cloud, M_raw, Pinv, size: int, prec: int = C64):
    """FP32 targets [N*size*7, 14] from a raw-rows buffer and the inverse self blocks of fill_Z."""
    Y = torch.empty((cl.n * size * 7, MLP_NOUT), dtype=torch.float32, device=cl.device)
    _check(lib().chaff_nbhd_mlp_targets(cl.handle, prec, _ptr(M_raw), _ptr(Pinv), _ptr(Y), _stream()))
    return Y


def nbhd_mlp_precond(cl: Cloud, theta, Pinv, size: int, prec: int = C64):
    """The learned neighbourhood-inverse preconditioner (chaff_nbhd_mlp_precond): a PRECOND_NBHD buffer."""
    nbytes = lib().chaff_nbhd_precond_bytes(cl.handle, prec, int(size))
    wsb = lib().chaff_nbhd_mlp_workspace_bytes(cl.handle, int(size))
    if nbytes == 0 or wsb == 0:
        raise ChaffError(EINVAL, last_error() or "bad learned preconditioner arguments")
    M = torch.empty(nbytes, dtype=torch.uint8, device=cl.device)
    ws = torch.empty(wsb, dtype=torch.uint8, device=cl.device)
    _check(lib().chaff_nbhd_mlp_precond(cl.handle, prec, int(size), _ptr(theta), _ptr(Pinv), _ptr(M), _ptr(ws),
                                        wsb, _stream()))
    return M


def nbhd_table(cl: Cloud, M, size: int):
    """[N, size] int32 view of the neighbourhoods (internal indices, -1 unused) of a buffer."""
    return M[NBHD_HEADER:NBHD_HEADER + cl.n * size * 4].view(torch.int32).view(cl.n, size)


def nbhd_blocks(cl: Cloud, M, size: int, prec: int = C64):
    """[nnzb, 7, 7] complex view of the preconditioner's blocks (Z's block order)."""
    off = NBHD_HEADER + (cl.n * size * 4 + 255) // 256 * 256
    dt = torch.complex64 if prec == C64 else torch.complex128
    esz = 8 if prec == C64 else 16
    return M[off:off + cl.nnzb * cl.nb * cl.nb * esz].view(dt).view(cl.nnzb, cl.nb, cl.nb)


def cluster_apply(cl: Cloud, M, X, prec: int = C64, Y=None):
    """Y = M X on the internal order (chaff_cluster_apply); X is [N*7, s]."""
    if Y is None:
        Y = torch.empty_like(X)
    _check(lib().chaff_cluster_apply(cl.handle, prec, _ptr(M), _ptr(X), _ptr(Y), X.shape[1], _stream()))
    return Y


def solve(cl: Cloud, Z, Pinv, k_hat, e_hat, opts: SolveOpts | None = None, x0=None,
          raise_on_noconv: bool = True):
    """Excitation + preconditioned restarted GMRES (+ FP64 refinement) (chaff_solve).

    Returns (X [N*7, R] complex128 in caller wire order, stats dict).
    """
    opts = opts or solve_opts()
    kh = _dev_f64(_2d(k_hat), cl.device)
    eh = _dev_f64(_2d(e_hat), cl.device)
    R = kh.shape[0]
    if x0 is not None:
        X = x0.to(device=cl.device, dtype=torch.complex128).contiguous().clone()
        opts.use_x0 = 1
    else:
        X = torch.empty((cl.n * cl.nb, R), dtype=torch.complex128, device=cl.device)
    need = lib().chaff_solve_workspace_bytes(cl.handle, C.byref(opts), R)
    if need == 0:
        raise ChaffError(EINVAL, last_error() or "bad solve options")
    ws = torch.empty(need, dtype=torch.uint8, device=cl.device)
    stats = SolveStats()
    rel = np.zeros(cl.n_clouds * R, dtype=np.float64)
    st = lib().chaff_solve(cl.handle, C.byref(opts), _ptr(Z), _ptr(Pinv), _ptr(kh), _ptr(eh), R,
                           _ptr(X), _ptr(ws), need, C.byref(stats),
                           rel.ctypes.data_as(C.c_void_p), _stream())
    info = {"cycles": stats.cycles, "iterations": stats.iterations,
            "max_rel_residual": stats.max_rel_residual, "seconds": stats.seconds,
            "rel_res": rel.reshape(cl.n_clouds, R), "status": st}
    if st != OK and not (st == ENOCONV and not raise_on_noconv):
        _check(st)
    return X, info


def excitation(cl: Cloud, k_hat, e_hat):
    kh = _dev_f64(_2d(k_hat), cl.device)
    eh = _dev_f64(_2d(e_hat), cl.device)
    U = torch.empty((cl.n * cl.nb, kh.shape[0]), dtype=torch.complex128, device=cl.device)
    _check(lib().chaff_excitation(cl.handle, _ptr(kh), _ptr(eh), kh.shape[0], _ptr(U), _stream()))
    return U


def spmm(cl: Cloud, Z, X, prec: int = C64, variant: int = -1, Y=None):
    """Y = Z X on the internal order (chaff_spmm); X is [N*nb, s]."""
    if Y is None:
        Y = torch.empty_like(X)
    _check(lib().chaff_spmm(cl.handle, prec, _ptr(Z), _ptr(X), _ptr(Y), X.shape[1], variant, _stream()))
    return Y


def rcs(cl: Cloud, X, obs_dir, obs_pol, monostatic: bool):
    """sigma per cloud (chaff_rcs): [n_clouds, R] monostatic or [n_clouds, R, M] bistatic."""
    d = _dev_f64(_2d(obs_dir), cl.device)
    p = _dev_f64(_2d(obs_pol), cl.device)
    R = X.shape[1]
    M = d.shape[0]
    need = lib().chaff_rcs_workspace_bytes(cl.handle, R, M, int(monostatic))
    ws = torch.empty(need, dtype=torch.uint8, device=cl.device)
    shape = (cl.n_clouds, R) if monostatic else (cl.n_clouds, R, M)
    sig = torch.empty(shape, dtype=torch.float64, device=cl.device)
    _check(lib().chaff_rcs(cl.handle, _ptr(X), R, _ptr(d), _ptr(p), M, int(monostatic), _ptr(sig),
                           _ptr(ws), need, _stream()))
    return sig


def rcs_noalloc(cl: Cloud, X, obs_dir, obs_pol, monostatic: bool):
    """sigma per cloud through chaff_rcs_noalloc (no workspace; the library's fixed scratch)."""
    d = _dev_f64(_2d(obs_dir), cl.device)
    p = _dev_f64(_2d(obs_pol), cl.device)
    R = X.shape[1]
    M = d.shape[0]
    shape = (cl.n_clouds, R) if monostatic else (cl.n_clouds, R, M)
    sig = torch.empty(shape, dtype=torch.float64, device=cl.device)
    _check(lib().chaff_rcs_noalloc(cl.handle, _ptr(X), R, _ptr(d), _ptr(p), M, int(monostatic), _ptr(sig),
                                   _stream()))
    return sig


def autotune(cl: Cloud, Z, s: int, prec: int = C64):
    """Time every product variant for this cloud and RHS count; later variant -1 calls use the best."""
    dt = torch.complex64 if prec == C64 else torch.complex128
    X = torch.ones((cl.n * cl.nb, s), dtype=dt, device=cl.device)
    Y = torch.empty_like(X)
    best = C.c_int32(-1)
    ms = C.c_double(0.0)
    _check(lib().chaff_autotune(cl.handle, prec, _ptr(Z), _ptr(X), _ptr(Y), s, C.byref(best), C.byref(ms),
                                _stream()))
    return int(best.value), float(ms.value)


def tune_report() -> list:
    import json
    n = lib().chaff_tune_report(None, 0)
    buf = C.create_string_buffer(n)
    lib().chaff_tune_report(buf, n)
    return json.loads(buf.value.decode())


def tune_save(path: str):
    """Write the product-variant tuning table to a JSON file (chaff_tune_save)."""
    _check(lib().chaff_tune_save(os.fsencode(path)))


def tune_load(path: str) -> int:
    """Merge a tuning table written by tune_save into this process's table (chaff_tune_load)."""
    n = C.c_int32(0)
    _check(lib().chaff_tune_load(os.fsencode(path), C.byref(n)))
    return int(n.value)


def destroy(cl: Cloud):
    if cl.handle:
        lib().chaff_destroy(cl.handle)
        cl.handle = None


def profile_enable(on: bool):
    _check(lib().chaff_profile_enable(1 if on else 0))


def profile_read() -> dict:
    """{kernel: dict(launches, total_ms, min_ms, max_ms, bytes, flops)} of the tracked launches
    (bytes / flops: algorithmic HBM bytes and flops summed over launches, 0 where not stated)."""
    buf = (KernelTime * 64)()
    n = lib().chaff_profile_read(C.cast(buf, C.c_void_p), 64)
    return {buf[i].name.decode(): dict(launches=int(buf[i].launches), total_ms=buf[i].total_ms,
                                       min_ms=buf[i].min_ms, max_ms=buf[i].max_ms, bytes=buf[i].bytes,
                                       flops=buf[i].flops)
            for i in range(n)}


# ------------------------------------------------------------------ learned initial guess

MLP_NFEAT, MLP_HIDDEN, MLP_NOUT, MLP_NPARAM = 192, 128, 14, 59534


def mlp_features(cl: Cloud, k_hat, e_hat, row0: int = 0, n_rows: int | None = None):
    """BF16 feature bit patterns [n_rows, 192] (int16) of rows row0.. (row = p*R + r)."""
    kh = _dev_f64(_2d(k_hat), cl.device)
    eh = _dev_f64(_2d(e_hat), cl.device)
    R = kh.shape[0]
    if n_rows is None:
        n_rows = cl.n * R - row0
    feat = torch.empty((max(n_rows, 1), MLP_NFEAT), dtype=torch.int16, device=cl.device)
    _check(lib().chaff_mlp_features(cl.handle, _ptr(kh), _ptr(eh), R, row0, n_rows, _ptr(feat), _stream()))
    return feat[:n_rows]


def mlp_targets(cl: Cloud, Pinv, k_hat, e_hat, X, prec: int = C64):
    """Network targets [N*R, 14] float32 from currents X [N*7, R] complex128 (caller order)."""
    kh = _dev_f64(_2d(k_hat), cl.device)
    eh = _dev_f64(_2d(e_hat), cl.device)
    R = kh.shape[0]
    X = X.to(device=cl.device, dtype=torch.complex128).contiguous()
    Y = torch.empty((cl.n * R, MLP_NOUT), dtype=torch.float32, device=cl.device)
    _check(lib().chaff_mlp_targets(cl.handle, prec, _ptr(Pinv), _ptr(kh), _ptr(eh), R, _ptr(X), _ptr(Y),
                                   _stream()))
    return Y


def mlp_forward(theta, feat):
    """Network outputs [rows, 14] float32 of BF16 features [rows, 192] (int16 bit patterns)."""
    rows = feat.shape[0]
    need = lib().chaff_mlp_workspace_bytes(rows, 0)
    ws = torch.empty(need, dtype=torch.uint8, device=feat.device)
    Y = torch.empty((rows, MLP_NOUT), dtype=torch.float32, device=feat.device)
    _check(lib().chaff_mlp_forward(_ptr(theta), _ptr(feat), rows, _ptr(Y), _ptr(ws), need, _stream()))
    return Y


def mlp_grad(theta, feat, T, idx=None, n_rows: int | None = None):
    """(gradient [59534] float32, loss [1] float32) over rows idx (or all rows)."""
    rows = n_rows if n_rows is not None else (idx.shape[0] if idx is not None else feat.shape[0])
    need = lib().chaff_mlp_workspace_bytes(rows, 1)
    ws = torch.empty(need, dtype=torch.uint8, device=feat.device)
    g = torch.empty(MLP_NPARAM, dtype=torch.float32, device=feat.device)
    loss = torch.empty(1, dtype=torch.float32, device=feat.device)
    _check(lib().chaff_mlp_grad(_ptr(theta), _ptr(feat), _ptr(T), _ptr(idx), rows, _ptr(g), _ptr(loss),
                                _ptr(ws), need, _stream()))
    return g, loss


def mlp_adam(theta, m, v, grad, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One in-place Adam step on theta, m, v."""
    _check(lib().chaff_mlp_adam(_ptr(theta), _ptr(m), _ptr(v), _ptr(grad), t, lr, beta1, beta2, eps, _stream()))


class MlpTrainer:
    """FP32 master parameters, Adam moments and the training workspace for one batch size."""

    def __init__(self, theta0, batch: int, device="cuda", beta1=0.9, beta2=0.999, eps=1e-8):
        self.theta = torch.as_tensor(np.asarray(theta0, dtype=np.float32), device=device).contiguous()
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.t = 0
        self.batch = batch
        self.betas = (beta1, beta2)
        self.eps = eps
        self.need = lib().chaff_mlp_workspace_bytes(batch, 1)
        self.ws = torch.empty(self.need, dtype=torch.uint8, device=device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)

    def step(self, feat, T, idx, lr: float):
        """One Adam step on the rows idx [<= batch] (int64, device) of feat / T; loss stays on the device."""
        rows = idx.shape[0]
        if rows > self.batch:
            raise ValueError("more rows than the trainer's batch size")
        self.t += 1
        _check(lib().chaff_mlp_train_step(_ptr(self.theta), _ptr(self.m), _ptr(self.v), self.t, lr,
                                          self.betas[0], self.betas[1], self.eps, _ptr(feat), _ptr(T),
                                          _ptr(idx), rows, _ptr(self.loss), _ptr(self.ws), self.need,
                                          _stream()))
        return self.loss


def mlp_guess(cl: Cloud, Pinv, theta, k_hat, e_hat, prec: int = C64):
    """Initial currents X [N*7, R] complex128 (caller order): isolated response + network correction."""
    kh = _dev_f64(_2d(k_hat), cl.device)
    eh = _dev_f64(_2d(e_hat), cl.device)
    R = kh.shape[0]
    need = lib().chaff_mlp_guess_workspace_bytes(cl.handle, R)
    ws = torch.empty(need, dtype=torch.uint8, device=cl.device)
    X = torch.empty((cl.n * NB, R), dtype=torch.complex128, device=cl.device)
    _check(lib().chaff_mlp_guess(cl.handle, prec, _ptr(Pinv), _ptr(theta), _ptr(kh), _ptr(eh), R, _ptr(X),
                                 _ptr(ws), need, _stream()))
    return X


def version() -> str:
    return lib().chaff_version().decode()
