"""Seeded synthetic chaff-cloud workloads.

This module only draws random geometry and incidence directions; it holds
none of the method's arithmetic.  Both the FP64 oracle (through the tests and
the golden-value script) and the GPU path take their inputs from here, so the
two sides always see identical arrays.

The paper's workloads (Sec. III and IV) are random clouds of thin wires with
uniformly random orientation, uniform or Gaussian spatial distribution and one
or several lengths.  The paper uses no public dataset.  The five workloads
below follow that recipe at the sizes the hot path is measured on:

* ``c1``  64 half-wave wires uniform in a 10-wavelength cube (448 unknowns);
* ``c2``  2,000 wires, Gaussian positions (sigma 15 wavelengths), lengths
  uniform in [0.4, 0.6] wavelengths (14,000 unknowns), d_c = 1.5 wavelengths;
* ``c3``  20,000 wires, Gaussian (sigma 40 wavelengths), plus 16 side clouds
  of 500-5,000 wires, 360 azimuth incidences, d_c = 2 wavelengths;
* ``c4``  the learned-guess set: 200 training clouds of 2,000-10,000 wires and
  a 100,000-wire uniform-sphere evaluation cloud (radius 40 wavelengths);
* ``c5``  1,000,000 wires uniform in a sphere of radius 50 wavelengths,
  d_c = 1 wavelength, 64 azimuth incidences.

The statistical ensembles (``ensemble``) draw many independent trials of
identical or two-length wires uniform in a sphere whose radius follows from
the mean spacing d_mean (volume per wire d_mean^3), with a physical wire
radius of 10 micrometres.

Random draws are made with ``numpy.random.default_rng(seed)`` in a fixed
order: positions, then orientations, then lengths, then angles.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

WAVELENGTH = 0.1          # metres (3 GHz with c0 = 3e8 m/s; lambda is the definition)
RADIUS_FRAC = 1e-4        # wire radius in wavelengths
N_SEG = 8                 # segments per wire -> 7 rooftop unknowns


@dataclass
class Cloud:
    """Wires of one or more independent clouds, concatenated.

    ``cloud_off[c]:cloud_off[c+1]`` are the wires of cloud ``c``; pairs never
    cross clouds.  All lengths in metres.
    """
    center: np.ndarray            # [N,3] float64
    tangent: np.ndarray           # [N,3] float64, unit
    length: np.ndarray            # [N]   float64
    radius: np.ndarray            # [N]   float64
    cloud_off: np.ndarray         # [C+1] int64
    wavelength: float = WAVELENGTH
    d_c: float = math.inf
    n_seg: int = N_SEG            # segments per wire (n_seg - 1 rooftop unknowns)

    @property
    def n(self) -> int:
        return int(self.center.shape[0])

    @property
    def n_clouds(self) -> int:
        return int(self.cloud_off.shape[0] - 1)


@dataclass
class Incidence:
    """Plane-wave incidences (one per right-hand side).

    ``k_hat`` is the propagation direction (unit), ``e_hat`` the unit
    polarisation, orthogonal to it.  A wave "incident from d" has k_hat = -d.
    Monostatic observation of RHS r uses direction -k_hat[r] and the same
    polarisation.
    """
    k_hat: np.ndarray             # [R,3] float64
    e_hat: np.ndarray             # [R,3] float64


@dataclass
class Workload:
    name: str
    cloud: Cloud
    inc: Incidence
    notes: dict = field(default_factory=dict)


# --------------------------------------------------------------------------- draws

def _isotropic(rng: np.random.Generator, n: int) -> np.ndarray:
    g = rng.standard_normal((n, 3))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def _uniform_ball(rng: np.random.Generator, n: int, radius: float) -> np.ndarray:
    d = _isotropic(rng, n)
    r = radius * rng.random(n) ** (1.0 / 3.0)
    return d * r[:, None]


def single_cloud(center, tangent, length, wavelength=WAVELENGTH, d_c=math.inf,
                 radius=None, n_seg: int = N_SEG) -> Cloud:
    center = np.ascontiguousarray(center, dtype=np.float64).reshape(-1, 3)
    tangent = np.ascontiguousarray(tangent, dtype=np.float64).reshape(-1, 3)
    length = np.ascontiguousarray(length, dtype=np.float64).reshape(-1)
    n = center.shape[0]
    if radius is None:
        radius = np.full(n, RADIUS_FRAC * wavelength)
    radius = np.ascontiguousarray(np.broadcast_to(radius, (n,)), dtype=np.float64)
    return Cloud(center, tangent, length, radius,
                 np.array([0, n], dtype=np.int64), wavelength, d_c, n_seg)


def concat_clouds(clouds: list[Cloud]) -> Cloud:
    off = [0]
    for c in clouds:
        off.append(off[-1] + c.n)
    lam = clouds[0].wavelength
    dc = clouds[0].d_c
    ns = clouds[0].n_seg
    assert all(c.wavelength == lam and c.d_c == dc and c.n_seg == ns for c in clouds)
    return Cloud(np.concatenate([c.center for c in clouds]),
                 np.concatenate([c.tangent for c in clouds]),
                 np.concatenate([c.length for c in clouds]),
                 np.concatenate([c.radius for c in clouds]),
                 np.array(off, dtype=np.int64), lam, dc, ns)


def theta_hat(theta: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """Spherical unit vector theta-hat at (theta, phi) (radians)."""
    return np.stack([np.cos(theta) * np.cos(phi), np.cos(theta) * np.sin(phi),
                     -np.sin(theta)], axis=-1)


def phi_hat(theta: np.ndarray, phi: np.ndarray) -> np.ndarray:
    return np.stack([-np.sin(phi), np.cos(phi), np.zeros_like(phi)], axis=-1)


def r_hat(theta: np.ndarray, phi: np.ndarray) -> np.ndarray:
    return np.stack([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi),
                     np.cos(theta)], axis=-1)


def incidence_from_z() -> Incidence:
    """Theta-polarised wave arriving from +z: k_hat = -z, e_hat = theta-hat(0,0) = +x."""
    return Incidence(np.array([[0.0, 0.0, -1.0]]), np.array([[1.0, 0.0, 0.0]]))


def azimuth_incidences(n_angles: int, step_deg: float | None = None) -> Incidence:
    """V-polarised (theta-hat = -z) waves arriving from azimuth phi_i in the xy-plane.

    phi_i = i * step (default 360/n degrees); arriving from d = (cos phi, sin phi, 0)
    means k_hat = -d.
    """
    step = 360.0 / n_angles if step_deg is None else step_deg
    phi = np.deg2rad(np.arange(n_angles) * step)
    d = np.stack([np.cos(phi), np.sin(phi), np.zeros_like(phi)], axis=1)
    e = np.tile(np.array([0.0, 0.0, -1.0]), (n_angles, 1))
    return Incidence(-d, e)


def random_incidences(rng: np.random.Generator, n: int) -> Incidence:
    """Isotropic arrival directions with polarisation uniform in the transverse plane."""
    d = _isotropic(rng, n)
    k = -d
    # orthonormal transverse frame from theta/phi-hat of d
    th = np.arccos(np.clip(d[:, 2], -1.0, 1.0))
    ph = np.arctan2(d[:, 1], d[:, 0])
    psi = rng.random(n) * 2.0 * np.pi
    e = np.cos(psi)[:, None] * theta_hat(th, ph) + np.sin(psi)[:, None] * phi_hat(th, ph)
    return Incidence(k, e)


def bistatic_grid(step_deg: float = 1.0):
    """Full sphere grid theta = 0..180, phi = 0..359 (1 degree: 181 x 360 = 65,160).

    Returns (theta, phi, r_hat, theta_hat, phi_hat), each flattened theta-major.
    """
    th = np.deg2rad(np.arange(0.0, 180.0 + 1e-9, step_deg))
    ph = np.deg2rad(np.arange(0.0, 360.0 - 1e-9, step_deg))
    T, P = np.meshgrid(th, ph, indexing="ij")
    T = T.ravel()
    P = P.ravel()
    return T, P, r_hat(T, P), theta_hat(T, P), phi_hat(T, P)


# --------------------------------------------------------------------------- configs

def c1(seed: int = 1, d_c: float = 2.0) -> Workload:
    """64 half-wave wires uniform in a 10-wavelength cube; one wave from +z."""
    lam = WAVELENGTH
    rng = np.random.default_rng(seed)
    n = 64
    c = rng.uniform(-5.0 * lam, 5.0 * lam, (n, 3))
    t = _isotropic(rng, n)
    L = np.full(n, 0.5 * lam)
    return Workload("c1", single_cloud(c, t, L, lam, d_c * lam), incidence_from_z(),
                    {"d_c_over_lambda": d_c})


def c2(seed: int = 2, n: int = 2000) -> Workload:
    """2,000 wires, Gaussian sigma 15 wavelengths, L ~ U[0.4,0.6] wavelengths, d_c 1.5."""
    lam = WAVELENGTH
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((n, 3)) * 15.0 * lam
    t = _isotropic(rng, n)
    L = rng.uniform(0.4 * lam, 0.6 * lam, n)
    return Workload("c2", single_cloud(c, t, L, lam, 1.5 * lam), incidence_from_z())


def _gauss_cloud(seed: int, n: int, sigma_lam: float, d_c_lam: float) -> Cloud:
    lam = WAVELENGTH
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((n, 3)) * sigma_lam * lam
    t = _isotropic(rng, n)
    L = rng.uniform(0.4 * lam, 0.6 * lam, n)
    return single_cloud(c, t, L, lam, d_c_lam * lam)


def c3(n_main: int = 20000, n_side: int = 16, n_angles: int = 360) -> Workload:
    """Main Gaussian cloud (sigma 40 wavelengths) plus uneven side clouds, 360 azimuths."""
    clouds = [_gauss_cloud(3, n_main, 40.0, 2.0)]
    sizes = []
    for j in range(n_side):
        rng = np.random.default_rng(300 + j)
        nj = int(rng.integers(500, 5001))
        sizes.append(nj)
        sig = 40.0 * (nj / 20000.0) ** (1.0 / 3.0)
        clouds.append(_gauss_cloud(300 + j + 1000, nj, sig, 2.0))
    return Workload("c3", concat_clouds(clouds), azimuth_incidences(n_angles),
                    {"side_sizes": sizes})


def _sphere_cloud(seed: int, n: int, radius_lam: float, d_c_lam: float) -> Cloud:
    lam = WAVELENGTH
    rng = np.random.default_rng(seed)
    c = _uniform_ball(rng, n, radius_lam * lam)
    t = _isotropic(rng, n)
    L = rng.uniform(0.4 * lam, 0.6 * lam, n)
    return single_cloud(c, t, L, lam, d_c_lam * lam)


def c4_train_cloud(j: int) -> Workload:
    """Training cloud j (0..199): N ~ U{2000..10000}, uniform sphere at the eval density."""
    rng = np.random.default_rng(4000 + j)
    n = int(rng.integers(2000, 10001))
    radius = 40.0 * (n / 1e5) ** (1.0 / 3.0)
    cloud = _sphere_cloud(40000 + j, n, radius, 1.5)
    inc = random_incidences(np.random.default_rng(41000 + j), 8)
    return Workload(f"c4_train_{j}", cloud, inc)


def c4_eval(n: int = 100000) -> Workload:
    cloud = _sphere_cloud(4999, n, 40.0 * (n / 1e5) ** (1.0 / 3.0), 1.5)
    inc = random_incidences(np.random.default_rng(49990), 8)
    return Workload("c4_eval", cloud, inc)


def c5_train_cloud(j: int) -> Workload:
    """Training cloud j for the learned guess at the 10^6-wire cloud's density
    (1.91 wires per cubic wavelength) and d_c = 1 wavelength: N ~ U{5000..20000},
    uniform sphere of radius 50 lambda (N/10^6)^(1/3), 8 random incidences."""
    rng = np.random.default_rng(5000 + j)
    n = int(rng.integers(5000, 20001))
    cloud = _sphere_cloud(50000 + j, n, 50.0 * (n / 1e6) ** (1.0 / 3.0), 1.0)
    inc = random_incidences(np.random.default_rng(51000 + j), 8)
    return Workload(f"c5_train_{j}", cloud, inc)


def c5(n: int = 1_000_000, n_angles: int = 64) -> Workload:
    """10^6 wires uniform in a sphere of radius 50 wavelengths, d_c = 1 wavelength."""
    radius = 50.0 * (n / 1e6) ** (1.0 / 3.0)
    return Workload("c5", _sphere_cloud(5, n, radius, 1.0),
                    azimuth_incidences(n_angles, 360.0 / n_angles))


def random_cloud(seed: int, n: int, box_lam: float = 4.0, d_c_lam: float = math.inf,
                 L_lo: float = 0.4, L_hi: float = 0.6, n_seg: int = N_SEG) -> Cloud:
    """Small helper for tests: n wires uniform in a cube of side box_lam wavelengths."""
    lam = WAVELENGTH
    rng = np.random.default_rng(seed)
    c = rng.uniform(-0.5 * box_lam * lam, 0.5 * box_lam * lam, (n, 3))
    t = _isotropic(rng, n)
    L = rng.uniform(L_lo * lam, L_hi * lam, n)
    return single_cloud(c, t, L, lam, d_c_lam * lam, n_seg=n_seg)


# --------------------------------------------------------------------------- the paper's discretisation

# Sec. IV (computational statistics): clouds of 10^2 .. 10^6 chaffs uniform in a
# sphere at 119.37 chaffs per cubic metre, 13 GHz, chaff diameter 20 um and 19
# rooftop unknowns per chaff (Sec. II-A).  The chaff length is not printed
# there; the half-wave length at 13 GHz (c/(2 f), the 11.53 mm chaffs of
# Sec. III-C) is used, and d_c = 2 wavelengths, the paper's default.
PAPER_DENSITY = 119.37        # chaffs per m^3
PAPER_FREQ = 13.0e9           # Hz
PAPER_NSEG = 20               # N_v = 19 unknowns per chaff


def paper_cloud(n: int = 100_000, seed: int = 7, d_c_lam: float = 2.0) -> Cloud:
    """n identical half-wave chaffs (13 GHz) uniform in the sphere of the paper's density."""
    lam = C0 / PAPER_FREQ
    a = (3.0 * n / (4.0 * math.pi * PAPER_DENSITY)) ** (1.0 / 3.0)
    rng = np.random.default_rng(seed)
    c = _uniform_ball(rng, n, a)
    t = _isotropic(rng, n)
    L = np.full(n, C0 / (2.0 * PAPER_FREQ))
    return single_cloud(c, t, L, lam, d_c_lam * lam, np.full(n, WIRE_RADIUS), PAPER_NSEG)


def n2(n: int = 100_000, n_angles: int = 64) -> Workload:
    """The paper's 10^5-chaff, 2-million-unknown case with its N_v = 19 discretisation,
    64 V-polarised azimuth incidences (5.625 degree step)."""
    return Workload("n2", paper_cloud(n), azimuth_incidences(n_angles, 360.0 / n_angles))


CONFIGS = {"c1": c1, "c2": c2, "c3": c3, "c4_eval": c4_eval, "c5": c5, "n2": n2}


# --------------------------------------------------------------------------- ensembles

# Speed of light used to turn frequencies into wavelengths in the ensemble
# recipes (the paper quotes frequencies in GHz and lengths in metres).
C0 = 3.0e8
# Physical wire radius of the ensembles: D = 20 micrometres (Sec. II).
WIRE_RADIUS = 10e-6


def sphere_radius_for_spacing(n: int, d_mean: float) -> float:
    """Radius of the sphere whose volume per wire is d_mean^3: (4/3) pi a^3 = n d_mean^3."""
    return d_mean * (3.0 * n / (4.0 * math.pi)) ** (1.0 / 3.0)


def spacing_of_sphere(n: int, a: float) -> float:
    """Mean spacing d_mean = (V / n)^(1/3) of n wires in a sphere of radius a."""
    return (4.0 * math.pi * a ** 3 / (3.0 * n)) ** (1.0 / 3.0)


def ensemble_trial(seed: int, n: int, sphere_radius: float, length, wavelength: float,
                   d_c: float, wire_radius: float = WIRE_RADIUS) -> Cloud:
    """One trial of a statistical ensemble (Sec. III-B, III-C, IV): n wires
    uniform in a sphere, isotropic orientations.  ``length`` is one length for
    every wire or a sequence of lengths that the wires take in turn (wire i
    gets length[i % len(length)])."""
    rng = np.random.default_rng(seed)
    c = _uniform_ball(rng, n, sphere_radius)
    t = _isotropic(rng, n)
    lens = np.atleast_1d(np.asarray(length, dtype=np.float64))
    L = lens[np.arange(n) % lens.size]
    return single_cloud(c, t, L, wavelength, d_c, np.full(n, wire_radius))


def ensemble(seed0: int, trials: int, n: int, sphere_radius: float, length, wavelength: float,
             d_c: float, wire_radius: float = WIRE_RADIUS) -> Cloud:
    """``trials`` independent trials as the clouds of one multi-cloud input;
    trial t is ``ensemble_trial(seed0 + t, ...)`` whatever the trial count."""
    return concat_clouds([ensemble_trial(seed0 + t, n, sphere_radius, length, wavelength, d_c, wire_radius)
                          for t in range(trials)])


def v_incidence() -> Incidence:
    """The ensembles' single incidence: V-polarised (theta-hat = -z) wave
    arriving from +x along the xy-plane."""
    return azimuth_incidences(1)


# --------------------------------------------------------------------------- learned guess

MLP_LAYERS = ((192, 128), (128, 128), (128, 128), (128, 14))   # (inputs, outputs) per layer


def mlp_init(seed: int) -> np.ndarray:
    """Initial network parameters, flat float64: per layer W [n_in][n_out]
    (Glorot-uniform draw), then b [n_out] (zeros)."""
    rng = np.random.default_rng(seed)
    parts = []
    for n_in, n_out in MLP_LAYERS:
        lim = math.sqrt(6.0 / (n_in + n_out))
        parts.append(rng.uniform(-lim, lim, n_in * n_out))
        parts.append(np.zeros(n_out))
    return np.concatenate(parts)


def shuffle_order(seed: int, n: int) -> np.ndarray:
    """A seeded permutation of n training rows (int64)."""
    return np.random.default_rng(seed).permutation(n).astype(np.int64)
