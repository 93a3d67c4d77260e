"""Seeded synthetic inputs for the parabolic-mirror Stratton-Chu solves.

This module only *describes* workloads: mirror parameters, quadrature sizes,
observation grids, frequency samples and spectral amplitudes, and seeded
random draws.  It contains none of the diffraction arithmetic, so both the
CPU oracle (``oracle/``) and the HIP library (``paper_1609_08146_amd``) can
consume the same inputs without sharing any of the method's code.

Units: lengths in metres (or in wavelengths for the unit-wavelength case),
c = 1 so that the wavenumber k equals the angular frequency (Sec. II, the
Lorentz-Heaviside convention, and Sec. III-B, the Fourier convention
F(r,t) = int F(r,k) e^{-ikt} dk).  Times are c*t, in the length unit.

The paper's own workloads are parameter sets (Table I); none of them is a
public dataset.  The configurations below stand in for them:

* ``mono``      -- monochromatic, lambda = 1, f = 20, aperture 40, 200x200 nodes,
                   32x32 focal-plane grid over +-2 lambda (NA = 1).
* ``broadband`` -- 800 nm carrier, Gaussian spectrum of 10 fs intensity FWHM,
                   128 samples over +-3 sigma, f = 0.1 m, aperture radius 0.075 m,
                   w0 = 0.05 m, 400x400 nodes, 64x64 focal plane +-4 lambda0 plus
                   64 axial points, 256 time samples about the focal arrival 2f.
* ``stress``    -- f = 5 cm, aperture radius 15 cm, w0 = 7 cm, 64 samples,
                   800x800 nodes, 128x128 focal plane over +-2 lambda0.
* ``table1``    -- the Table I parameters: f = 6.75 cm, aperture 12.5 cm,
                   w0 = 10 cm, super-Gaussian power spectrum (820 nm, 70 nm,
                   order 3, 100 samples) normalised to 150 J.
* ``sweep``     -- 256 seeded instances of uneven size (batched launch).
* ``serving``   -- a seeded Poisson stream of requests drawn like ``sweep``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

C_LIGHT = 299_792_458.0          # m/s, only used to turn SI frequencies into wavenumbers
LAMBDA0 = 800e-9                 # m, carrier wavelength of the broadband workloads
TAU_FWHM = 10e-15                # s, intensity FWHM of the broadband pulse

SWEEP_SEED = 160908146
SERVING_SEED = 160908147


@dataclass
class Workload:
    """One mirror + beam + observation set.

    ``k``        wavenumbers (c = 1), shape [n_k]
    ``spectrum`` complex spectral amplitude multiplying the beam at each k, [n_k]
    ``obs``      observation points, shape [n_obs, 3]
    ``w0``       Gaussian waist of the collimated incident beam (inf = plane wave)
    ``pol``      polarisation angle about z (0 = x-polarised)
    ``consistent`` 0: E_x = G e^{-ikz}, B = -y G e^{-ikz};  1: curl-consistent pair
    ``beam``     0 linearly polarised Gaussian, 1 radially, 2 azimuthally polarised
    ``t``        time samples (c*t) for the semi-discrete transform, or None
    ``dk``       frequency spacing used as the transform weight
    """

    name: str
    f: float
    a: float
    n_r: int
    n_phi: int
    k: np.ndarray
    spectrum: np.ndarray
    obs: np.ndarray
    w0: float
    pol: float = 0.0
    consistent: int = 0
    t: Optional[np.ndarray] = None
    dk: float = 1.0
    meta: dict = field(default_factory=dict)
    beam: int = 0                 # 0 linearly, 1 radially, 2 azimuthally polarised

    @property
    def n_k(self) -> int:
        return int(self.k.shape[0])

    @property
    def n_obs(self) -> int:
        return int(self.obs.shape[0])

    @property
    def n_nodes(self) -> int:
        """Surface quadrature nodes (the rim nodes of the line integral excluded)."""
        return self.n_r * self.n_phi

    @property
    def evals(self) -> int:
        """Integrand evaluations: observation points x frequencies x surface nodes."""
        return self.n_obs * self.n_k * self.n_nodes

    def subset(self, obs_idx=None, k_idx=None, name=None) -> "Workload":
        """Same mirror and quadrature, a subset of observation points and/or frequencies."""
        obs = self.obs if obs_idx is None else self.obs[np.asarray(obs_idx)]
        k = self.k if k_idx is None else self.k[np.asarray(k_idx)]
        sp = self.spectrum if k_idx is None else self.spectrum[np.asarray(k_idx)]
        meta = dict(self.meta)
        if k_idx is not None and "eps" in meta:
            meta["eps"] = np.ascontiguousarray(meta["eps"][np.asarray(k_idx)])
        return replace(self, name=name or self.name + "-subset", obs=np.ascontiguousarray(obs),
                       k=np.ascontiguousarray(k), spectrum=np.ascontiguousarray(sp), meta=meta)

    def with_nodes(self, n_r: int, n_phi: int) -> "Workload":
        return replace(self, n_r=int(n_r), n_phi=int(n_phi))


# --------------------------------------------------------------------------- grids

def focal_plane(half_width: float, n: int, z: float = 0.0) -> np.ndarray:
    """n x n points, linspace(-h, h, n)^2 in the plane z (x fastest varying)."""
    s = np.linspace(-half_width, half_width, n)
    yy, xx = np.meshgrid(s, s, indexing="ij")
    pts = np.stack([xx.ravel(), yy.ravel(), np.full(n * n, z)], axis=-1)
    return np.ascontiguousarray(pts)


def axial_line(half_len: float, n: int) -> np.ndarray:
    """n points on the optical axis, z = linspace(-L, L, n)."""
    z = np.linspace(-half_len, half_len, n)
    return np.ascontiguousarray(np.stack([np.zeros(n), np.zeros(n), z], axis=-1))


# --------------------------------------------------------------------------- spectra

def gaussian_spectrum(n_k: int, lam0: float = LAMBDA0, tau: float = TAU_FWHM, n_sigma: float = 3.0):
    """Uniform wavenumber samples of a Gaussian pulse spectrum.

    tau is the intensity FWHM, so the spectral field amplitude is
    A(w) = exp(-(w - w0)^2 / (2 sigma_w^2)) with sigma_w = 2 sqrt(ln 2) / tau.
    Samples are uniform on w0 +- n_sigma sigma_w, end points included; n_k = 1
    gives the carrier alone.  Returns (k, amplitude, dk) with k = w / c.
    """
    k0 = 2.0 * math.pi / lam0
    sigma_k = 2.0 * math.sqrt(math.log(2.0)) / tau / C_LIGHT
    if n_k == 1:
        return np.array([k0]), np.array([1.0 + 0j]), 2.0 * n_sigma * sigma_k
    k = np.linspace(k0 - n_sigma * sigma_k, k0 + n_sigma * sigma_k, n_k)
    amp = np.exp(-((k - k0) ** 2) / (2.0 * sigma_k ** 2)).astype(np.complex128)
    return k, amp, float(k[1] - k[0])


def super_gaussian_power(n_k: int, lam_c: float, dlam: float, order: int, cut: float = 1.5):
    """Uniform wavenumber samples of a super-Gaussian power spectrum in wavelength.

    eps(lambda) = exp(-((lambda - lam_c) / dlam)^(2 order)) -- the form of
    Sec. IV-B with the minus sign of the exponent restored -- read as energy
    per unit k at lambda = 2 pi / k (unnormalised; the library scales it to the
    total energy).  Samples are uniform in k over lambda in
    [lam_c - cut dlam, lam_c + cut dlam], end points included (at cut = 1.5 and
    order 3 the edges sit at exp(-11.4) of the peak).  Returns (k, eps, dk).
    """
    k = np.linspace(2.0 * math.pi / (lam_c + cut * dlam), 2.0 * math.pi / (lam_c - cut * dlam), n_k)
    lam = 2.0 * math.pi / k
    eps = np.exp(-(((lam - lam_c) / dlam) ** (2 * order)))
    return k, eps, float(k[1] - k[0]) if n_k > 1 else 1.0


def time_window(dk: float, n_t: int, t_center: float) -> np.ndarray:
    """n_t samples t_m = t_c + (m - n_t/2) dt with dt = 2 pi / (n_t dk) (one period of the sum)."""
    dt = 2.0 * math.pi / (n_t * dk)
    return t_center + (np.arange(n_t) - n_t // 2) * dt


# --------------------------------------------------------------------------- named configs

# Table I of the paper: parabola r_max = 0.125 m, f = 0.0675 m; incident beam
# w0 = 0.100 m, lambda_c = 820 nm, delta lambda = 70 nm, super-Gaussian order
# n = 3, total energy 150 J; 100 frequency samples (Fig. 1 caption).
TABLE1 = dict(r_max=0.125, f=0.0675, w0=0.100, lam_c=820e-9, dlam=70e-9, order=3, e_tot=150.0, n_freq=100)


def table1(n_k: int = TABLE1["n_freq"], n_nodes: int = 400, n_plane: int = 64) -> Workload:
    """The Table I configuration (x-polarised literal Gaussian beam, Sec. IV-B).

    The power spectrum samples are in ``meta["eps"]`` (unnormalised) with the
    total energy ``meta["e_tot"]``; ``spectrum`` is 1, the energy
    normalisation is part of the method.  Focal plane +-2 lambda_c and 64 axial
    points over +-4 lambda_c; 256 time samples about the focal arrival 2f.
    """
    T = TABLE1
    k, eps, dk = super_gaussian_power(n_k, T["lam_c"], T["dlam"], T["order"])
    lam_c = T["lam_c"]
    obs = np.concatenate([focal_plane(2.0 * lam_c, n_plane), axial_line(4.0 * lam_c, 64)])
    return Workload(name="table1", f=T["f"], a=T["r_max"], n_r=n_nodes, n_phi=n_nodes, k=k,
                    spectrum=np.ones(n_k, np.complex128), obs=obs, w0=T["w0"],
                    t=time_window(dk, 256, 2.0 * T["f"]), dk=dk,
                    meta=dict(eps=eps, e_tot=T["e_tot"]))


def mono() -> Workload:
    """Monochromatic unit-wavelength case: lambda = 1, f = 20, aperture 40 (NA = 1)."""
    k = np.array([2.0 * math.pi])
    return Workload(name="mono", f=20.0, a=40.0, n_r=200, n_phi=200, k=k,
                    spectrum=np.array([1.0 + 0j]), obs=focal_plane(2.0, 32), w0=20.0,
                    t=None, dk=1.0)


def broadband(n_k: int = 128, n_nodes: int = 400) -> Workload:
    """800 nm / 10 fs pulse, f = 0.1 m, aperture radius 0.075 m, w0 = 0.05 m."""
    k, amp, dk = gaussian_spectrum(n_k)
    obs = np.concatenate([focal_plane(4 * LAMBDA0, 64), axial_line(4 * LAMBDA0, 64)])
    f = 0.1
    return Workload(name="broadband", f=f, a=0.075, n_r=n_nodes, n_phi=n_nodes, k=k, spectrum=amp,
                    obs=obs, w0=0.05, t=time_window(dk, 256, 2.0 * f), dk=dk)


def stress(n_k: int = 64, n_nodes: int = 800) -> Workload:
    """Precision stress: f = 5 cm, aperture radius 15 cm (rim above the focal plane), kR ~ 1.6e6 rad."""
    k, amp, dk = gaussian_spectrum(n_k)
    f = 0.05
    return Workload(name="stress", f=f, a=0.15, n_r=n_nodes, n_phi=n_nodes, k=k, spectrum=amp,
                    obs=focal_plane(2 * LAMBDA0, 128), w0=0.07, t=time_window(dk, 256, 2.0 * f), dk=dk)


def sweep_instance(rng: np.random.Generator, index: int = 0) -> Workload:
    """One instance of the batched sweep, drawn in a fixed order from ``rng``."""
    f = rng.uniform(0.02, 0.2)
    a = rng.uniform(1.0, 3.0) * f
    w0 = rng.uniform(0.3, 0.7) * a
    n_k = int(min(256, max(1, round(math.exp(rng.uniform(0.0, math.log(256.0)))))))
    n_g = int(rng.integers(16, 129))
    n_ax = int(rng.integers(16, 129))
    n = int(rng.integers(100, 601))
    k, amp, dk = gaussian_spectrum(n_k)
    obs = np.concatenate([focal_plane(4 * LAMBDA0, n_g), axial_line(4 * LAMBDA0, n_ax)])
    return Workload(name=f"sweep{index}", f=f, a=a, n_r=n, n_phi=n, k=k, spectrum=amp, obs=obs, w0=w0,
                    t=time_window(dk, 256, 2.0 * f), dk=dk)


def sweep(n_instances: int = 256, seed: int = SWEEP_SEED) -> List[Workload]:
    rng = np.random.default_rng(seed)
    return [sweep_instance(rng, i) for i in range(n_instances)]


def serving_arrivals(rate_hz: float, duration_s: float, seed: int = SERVING_SEED):
    """Poisson arrival times (s) and a generator of requests drawn like ``sweep``.

    Two independent streams are spawned from the seed: one for the inter-arrival
    gaps and one for the request parameters.
    """
    ss = np.random.SeedSequence(seed)
    s_time, s_req = ss.spawn(2)
    rt = np.random.default_rng(s_time)
    times = []
    t = 0.0
    while True:
        t += rt.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        times.append(t)
    rq = np.random.default_rng(s_req)
    return np.array(times), (lambda i: sweep_instance(rq, i))


# --------------------------------------------------------------------------- random tables

# --------------------------------------------------------------------------- general mirror surfaces
# A general surface is handed to the method as its quadrature: nodes, area-weighted
# normals n dS (pointing toward the incoming beam), and the boundary as nodes with the
# surface normal and oriented line elements dl.  These build such data for pieces of
# the paraboloid z = (x^2 + y^2)/4f - f (off-axis segments and annuli) and for an ellipsoidal
# cap, the non-parabolic surface Sec. III-C-1 discusses.

def _paraboloid_piece(f, cx, rho_lo, rho_hi, n_rho, n_psi):
    """Polar tensor grid (Gauss-Legendre in rho, trapezoid in psi) of the projected region
    cx + rho e^{i psi}, rho in [rho_lo, rho_hi], lifted onto the paraboloid."""
    xg, wg = np.polynomial.legendre.leggauss(n_rho)
    rho = rho_lo + (rho_hi - rho_lo) * (xg + 1.0) / 2.0
    wr = (rho_hi - rho_lo) * wg / 2.0
    psi = 2.0 * math.pi * np.arange(n_psi) / n_psi
    dpsi = 2.0 * math.pi / n_psi
    R, P = np.meshgrid(rho, psi, indexing="ij")
    W = (wr[:, None] * rho[:, None] * dpsi) * np.ones_like(P)
    x = cx + R * np.cos(P)
    y = R * np.sin(P)
    z = (x * x + y * y) / (4.0 * f) - f
    xyz = np.stack([x, y, z], axis=-1).reshape(-1, 3)
    n = np.stack([-x / (2.0 * f), -y / (2.0 * f), np.ones_like(x)], axis=-1).reshape(-1, 3)
    return xyz, n * W.reshape(-1, 1)


def _paraboloid_circle(f, cx, rho, n_psi, outer=True):
    """Boundary circle cx + rho e^{i psi} on the paraboloid: nodes, normals, dl (counter-clockwise
    seen from +z for an outer edge, clockwise for a hole)."""
    psi = 2.0 * math.pi * np.arange(n_psi) / n_psi
    dpsi = 2.0 * math.pi / n_psi
    c, s = np.cos(psi), np.sin(psi)
    x, y = cx + rho * c, rho * s
    z = (x * x + y * y) / (4.0 * f) - f
    n = np.stack([-x / (2.0 * f), -y / (2.0 * f), np.ones_like(x)], axis=-1)
    dx, dy = -rho * s, rho * c
    dz = (x * dx + y * dy) / (2.0 * f)
    dl = np.stack([dx, dy, dz], axis=-1) * dpsi * (1.0 if outer else -1.0)
    return np.stack([x, y, z], axis=-1), n, dl


def oap_segment(f: float, cx: float, radius: float, n_rho: int, n_psi: int):
    """Off-axis paraboloid segment whose aperture is the disk of `radius` about (cx, 0):
    (xyz, ndS, rim_xyz, rim_n, rim_dl)."""
    xyz, ndS = _paraboloid_piece(f, cx, 0.0, radius, n_rho, n_psi)
    return (xyz, ndS) + _paraboloid_circle(f, cx, radius, n_psi)


def paraboloid_annulus(f: float, a_in: float, a_out: float, n_rho: int, n_psi: int):
    """On-axis paraboloid annulus a_in <= r <= a_out with its two boundary circles."""
    xyz, ndS = _paraboloid_piece(f, 0.0, a_in, a_out, n_rho, n_psi)
    o = _paraboloid_circle(f, 0.0, a_out, n_psi, outer=True)
    i = _paraboloid_circle(f, 0.0, a_in, n_psi, outer=False)
    return (xyz, ndS) + tuple(np.concatenate([u, v]) for u, v in zip(o, i))


def ellipsoid_cap(f: float, c: float, r_max: float, n_r: int, n_phi: int):
    """Lower cap of the ellipsoid z^2/c^2 + (x^2 + y^2)/a^2 = 1 with a^2 = 2 f c (the ellipsoid
    whose vertex curvature is that of the paraboloid of focal length f, reached as c -> inf),
    shifted up by e = sqrt(c^2 - a^2) so that its lower focus lies at the origin:
        z = e - c sqrt(1 - r^2/a^2),  0 <= r <= r_max < a.
    Gauss-Legendre in r x trapezoid in phi like the built-in paraboloid, with n dS = n~ r dr dphi,
    n~ = (-z' cos phi, -z' sin phi, 1), and the rim r = r_max with dl counter-clockwise seen from
    +z.  Returns (xyz, ndS, rim_xyz, rim_n, rim_dl).  Needs c > 2f (a prolate ellipsoid)."""
    a2 = 2.0 * f * c
    if not (c * c > a2 and r_max * r_max < a2):
        raise ValueError("ellipsoid_cap needs c > 2f and r_max < sqrt(2 f c)")
    e = math.sqrt(c * c - a2)
    xg, wg = np.polynomial.legendre.leggauss(n_r)
    r = r_max * (xg + 1.0) / 2.0
    wr = r_max * wg / 2.0
    phi = 2.0 * math.pi * np.arange(n_phi) / n_phi
    dphi = 2.0 * math.pi / n_phi
    R, P = np.meshgrid(r, phi, indexing="ij")
    root = np.sqrt(1.0 - R * R / a2)
    z = e - c * root
    dz = c * R / (a2 * root)
    x, y = R * np.cos(P), R * np.sin(P)
    xyz = np.stack([x, y, z], axis=-1).reshape(-1, 3)
    n = np.stack([-dz * np.cos(P), -dz * np.sin(P), np.ones_like(R)], axis=-1).reshape(-1, 3)
    ndS = n * (wr[:, None] * R * dphi).reshape(-1, 1)
    cp, sp = np.cos(phi), np.sin(phi)
    root_m = math.sqrt(1.0 - r_max * r_max / a2)
    z_m, dz_m = e - c * root_m, c * r_max / (a2 * root_m)
    rim_xyz = np.stack([r_max * cp, r_max * sp, np.full(n_phi, z_m)], axis=-1)
    rim_n = np.stack([-dz_m * cp, -dz_m * sp, np.ones(n_phi)], axis=-1)
    rim_dl = np.stack([-r_max * sp, r_max * cp, np.zeros(n_phi)], axis=-1) * dphi
    return xyz, ndS, rim_xyz, rim_n, rim_dl


def shifted_gaussian_fields(pts, k, w0: float, cx: float, spectrum=None):
    """Literal x-polarised collimated Gaussian beam along -z centred on (cx, 0):
    E = x G e^{-ikz}, B = -y G e^{-ikz}, G = exp(-((x - cx)^2 + y^2)/w0^2); [n_k, n_pts, 3] each."""
    pts = np.asarray(pts, float).reshape(-1, 3)
    k = np.asarray(k, float).ravel()
    amp = np.ones(k.shape[0], complex) if spectrum is None else np.asarray(spectrum, complex)
    G = np.exp(-((pts[:, 0] - cx) ** 2 + pts[:, 1] ** 2) / (w0 * w0))
    ph = np.exp(-1j * np.outer(k, pts[:, 2])) * G[None, :] * amp[:, None]
    E = np.zeros((k.shape[0], pts.shape[0], 3), complex)
    B = np.zeros_like(E)
    E[:, :, 0] = ph
    B[:, :, 1] = -ph
    return E, B


def random_incident_tables(n_k: int, n_nodes_total: int, seed: int):
    """Seeded complex tables E_inc, B_inc of shape [n_k, n_nodes_total, 3] (complex128).

    Used to exercise the quadrature as a plain linear map of arbitrary tables;
    each entry is uniform in the unit complex disc's bounding square.
    """
    rng = np.random.default_rng(seed)
    shape = (n_k, n_nodes_total, 3)
    E = rng.uniform(-1, 1, shape) + 1j * rng.uniform(-1, 1, shape)
    B = rng.uniform(-1, 1, shape) + 1j * rng.uniform(-1, 1, shape)
    return np.ascontiguousarray(E), np.ascontiguousarray(B)


def random_points(n: int, half_width: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.uniform(-half_width, half_width, (n, 3)))
