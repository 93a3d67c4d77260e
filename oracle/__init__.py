"""CPU oracle for the physical-optics Stratton-Chu mirror integrals.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product library.  It wraps the plain
C implementation in ``sc_oracle.c`` (FP64, long-double phase) with numpy
arrays.  Every function follows the paper directly:

* ``gauss_legendre``          -- quadrature rule of Sec. III-C (Gauss-Legendre in r)
* ``mirror``                  -- paraboloid z = r^2/4f - f, cylindrical nodes (Sec. III-A/C)
* ``incident``/``incident_tables`` -- collimated beam along -z on the mirror (Sec. III-A)
* ``incident_lg``/``incident_lg_tables`` -- Laguerre-Gauss mode sets, the expansion basis of Sec. III-A
* ``reflected_field``         -- Stokes-converted POA integrals (Sec. II, eq. stratton-chu-poa-og)
* ``reflected_field_dgrad``   -- double-gradient POA form (Sec. II, eq. stratton-chu-poa), cross-check
* ``time_transform``          -- semi-discrete Fourier sum (Sec. III-B, eq. impl.semiDiscreteFFT)

Parity pins for all of these live in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None

PLANE, GAUSSIAN, GAUSSIAN_CONSISTENT = 0, 1, 2
RADIAL, RADIAL_CONSISTENT, AZIMUTHAL, AZIMUTHAL_CONSISTENT = 3, 4, 5, 6
PARABOLOID, FLAT = 0, 1


def compile_source(src: str, out: str) -> str:
    """Compile an oracle C source with gcc (OpenMP, -O2, no fast-math) into a shared library."""
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11",
                           "-o", tmp, src, "-lquadmath", "-lm"])
    os.replace(tmp, out)
    return out


def build(force: bool = False) -> str:
    """Build oracle/_build/liboracle.so (rebuilt when the source is newer)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        compile_source(_SRC, _LIB_PATH)
    return _LIB_PATH


def open_library(path: str):
    """Load an oracle build (the default one, or a test's deliberately broken copy)."""
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER(ctypes.c_double)
    I, D = ctypes.c_int, ctypes.c_double
    lib.orc_gauss_legendre.argtypes = [I, P, P]
    lib.orc_mirror.argtypes = [I, D, D, I, I, P, P, P, P]
    lib.orc_incident.argtypes = [I, I, P, D, D, D, D, D, P, P]
    lib.orc_incident_lg.argtypes = [I, ctypes.POINTER(ctypes.c_int), P, D, I, P, D, D, D, P, P]
    lib.orc_reflected_field.argtypes = [I, I, P, P, P, P, I, P, P, P, I, P, P, P, I, I]
    lib.orc_reflected_field_dgrad.argtypes = [I, P, P, P, I, I, P, P, I, P, P, I]
    lib.orc_time_transform.argtypes = [I, P, D, I, P, ctypes.c_long, P, P, I]
    lib.orc_incident_power.argtypes = [I, I, I, P, P, P, P, P]
    lib.orc_max_threads.restype = I
    return lib


_override = None


class use_library:
    """Context manager: route every oracle call through another build (mutation tests)."""

    def __init__(self, path: str):
        self.lib = open_library(path)

    def __enter__(self):
        global _override
        self._prev = _override
        _override = self.lib
        return self

    def __exit__(self, *exc):
        global _override
        _override = self._prev
        return False


def _load():
    global _lib
    if _override is not None:
        return _override
    if _lib is None:
        _lib = open_library(build())
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    if a.dtype == np.complex128:
        return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert a.dtype == np.float64, a.dtype
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


def max_threads() -> int:
    return int(_load().orc_max_threads())


def gauss_legendre(n: int):
    """Gauss-Legendre nodes (ascending) and weights on [-1, 1]."""
    x = np.empty(n)
    w = np.empty(n)
    if _load().orc_gauss_legendre(int(n), _p(x), _p(w)) != 0:
        raise ValueError("n must be >= 1")
    return x, w


@dataclass
class Mirror:
    f: float
    a: float
    n_r: int
    n_phi: int
    kind: int
    pos: np.ndarray   # [n_tot, 3]
    nrm: np.ndarray   # [n_tot, 3] unnormalised normal n~ (n dS = n~ r dr dphi)
    wgt: np.ndarray   # [n_tot] surface weights, then the trapezoid step for rim nodes
    tan: np.ndarray   # [n_phi, 3] rim tangent dr_s/dphi (a general surface: [n_rim, 3] line elements dl)
    n_surface: int = -1    # general surfaces only (then n_r = n_phi = 0)
    n_boundary: int = -1

    @property
    def n_surf(self) -> int:
        return self.n_surface if self.n_surface >= 0 else self.n_r * self.n_phi

    @property
    def n_rim(self) -> int:
        return self.n_boundary if self.n_boundary >= 0 else self.n_phi

    @property
    def n_tot(self) -> int:
        return self.n_surf + self.n_rim


def mirror(f: float, a: float, n_r: int, n_phi: int, kind: int = PARABOLOID) -> Mirror:
    n_tot = (n_r + 1) * n_phi
    pos = np.empty((n_tot, 3))
    nrm = np.empty((n_tot, 3))
    wgt = np.empty(n_tot)
    tan = np.empty((n_phi, 3))
    rc = _load().orc_mirror(int(kind), float(f), float(a), int(n_r), int(n_phi),
                            _p(pos), _p(nrm), _p(wgt), _p(tan))
    if rc != 0:
        raise ValueError("invalid mirror parameters")
    return Mirror(f, a, n_r, n_phi, kind, pos, nrm, wgt, tan)


def surface(xyz, ndS, rim_xyz=None, rim_n=None, rim_dl=None) -> Mirror:
    """A general mirror from its quadrature: surface nodes with n dS (weight 1), boundary nodes with
    the surface normal (direction) and the oriented line element dl (weight 1)."""
    xyz, ndS = _f64(xyz).reshape(-1, 3), _f64(ndS).reshape(-1, 3)
    if rim_xyz is None:
        rim_xyz, rim_n, rim_dl = np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 3))
    rim_xyz, rim_n, rim_dl = (_f64(a).reshape(-1, 3) for a in (rim_xyz, rim_n, rim_dl))
    pos = np.ascontiguousarray(np.concatenate([xyz, rim_xyz]))
    nrm = np.ascontiguousarray(np.concatenate([ndS, rim_n]))
    wgt = np.ones(pos.shape[0])
    return Mirror(np.nan, np.nan, 0, 0, -1, pos, nrm, wgt, np.ascontiguousarray(rim_dl), xyz.shape[0],
                  rim_xyz.shape[0])


def incident(kind: int, pts, k: float, w0: float = np.inf, pol: float = 0.0, amp: complex = 1.0):
    """Incident E, B (complex [n, 3]) of a collimated beam travelling along -z."""
    pts = _f64(pts).reshape(-1, 3)
    n = pts.shape[0]
    E = np.empty((n, 3), np.complex128)
    B = np.empty((n, 3), np.complex128)
    _load().orc_incident(int(kind), n, _p(pts), float(k), float(w0), float(pol),
                         float(np.real(amp)), float(np.imag(amp)), _p(E), _p(B))
    return E, B


def incident_tables(m: Mirror, k, kind: int, w0: float = np.inf, pol: float = 0.0, spectrum=None):
    """E_inc, B_inc tables [n_k, n_tot, 3] on the mirror nodes (rim row included)."""
    k = _f64(k).ravel()
    spectrum = np.ones(k.shape[0], np.complex128) if spectrum is None else _c128(spectrum)
    E = np.empty((k.shape[0], m.n_tot, 3), np.complex128)
    B = np.empty_like(E)
    for i, kk in enumerate(k):
        E[i], B[i] = incident(kind, m.pos, kk, w0, pol, spectrum[i])
    return E, B


def incident_lg(modes, pts, k: float, w0: float, amp: complex = 1.0):
    """Incident E, B (complex [n, 3]) of a Laguerre-Gauss mode set (Sec. III-A): modes is a list of
    (p, l, ex, ey) with complex amplitudes ex, ey of the x- and y-polarised parts."""
    pts = _f64(pts).reshape(-1, 3)
    n = pts.shape[0]
    pl = np.ascontiguousarray(np.array([[int(m[0]), int(m[1])] for m in modes], dtype=np.int32).reshape(-1, 2))
    exy = _f64([[np.real(m[2]), np.imag(m[2]), np.real(m[3]), np.imag(m[3])] for m in modes]).reshape(-1, 4)
    E = np.empty((n, 3), np.complex128)
    B = np.empty((n, 3), np.complex128)
    _load().orc_incident_lg(len(modes), pl.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _p(exy), float(w0), n,
                            _p(pts), float(k), float(np.real(amp)), float(np.imag(amp)), _p(E), _p(B))
    return E, B


def incident_lg_tables(m: Mirror, k, modes, w0: float, spectrum=None):
    """E_inc, B_inc tables [n_k, n_tot, 3] of a Laguerre-Gauss mode set on the mirror nodes."""
    k = _f64(k).ravel()
    spectrum = np.ones(k.shape[0], np.complex128) if spectrum is None else _c128(spectrum)
    E = np.empty((k.shape[0], m.n_tot, 3), np.complex128)
    B = np.empty_like(E)
    for i, kk in enumerate(k):
        E[i], B[i] = incident_lg(modes, m.pos, kk, w0, spectrum[i])
    return E, B


def reflected_field(m: Mirror, k, Einc, Binc, obs, line_term: bool = True, threads: int = 0):
    """Reflected E, B [n_k, n_obs, 3] by the Stokes-converted POA integrals."""
    k = _f64(k).ravel()
    obs = _f64(obs).reshape(-1, 3)
    Einc = _c128(Einc)
    Binc = _c128(Binc)
    assert Einc.shape == (k.shape[0], m.n_tot, 3) and Binc.shape == Einc.shape
    E = np.empty((k.shape[0], obs.shape[0], 3), np.complex128)
    B = np.empty_like(E)
    _load().orc_reflected_field(m.n_surf, m.n_rim, _p(m.pos), _p(m.nrm), _p(m.wgt), _p(m.tan),
                                k.shape[0], _p(k), _p(Einc), _p(Binc), obs.shape[0], _p(obs),
                                _p(E), _p(B), int(bool(line_term)), int(threads))
    return E, B


def reflected_field_dgrad(m: Mirror, k, Binc, obs, threads: int = 0):
    """Reflected E [n_k, n_obs, 3] by the double-gradient POA form (no line integral)."""
    k = _f64(k).ravel()
    obs = _f64(obs).reshape(-1, 3)
    Binc = _c128(Binc)
    E = np.empty((k.shape[0], obs.shape[0], 3), np.complex128)
    _load().orc_reflected_field_dgrad(m.n_surf, _p(m.pos), _p(m.nrm), _p(m.wgt), m.n_tot,
                                      k.shape[0], _p(k), _p(Binc), obs.shape[0], _p(obs), _p(E),
                                      int(threads))
    return E


def time_transform(k, dk: float, t, F, threads: int = 0):
    """F(t_m) = sum_n F_n e^{-i k_n t_m} dk for F of shape [n_k, ...] (complex)."""
    k = _f64(k).ravel()
    t = _f64(t).ravel()
    F = _c128(F)
    tail = F.shape[1:]
    n_x = int(np.prod(tail)) if tail else 1
    Ft = np.empty((t.shape[0],) + tail, np.complex128)
    _load().orc_time_transform(k.shape[0], _p(k), float(dk), t.shape[0], _p(t), n_x,
                               _p(F.reshape(k.shape[0], n_x)), _p(Ft), int(threads))
    return Ft


def incident_power(m: Mirror, Einc, Binc):
    """P_n = 4 pi SS Re(E_n x B_n^*) . dA over the aperture, dA along -z (Sec. III-B); [n_k]."""
    E = _c128(Einc)
    B = _c128(Binc)
    n_k = E.shape[0]
    P = np.empty(n_k)
    _load().orc_incident_power(n_k, m.n_surf, m.n_tot, _p(m.nrm), _p(m.wgt), _p(E.reshape(n_k, -1)),
                               _p(B.reshape(n_k, -1)), _p(P))
    return P


def energy_amplitudes(P, eps, e_tot: float = 0.0, dk: float = 0.0):
    """Amplitudes E0_n = sqrt(eps_n / P_n) that give component n the power eps_n
    (Sec. III-B, eq. normalizationAmplitude); with e_tot > 0 the power spectrum is
    first scaled so that sum_n eps_n dk = e_tot (the discrete eq. totalEnergy)."""
    eps = np.asarray(eps, dtype=np.float64)
    if e_tot > 0:
        eps = eps * (e_tot / (np.sum(eps) * dk))
    return np.sqrt(eps / np.asarray(P, dtype=np.float64))


# --------------------------------------------------------------------------- diagnostics (Sec. IV-A)
# Fields on 13-point stencils: the point, then offsets -2h, -h, +h, +2h along x, y and z.
# Derivatives are 4th-order central differences (f(-2h) - 8 f(-h) + 8 f(h) - f(2h)) / (12 h).

_STENCIL_OFFSETS = (-2.0, -1.0, 1.0, 2.0)


def stencil(xyz, h: float) -> np.ndarray:
    """The 13-point stencil of every point of xyz [n, 3], as [13 n, 3]."""
    xyz = _f64(xyz).reshape(-1, 3)
    out = np.repeat(xyz[:, None, :], 13, axis=1)
    for a in range(3):
        for j, o in enumerate(_STENCIL_OFFSETS):
            out[:, 1 + 4 * a + j, a] += o * h
    return out.reshape(-1, 3)


def _fd4(m2, m1, p1, p2, step):
    return (m2 - 8.0 * m1 + 8.0 * p1 - p2) / (12.0 * step)


def _curl(F, h):
    """curl at the stencil centres of F [..., n_pts, 13, 3]."""
    d = [_fd4(*(F[..., 1 + 4 * a + j, :] for j in range(4)), h) for a in range(3)]   # d[a][..., c] = d_a F_c
    return np.stack([d[1][..., 2] - d[2][..., 1], d[2][..., 0] - d[0][..., 2], d[0][..., 1] - d[1][..., 0]],
                    axis=-1)


def _vnorm(v):
    return np.sqrt(np.sum(np.abs(v) ** 2, axis=-1))


def _residual(r1, r2, n1, n2, n3, n4):
    """|2 r1 / (max n1 + max n2) + 2 r2 / (max n3 + max n4)|, maxima over the points (axis 1)."""
    d1 = (n1.max(axis=1) + n2.max(axis=1))[:, None, None]
    d2 = (n3.max(axis=1) + n4.max(axis=1))[:, None, None]
    return _vnorm(2.0 * r1 / d1 + 2.0 * r2 / d2)


def maxwell_residual_freq(k, E, B, n_pts: int, h: float):
    """|e_f| [n_k, n_pts] (eq. relDiffMaxwellFreq) from E, B [n_k, 13 n_pts, 3] on the stencils:
    e_f = 2 (curl E - ik B) / (max|curl E| + max|ik B|) + 2 (curl B + ik E) / (max|curl B| + max|ik E|)."""
    k = _f64(k).reshape(-1, 1, 1)
    E = _c128(E).reshape(k.shape[0], n_pts, 13, 3)
    B = _c128(B).reshape(k.shape[0], n_pts, 13, 3)
    cE, cB = _curl(E, h), _curl(B, h)
    ikB, ikE = 1j * k * B[:, :, 0], 1j * k * E[:, :, 0]
    return _residual(cE - ikB, cB + ikE, _vnorm(cE), _vnorm(ikB), _vnorm(cB), _vnorm(ikE))


def maxwell_residual_time(k, dk: float, t, dt: float, E, B, n_pts: int, h: float, threads: int = 0):
    """|e_t| [n_t, n_pts] (eq. relDiffMaxwellTime) on the physical fields 2 Re F(t), F(t) the
    semi-discrete sum of E, B [n_k, 13 n_pts, 3]; time derivatives by differences of step dt:
    e_t = 2 (curl E + dB/dt) / (max|curl E| + max|dB/dt|) + 2 (curl B - dE/dt) / (max|curl B| + max|dE/dt|)."""
    t = _f64(t).ravel()
    ts = (t[:, None] + dt * np.arange(-2, 3)[None, :]).ravel()
    Et = 2.0 * time_transform(k, dk, ts, E, threads).real.reshape(t.shape[0], 5, n_pts, 13, 3)
    Bt = 2.0 * time_transform(k, dk, ts, B, threads).real.reshape(t.shape[0], 5, n_pts, 13, 3)
    cE, cB = _curl(Et[:, 2], h), _curl(Bt[:, 2], h)
    dE = _fd4(Et[:, 0, :, 0], Et[:, 1, :, 0], Et[:, 3, :, 0], Et[:, 4, :, 0], dt)
    dB = _fd4(Bt[:, 0, :, 0], Bt[:, 1, :, 0], Bt[:, 3, :, 0], Bt[:, 4, :, 0], dt)
    return _residual(cE + dB, cB - dE, _vnorm(cE), _vnorm(dB), _vnorm(cB), _vnorm(dE))


def field_energy(k, dk: float, t, E, B, dV: float, threads: int = 0):
    """W(t) = 1/2 dV sum_points (|2 Re E(t)|^2 + |2 Re B(t)|^2) (Lorentz-Heaviside, c = 1), [n_t]."""
    Et = 2.0 * time_transform(k, dk, t, E, threads).real
    Bt = 2.0 * time_transform(k, dk, t, B, threads).real
    return 0.5 * dV * (np.sum(Et ** 2, axis=(1, 2)) + np.sum(Bt ** 2, axis=(1, 2)))


def solve(w, kind: int = GAUSSIAN, threads: int = 0, line_term: bool = True):
    """Mirror + Gaussian incident tables + reflected field for a ``workloads.Workload``."""
    beam = getattr(w, "beam", 0)
    if kind == GAUSSIAN and beam:
        kind = {1: RADIAL, 2: AZIMUTHAL}[beam] + (1 if getattr(w, "consistent", 0) else 0)
    else:
        kind = GAUSSIAN_CONSISTENT if (kind == GAUSSIAN and getattr(w, "consistent", 0)) else kind
    m = mirror(w.f, w.a, w.n_r, w.n_phi)
    Ei, Bi = incident_tables(m, w.k, kind, w.w0, w.pol, w.spectrum)
    return reflected_field(m, w.k, Ei, Bi, w.obs, line_term=line_term, threads=threads)
