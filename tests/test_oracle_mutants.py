"""Planted-mistake (mutation) tests for the oracle's pins.

Each mutant is a copy of ``oracle/sc_oracle.c`` with one plausible mistake
planted by text substitution -- a dropped term, a flipped sign, a wrong index,
a transposed output, a missing weight -- compiled with gcc on the CPU.  The
battery below re-runs the analytic pins against the mutant; every mutant must
fail at least one of them, and the unmodified source must pass them all.
This is what makes the oracle trustworthy before it is used to judge the HIP
path.
"""
import math
import os

import numpy as np
import pytest

import workloads

K = 2 * math.pi
SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "sc_oracle.c")

# (name, [(original, replacement, count)]): the original text must occur exactly ``count``
# times; a negative count -n means "occurs n times, replace only the first".
# (Normalising n in the rim term cannot be mutated into a mistake: n . dl = 0, so
# n x (n x B) . dl = -B . dl whatever the length of n.)
MUTANTS = [
    ("drop_ikJg", [("cld t1 = cmul(ik2, g);", "cld t1 = { 0.0L, 0.0L };", 1)]),
    ("drop_rho_grad", [("cld t2 = cscale(cmul(rho, fac), 2.0L);", "cld t2 = { 0.0L, 0.0L };", 1)]),
    ("rho_factor", [("cld t2 = cscale(cmul(rho, fac), 2.0L);", "cld t2 = cscale(cmul(rho, fac), 1.0L);", 1)]),
    ("drop_line", [("if (line_term) {", "if (0) {", 1)]),
    ("line_sign", [("cld m2ik = { 0.0L, 2.0L / k };", "cld m2ik = { 0.0L, -2.0L / k };", 1)]),
    ("line_weight", [("cld s = cscale(cmul(cmul(m2ik, b), fac), (ld)wgt[q]);",
                      "cld s = cmul(cmul(m2ik, b), fac);", 1)]),
    ("B_sign", [("cld f2 = cscale(fac, 2.0L * W);", "cld f2 = cscale(fac, -2.0L * W);", 1)]),
    ("B_cross_index", [("Jx[1] = cadd(cscale(J[2], Rv[0]), cscale(J[0], -Rv[2]));",
                        "Jx[1] = cadd(cscale(J[2], Rv[0]), cscale(J[0], -Rv[1]));", 1)]),
    ("J_cross_index", [("J[1] = cadd(cscale(Bi[0], n[2]), cscale(Bi[2], -n[0]));",
                        "J[1] = cadd(cscale(Bi[0], n[2]), cscale(Bi[2], -n[1]));", -2)]),
    ("E_weight", [("E[c] = cadd(E[c], cscale(cadd(cmul(J[c], t1), cscale(t2, Rv[c])), W));",
                   "E[c] = cadd(E[c], cadd(cmul(J[c], t1), cscale(t2, Rv[c])));", 1)]),
    ("normal_flipped", [("nrm[3 * q + 0] = -dFdr * c;", "nrm[3 * q + 0] = dFdr * c;", 1),
                        ("nrm[3 * q + 1] = -dFdr * s;", "nrm[3 * q + 1] = dFdr * s;", 1),
                        ("nrm[3 * q + 2] = 1.0;", "nrm[3 * q + 2] = -1.0;", 1)]),
    ("normal_tilt", [("nrm[3 * q + 0] = -dFdr * c;", "nrm[3 * q + 0] = dFdr * c;", 1),
                     ("nrm[3 * q + 1] = -dFdr * s;", "nrm[3 * q + 1] = dFdr * s;", 1)]),
    ("no_r_jacobian", [("wgt[q] = (i < n_r) ? wr * r * dphi : dphi;", "wgt[q] = (i < n_r) ? wr * dphi : dphi;", 1)]),
    ("radial_weight_half", [("double wr = (i < n_r) ? a * wg[i] / 2.0 : 0.0;",
                             "double wr = (i < n_r) ? a * wg[i] : 0.0;", 1)]),
    ("dphi", [("const double dphi = 2.0 * M_PI / (double)n_phi;", "const double dphi = M_PI / (double)n_phi;", 1)]),
    ("paraboloid_z", [("double z = (kind == 0) ? r * r / (4.0 * f) - f : 0.0;",
                       "double z = (kind == 0) ? r * r / (2.0 * f) - f : 0.0;", 1)]),
    ("R_direction", [("Rv[0] = (ld)rs[0] - (ld)ro[0];", "Rv[0] = (ld)ro[0] - (ld)rs[0];", 1),
                     ("Rv[1] = (ld)rs[1] - (ld)ro[1];", "Rv[1] = (ld)ro[1] - (ld)rs[1];", 1),
                     ("Rv[2] = (ld)rs[2] - (ld)ro[2];", "Rv[2] = (ld)ro[2] - (ld)rs[2];", 1)]),
    ("green_phase_sign", [("sincosl(k * *R, &s, &c);", "sincosl(-k * *R, &s, &c);", 1)]),
    ("grad_1overR_sign", [("cld ikm = { -1.0L / *R, k };", "cld ikm = { 1.0L / *R, k };", 1)]),
    ("no_4pi", [("ld inv = 1.0L / (4.0L * PI_L * *R);", "ld inv = 1.0L / (PI_L * *R);", 1)]),
    ("rim_B_sign", [("cld v = cadd(cscale(nB, (ld)n[c] / nn), cscale(Bi[c], -1.0L));",
                     "cld v = cadd(cscale(nB, (ld)n[c] / nn), cscale(Bi[c], 1.0L));", 1)]),
    ("rim_tangent_sign", [("tan[3 * j + 0] = -a * s;", "tan[3 * j + 0] = a * s;", 1),
                          ("tan[3 * j + 1] = a * c;", "tan[3 * j + 1] = -a * c;", 1)]),
    ("incident_B_sign", [("b[1][0] = -pr; b[1][1] = -pi;", "b[1][0] = pr; b[1][1] = pi;", 2)]),
    ("incident_phase_sign", [("ld ph = -(ld)k * (ld)Z;", "ld ph = (ld)k * (ld)Z;", 1)]),
    ("consistent_Ez_sign", [("e[2][0] = -c3 * pi; e[2][1] = c3 * pr;", "e[2][0] = c3 * pi; e[2][1] = -c3 * pr;", 1)]),
    ("consistent_c1", [("- 4.0 * y * y / (kw2 * kw2)", "- 4.0 * x * x / (kw2 * kw2)", 1)]),
    ("gauss_width", [("exp(-(x * x + y * y) / (w0 * w0))", "exp(-(x * x + y * y) / (2.0 * w0 * w0))", 1)]),
    ("pol_rotation", [("double y = -sp * X + cp * Y;", "double y = sp * X + cp * Y;", 1)]),
    ("gl_weight", [("qd wi = 2.0Q / ((1.0Q - zq * zq) * dpq * dpq);", "qd wi = 2.0Q / ((1.0Q + zq * zq) * dpq * dpq);", 1)]),
    ("gl_recurrence", [("ld p2 = ((2.0L * m + 1.0L) * x * p1 - (ld)m * p0) / (ld)(m + 1);",
                        "ld p2 = ((2.0L * m + 1.0L) * x * p1 - (ld)m * p0) / (ld)(m + 2);", 1),
                       ("qd p2 = ((2.0Q * m + 1.0Q) * x * p1 - (qd)m * p0) / (qd)(m + 1);",
                        "qd p2 = ((2.0Q * m + 1.0Q) * x * p1 - (qd)m * p0) / (qd)(m + 2);", 1)]),
    ("output_transpose", [("size_t off = ((size_t)ik * n_obs + o) * 6;", "size_t off = ((size_t)o * n_k + ik) * 6;", -2)]),
    ("dgrad_sign", [("cld c1 = { -1.0L / (R * R), k / R };", "cld c1 = { 1.0L / (R * R), k / R };", 1)]),
    ("time_sign", [("qd ph = -(qd)kv[n] * (qd)t[m];", "qd ph = (qd)kv[n] * (qd)t[m];", 1)]),
    ("time_reduction", [("qd red = ph - TWO_PI_Q * rintq(ph / TWO_PI_Q);", "qd red = ph - M_PIq * rintq(ph / M_PIq);", 1)]),
    ("time_dk", [("(double)(acc.re * (ld)dk)", "(double)(acc.re)", 1), ("(double)(acc.im * (ld)dk)", "(double)(acc.im)", 1)]),
    ("power_sign", [("acc += (ld)wgt[q] * (ld)nrm[3 * q + 2] * (-sz);", "acc += (ld)wgt[q] * (ld)nrm[3 * q + 2] * sz;", 1)]),
    ("power_drop_EyBx", [("- ((ld)e[2] * b[0] + (ld)e[3] * b[1])", "", 1)]),
    ("power_no_4pi", [("P[n] = (double)(4.0L * PI_L * acc);", "P[n] = (double)(acc);", 1)]),
    ("power_unweighted", [("acc += (ld)wgt[q] * (ld)nrm[3 * q + 2] * (-sz);", "acc += -sz;", 1)]),
    ("cyl_radial_B_sign", [("B[2] = -X * gr; B[3] = -X * gi;", "B[2] = X * gr; B[3] = X * gi;", 1)]),
    ("cyl_longitudinal_sign", [("double lr = -c * gi, li = c * gr;", "double lr = c * gi, li = -c * gr;", 1)]),
    ("cyl_longitudinal_coeff", [("(2.0 / k) * (r2 / (w0 * w0) - 1.0)", "(2.0 / k) * (r2 / (w0 * w0) + 1.0)", 1)]),
    ("cyl_azimuthal_E", [("E[0] = -Y * gr; E[1] = -Y * gi;", "E[0] = Y * gr; E[1] = Y * gi;", 1)]),
    ("power_with_rim", [("for (int q = 0; q < n_surf; ++q) {\n            const double *e = E + 6",
                         "for (int q = 0; q < n_tot; ++q) {\n            const double *e = E + 6", 1)]),
    ("lg_laguerre_sign", [("s += (j % 2) ? -term : term;", "s += term;", 1)]),
    ("lg_normalisation", [("ld C = sqrtl(2.0L * expl(", "ld C = sqrtl(1.0L * expl(", 1)]),
    ("lg_phase_sign", [("ui = u * sinl((ld)l * phi);", "ui = -u * sinl((ld)l * phi);", 1)]),
    ("lg_B_sign", [("B[6 * q + 2] = -(double)Exr; B[6 * q + 3] = -(double)Exi;",
                    "B[6 * q + 2] = (double)Exr; B[6 * q + 3] = (double)Exi;", 1)]),
    ("lg_width", [("expl(-r * r / ((ld)w0 * (ld)w0))", "expl(-r * r / (2.0L * (ld)w0 * (ld)w0))", 1)]),
    ("lg_radial_power", [("powl(rho, (ld)al)", "powl(rho, (ld)(al + 1))", 1)]),
    ("lg_binomial", [("lgammal((ld)(p - j + 1)) - lgammal((ld)(a + j + 1))",
                      "lgammal((ld)(p - j + 1)) - lgammal((ld)(j + 1))", 1)]),
]


# --------------------------------------------------------------------------- the battery

def _cis(x):
    return complex(math.cos(x), math.sin(x))


def pin_p1(orc):
    f, a = 20.0, 25.0
    ks = [K, 1.07 * K]
    m = orc.mirror(f, a, 60, 32)
    Ei, Bi = orc.incident_tables(m, ks, orc.PLANE)
    E, B = orc.reflected_field(m, ks, Ei, Bi, np.zeros((3, 3)))
    U = a * a / (4 * f)
    for i, k in enumerate(ks):
        ph = np.exp(2j * k * f)
        ex = ph * (2j * k * f * U / (f + U) + U * (U - 2 * f) / (f + U) ** 2 - 2j * f * U / (k * (f + U) ** 3))
        by = ph * (2j * k * f * U / (f + U) - U * (U + 2 * f) / (f + U) ** 2)
        if np.abs(E[i, :, 0] - ex).max() > 1e-9 * abs(ex) or np.abs(B[i, :, 1] - by).max() > 1e-9 * abs(by):
            return False
        if np.abs(E[i, :, 1:]).max() > 1e-9 * abs(ex):
            return False
    return True


def pin_p2(orc):
    a, zp = 10.0, 2.5
    m = orc.mirror(1.0, a, 200, 16, kind=orc.FLAT)
    Ei, Bi = orc.incident_tables(m, [K], orc.PLANE)
    E, _ = orc.reflected_field(m, [K], Ei, Bi, np.array([[0.0, 0.0, zp]]))
    Ra = math.hypot(a, zp)
    ex = _cis(K * Ra) - _cis(K * zp) - (a * a / (2 * Ra * Ra)) * (1 + 1j / (K * Ra)) * _cis(K * Ra)
    return abs(E[0, 0, 0] - ex) < 1e-9


def pin_forms(orc):
    # plane wave, and a narrow curl-consistent Gaussian (B_z != 0 on the mirror)
    m = orc.mirror(20.0, 40.0, 100, 48)
    obs = np.array([[0.3, 0.2, 0.1], [-1.0, 0.5, -0.7]])
    for kind, w0 in ((orc.PLANE, np.inf), (orc.GAUSSIAN_CONSISTENT, 5.0)):
        Ei, Bi = orc.incident_tables(m, [K], kind, w0)
        E, _ = orc.reflected_field(m, [K], Ei, Bi, obs)
        Edg = orc.reflected_field_dgrad(m, [K], Bi, obs)
        if not np.abs(E - Edg).max() < 1e-9 * np.abs(Edg).max():
            return False
    return True


def _fd_jac(F, h):
    d = np.zeros((3, 3), complex)
    for ax in range(3):
        fm2, fm1, fp1, fp2 = F[1 + 4 * ax: 5 + 4 * ax]
        d[ax] = (fm2 - 8 * fm1 + 8 * fp1 - fp2) / (12 * h)
    return d


def _stencil(p0, h):
    pts = [p0]
    for ax in range(3):
        for s in (-2, -1, 1, 2):
            d = np.zeros(3)
            d[ax] = s * h
            pts.append(p0 + d)
    return np.array(pts)


def _curl(d):
    return np.array([d[1, 2] - d[2, 1], d[2, 0] - d[0, 2], d[0, 1] - d[1, 0]])


def pin_maxwell(orc):
    h = 0.01
    m = orc.mirror(20.0, 40.0, 40, 32)
    Ei, Bi = workloads.random_incident_tables(1, m.n_tot, seed=11)
    E, B = orc.reflected_field(m, [K], Ei, Bi, _stencil(np.array([0.3, 0.2, 0.1]), h))
    s = K * max(np.abs(E[0, 0]).max(), np.abs(B[0, 0]).max())
    if np.abs(_curl(_fd_jac(E[0], h)) - 1j * K * B[0, 0]).max() / s > 1e-5:
        return False
    m = orc.mirror(20.0, 40.0, 80, 64)
    Ei, Bi = orc.incident_tables(m, [K], orc.GAUSSIAN_CONSISTENT, 20.0)
    E, B = orc.reflected_field(m, [K], Ei, Bi, _stencil(np.array([0.3, 0.2, 0.1]), h))
    dE, dB = _fd_jac(E[0], h), _fd_jac(B[0], h)
    s = K * np.abs(E[0, 0]).max()
    return (abs(np.trace(dE)) / s < 1e-5 and np.abs(_curl(dB) + 1j * K * E[0, 0]).max() / s < 1e-5)


def pin_symmetry(orc):
    m = orc.mirror(20.0, 40.0, 40, 32)
    Ei, Bi = orc.incident_tables(m, [K], orc.GAUSSIAN, 20.0)
    p = np.array([[0.7, 0.4, 0.3]])
    E, B = orc.reflected_field(m, [K], Ei, Bi, p)
    Ex, Bx = orc.reflected_field(m, [K], Ei, Bi, p * np.array([-1, 1, 1]))
    sE, sB = np.abs(E).max(), np.abs(B).max()
    ok = (np.abs(Ex - E * np.array([1, -1, -1])).max() < 1e-12 * sE
          and np.abs(Bx - B * np.array([-1, 1, 1])).max() < 1e-12 * sB)
    # 90-degree rotation x-pol -> y-pol, with the curl-consistent beam (not axisymmetric)
    rot = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    Ei, Bi = orc.incident_tables(m, [K], orc.GAUSSIAN_CONSISTENT, 5.0)
    E, B = orc.reflected_field(m, [K], Ei, Bi, p)
    Ei2, Bi2 = orc.incident_tables(m, [K], orc.GAUSSIAN_CONSISTENT, 5.0, pol=math.pi / 2)
    E2, B2 = orc.reflected_field(m, [K], Ei2, Bi2, p @ rot.T)
    sE, sB = np.abs(E).max(), np.abs(B).max()
    return ok and np.abs(E2 - E @ rot.T).max() < 1e-12 * sE and np.abs(B2 - B @ rot.T).max() < 1e-12 * sB


def pin_paraxial(orc):
    f, w0 = 2000.0, 100.0
    m = orc.mirror(f, 3 * w0, 100, 48)
    Ei, Bi = orc.incident_tables(m, [K], orc.GAUSSIAN, w0)
    zR = K * w0 * w0 / 2
    qm = -f / (1 - 1j * f / zR)
    obs = np.array([[0, 0, 0], [3, 0, 0], [0, 0, 50]], float)
    E, B = orc.reflected_field(m, [K], Ei, Bi, obs)
    q = qm + f + obs[:, 2]
    ex = -np.exp(1j * K * f) * (qm / q) * np.exp(1j * K * (obs[:, 0] ** 2) / (2 * q)) * np.exp(1j * K * (f + obs[:, 2]))
    sc = np.abs(ex).max()
    return np.abs(E[0, :, 0] - ex).max() / sc < 3e-3 and np.abs(B[0, :, 1] - ex).max() / sc < 3e-3


def pin_flux(orc):
    f, a, w0 = 20.0, 15.0, 6.0
    m = orc.mirror(f, a, 60, 48)
    Ei, Bi = orc.incident_tables(m, [K], orc.GAUSSIAN_CONSISTENT, w0)
    L, n = 6.0, 25
    h = 2 * L / (n - 1)
    E, B = orc.reflected_field(m, [K], Ei, Bi, workloads.focal_plane(L, n, 3.0))
    Sz = 0.5 * np.real(E[0, :, 0] * np.conj(B[0, :, 1]) - E[0, :, 1] * np.conj(B[0, :, 0]))
    p_inc = math.pi * w0 * w0 / 4 * (1 - math.exp(-2 * a * a / (w0 * w0)))
    return abs(Sz.sum() * h * h / p_inc - 1) < 1e-2


def pin_rules(orc):
    x, w = orc.gauss_legendre(17)
    p0, p1 = np.ones_like(x), x.copy()
    worst = abs(np.dot(w, p1))
    for mm in range(1, 33):
        p0, p1 = p1, ((2 * mm + 1) * x * p1 - mm * p0) / (mm + 1)
        worst = max(worst, abs(np.dot(w, p1)))
    if worst > 1e-14 or abs(w.sum() - 2) > 1e-14:
        return False
    f, a = 0.05, 0.15
    m = orc.mirror(f, a, 60, 32)
    W, n = m.wgt[: m.n_surf], m.nrm[: m.n_surf]
    area = 2 * math.pi * (4 * f * f / 3) * ((1 + a * a / (4 * f * f)) ** 1.5 - 1)
    r = np.hypot(m.pos[:, 0], m.pos[:, 1])
    return (abs(W.sum() / (math.pi * a * a) - 1) < 1e-12
            and abs(np.sum(W * np.linalg.norm(n, axis=1)) / area - 1) < 1e-10
            and np.abs(m.pos[:, 2] - (r * r / (4 * f) - f)).max() < 1e-15
            and np.all(n[:, 2] > 0) and np.all(np.einsum("ij,ij->i", n, -m.pos[: m.n_surf]) > 0)
            and np.allclose(m.tan[:, 1], a * np.cos(2 * np.pi * np.arange(32) / 32), atol=1e-15))


def pin_time(orc):
    n, k0, dk = 9, 5.0, 0.125
    k = k0 + dk * np.arange(n)
    t = np.linspace(-20.0, 20.0, 9) + 1e-3
    Ft = orc.time_transform(k, dk, t, np.ones((n, 1)))[:, 0]
    z = np.exp(-1j * dk * t)
    return np.abs(Ft - np.exp(-1j * k0 * t) * dk * (1 - z ** n) / (1 - z)).max() < 1e-12


def pin_power(orc):
    # aperture power of the incident beam: closed forms for the plane wave, the
    # literal Gaussian (x- and y-polarised) and the curl-consistent Gaussian
    f, a, w0 = 20.0, 25.0, 10.0
    m = orc.mirror(f, a, 60, 32)
    ks = [K, 1.3 * K]
    Ei, Bi = orc.incident_tables(m, ks, orc.PLANE)
    if np.abs(orc.incident_power(m, Ei, Bi) / (4 * math.pi * math.pi * a * a) - 1).max() > 1e-12:
        return False
    lit = 4 * math.pi * (math.pi * w0 * w0 / 2) * (1 - math.exp(-2 * a * a / (w0 * w0)))
    for pol in (0.0, math.pi / 2):
        Ei, Bi = orc.incident_tables(m, ks, orc.GAUSSIAN, w0, pol=pol)
        if np.abs(orc.incident_power(m, Ei, Bi) / lit - 1).max() > 1e-12:
            return False
    w0 = 5.0   # a = 5 w0: the clipped tail is exp(-50)
    Ei, Bi = orc.incident_tables(m, ks, orc.GAUSSIAN_CONSISTENT, w0)
    P = orc.incident_power(m, Ei, Bi)
    ex = [4 * math.pi * (math.pi * w0 * w0 / 2) * (1 + 1 / (k * w0) ** 2) for k in ks]
    return np.abs(P / np.array(ex) - 1).max() < 1e-12


def pin_cylindrical(orc):
    # aperture power closed form of the radial and azimuthal beams, and Maxwell's equations
    # of their curl-consistent variants
    a, w0 = 25.0, 6.0
    m = orc.mirror(20.0, a, 60, 32)
    b = 2 * a * a / (w0 * w0)
    ex = math.pi ** 2 * w0 * w0 * (1 - math.exp(-b) * (1 + b))
    for kind in (orc.RADIAL, orc.AZIMUTHAL):
        Ei, Bi = orc.incident_tables(m, [K], kind, w0)
        if abs(orc.incident_power(m, Ei, Bi)[0] / ex - 1) > 1e-12:
            return False
    h = 1e-3
    pts = _stencil(np.array([0.7, -0.4, 0.3]), h)
    E, B = orc.incident(orc.RADIAL_CONSISTENT, pts, K, 3.0)
    s = K * np.abs(E[0]).max()
    if np.abs(_curl(_fd_jac(B, h)) + 1j * K * E[0]).max() / s > 1e-9:
        return False
    E, B = orc.incident(orc.AZIMUTHAL_CONSISTENT, pts, K, 3.0)
    s = K * np.abs(B[0]).max()
    return np.abs(_curl(_fd_jac(E, h)) - 1j * K * B[0]).max() / s < 1e-9


def pin_lg(orc):
    # Laguerre-Gauss modes: LG_00 is the normalised Gaussian, aperture powers match the closed form
    # (scipy's Laguerre polynomials and incomplete gamma), modes of the same l and different p are
    # orthogonal on the plane, and LG_{0,+-1} make the radial beam
    from test_oracle_lg import aperture_power_closed_form
    w0 = 4.0
    pts = np.array([[0.5, -1.2, 0.3], [2.0, 1.0, -0.4], [-3.0, 0.5, 0.9]])
    E, B = orc.incident_lg([(0, 0, 1.0, 0.0)], pts, K, w0)
    Eg, Bg = orc.incident(orc.GAUSSIAN, pts, K, w0)
    c = math.sqrt(2 / math.pi) / w0
    if np.abs(E - c * Eg).max() > 1e-14 * np.abs(Eg).max() or np.abs(B - c * Bg).max() > 1e-14 * np.abs(Bg).max():
        return False
    m = orc.mirror(20.0, 6.0, 80, 32)
    for p, l in ((0, 1), (2, 1), (1, -2)):
        P = orc.incident_power(m, *orc.incident_lg_tables(m, [K], [(p, l, 1.0, 0.0)], w0))[0]
        if abs(P / aperture_power_closed_form(p, l, w0, 6.0) - 1) > 1e-11:
            return False
    m = orc.mirror(20.0, 7 * w0, 160, 32)
    P = orc.incident_power(m, *orc.incident_lg_tables(m, [K], [(0, 1, 1.0, 0.0), (2, 1, 1.0, 0.0)], w0))[0]
    if abs(P / (8 * math.pi) - 1) > 1e-11:
        return False
    al = 1 / (2 * math.sqrt(2) * c)
    E, B = orc.incident_lg([(0, 1, al, -1j * al), (0, -1, al, 1j * al)], pts, K, w0)
    Er, Br = orc.incident(orc.RADIAL, pts, K, w0)
    return np.abs(E - Er).max() < 1e-13 * np.abs(Er).max() and np.abs(B - Br).max() < 1e-13 * np.abs(Br).max()


BATTERY = [pin_p1, pin_p2, pin_forms, pin_maxwell, pin_symmetry, pin_paraxial, pin_flux, pin_rules, pin_time,
           pin_power, pin_cylindrical, pin_lg]


def run_battery(orc):
    out = {}
    for pin in BATTERY:
        try:
            with np.errstate(all="ignore"):
                out[pin.__name__] = bool(pin(orc))
        except Exception:
            out[pin.__name__] = False
    return out


def test_unmodified_oracle_passes_battery(orc):
    res = run_battery(orc)
    assert all(res.values()), res


@pytest.mark.parametrize("name,subs", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(orc, tmp_path, name, subs):
    src = open(SRC).read()
    for old, new, count in subs:
        assert src.count(old) == abs(count), f"mutation site for {name!r} not found as expected: {old!r}"
        src = src.replace(old, new, 1 if count < 0 else count)
    path = tmp_path / f"mut_{name}.c"
    path.write_text(src)
    lib = orc.compile_source(str(path), str(tmp_path / f"libmut_{name}.so"))
    with orc.use_library(lib):
        res = run_battery(orc)
    assert not all(res.values()), f"mutant {name} passed every pin: {res}"
