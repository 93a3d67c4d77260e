/*
 * sc_oracle.c -- CPU reference ("oracle") for the physical-optics Stratton-Chu
 * diffraction integrals of a field reflected off a parabolic mirror.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  The product path (the HIP
 * library) never calls it and shares no code with it.
 *
 * It is deliberately plain and slow: one loop per sum, FP64 everywhere, and
 * the large phase k*R (up to ~1e6 rad) plus the accumulations in x87
 * long double (64-bit mantissa), with glibc's sincosl for the exponentials;
 * the quadrature roots are refined and the phases k t of the time transform
 * formed in quad precision (__float128).
 *
 * What it computes (units c = 1, Lorentz-Heaviside, time factor e^{-ikt}):
 *
 *   Green's function (Sec. II):  g(r, r') = e^{ik|r-r'|} / (4 pi |r-r'|);
 *   the gradient acts on the surface variable r, so with R = r - r':
 *        grad g = (ik - 1/R) g R/|R|.
 *   Physical-optics current on a perfect conductor (Sec. II, POA): J = 2 n x B_inc.
 *   Reflected field, Stokes-converted form (Sec. II, eq. stratton-chu-poa-og):
 *        E' = 2 SS { ik (n x B_inc) g + (n . E_inc) grad g } dS
 *             - (2/ik) O grad g [ n x (n x B_inc) ] . dl
 *        B' = 2 SS (n x B_inc) x grad g dS
 *   The double-gradient form (Sec. II, eq. stratton-chu-poa) is provided as an
 *   independent cross-check:
 *        E' = 2 SS { ik (n x B_inc) g + (i/k) gradgrad g . (n x B_inc) } dS
 *   with gradgrad g = -I (1/R^2 - ik/R) g + Rh Rh (3/R^2 - 3ik/R - k^2) g
 *   (Appendix, explicit double gradient).
 *
 *   Discretisation (Sec. III-C): mirror z = F(r) = r^2/(4f) - f in cylindrical
 *   coordinates, tensor-product Gauss-Legendre in r on [0, a] and the
 *   trapezoid rule in phi; n dS = n~ r dr dphi with the unnormalised normal
 *   n~ = (-x/2f, -y/2f, 1) pointing from the mirror toward the focus and the
 *   incoming beam.  The rim line integral uses the same phi nodes with
 *   dl = (dr_s/dphi) dphi (increasing phi).
 *
 *   Semi-discrete transform to time (Sec. III-B, eq. impl.semiDiscreteFFT):
 *        F(t) = sum_n F_n e^{-i k_n t} dk.
 *
 * Conventions (all complex arrays are interleaved re, im doubles):
 *   node arrays:  the n_r*n_phi surface nodes in r-major order (i*n_phi + j),
 *                 followed by the n_phi rim nodes (r = a);
 *   incident tables: [n_k][n_nodes_total][3] complex;
 *   fields:          [n_k][n_obs][3] complex.
 */
#define _GNU_SOURCE 1   /* sincosl */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef long double ld;
typedef __float128 qd;
#include <quadmath.h>
#define TWO_PI_Q (2.0Q * M_PIq)

static const ld PI_L = 3.141592653589793238462643383279502884L;

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre rule on [-1, 1]: roots of P_n by Newton's method from the  */
/* usual cosine initial guess, iterated in long double and finished with two */
/* Newton steps in quad precision (__float128), so that every node and weight */
/* is the correctly rounded double of the exact rule.  Ascending order.      */
/* ------------------------------------------------------------------------ */
static void legendre_p(int n, ld x, ld *p, ld *dp)
{
    /* Bonnet recurrence: (m+1) P_{m+1} = (2m+1) x P_m - m P_{m-1} */
    ld p0 = 1.0L, p1 = x;
    if (n == 0) { *p = 1.0L; *dp = 0.0L; return; }
    for (int m = 1; m < n; ++m) {
        ld p2 = ((2.0L * m + 1.0L) * x * p1 - (ld)m * p0) / (ld)(m + 1);
        p0 = p1;
        p1 = p2;
    }
    *p = p1;
    /* P_n'(x) = n (x P_n - P_{n-1}) / (x^2 - 1) */
    *dp = (ld)n * (x * p1 - p0) / (x * x - 1.0L);
}

static void legendre_p_q(int n, qd x, qd *p, qd *dp)
{
    qd p0 = 1.0Q, p1 = x;
    for (int m = 1; m < n; ++m) {
        qd p2 = ((2.0Q * m + 1.0Q) * x * p1 - (qd)m * p0) / (qd)(m + 1);
        p0 = p1;
        p1 = p2;
    }
    *p = p1;
    *dp = (qd)n * (x * p1 - p0) / (x * x - 1.0Q);
}

int orc_gauss_legendre(int n, double *x, double *w)
{
    if (n < 1) return -1;
    for (int i = 0; i < n; ++i) {
        /* i-th root counted from x = +1 downward */
        ld z = cosl(PI_L * ((ld)i + 0.75L) / ((ld)n + 0.5L));
        ld p, dp;
        for (int it = 0; it < 100; ++it) {
            legendre_p(n, z, &p, &dp);
            ld dz = p / dp;
            z -= dz;
            if (fabsl(dz) < 1e-18L) break;
        }
        qd zq = (qd)z, pq, dpq;
        for (int it = 0; it < 2; ++it) {
            if (n == 1) { zq = 0.0Q; break; }
            legendre_p_q(n, zq, &pq, &dpq);
            zq -= pq / dpq;
        }
        if (n == 1) dpq = 1.0Q;
        else legendre_p_q(n, zq, &pq, &dpq);
        qd wi = 2.0Q / ((1.0Q - zq * zq) * dpq * dpq);
        /* store ascending */
        x[n - 1 - i] = (double)zq;
        w[n - 1 - i] = (double)wi;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Mirror discretisation.                                                    */
/* kind 0: paraboloid z = r^2/(4f) - f (focus at the origin);                */
/* kind 1: flat disk z = 0 (test geometry for a closed-form check).          */
/* pos, nrm: [n_tot][3]; wgt: [n_tot]; tan: [n_phi][3].                       */
/* wgt holds W_ij = w_i (a/2) * r_i * (2 pi / n_phi) for surface nodes and    */
/* the trapezoid step 2 pi / n_phi for rim nodes.                            */
/* ------------------------------------------------------------------------ */
int orc_mirror(int kind, double f, double a, int n_r, int n_phi,
               double *pos, double *nrm, double *wgt, double *tan)
{
    if (n_r < 1 || n_phi < 1 || !(a > 0.0) || (kind == 0 && !(f > 0.0))) return -1;
    double *xg = (double *)malloc(sizeof(double) * n_r);
    double *wg = (double *)malloc(sizeof(double) * n_r);
    orc_gauss_legendre(n_r, xg, wg);
    const double dphi = 2.0 * M_PI / (double)n_phi;
    for (int i = 0; i <= n_r; ++i) {
        /* i == n_r is the rim row */
        double r = (i < n_r) ? a * (1.0 + xg[i]) / 2.0 : a;
        double wr = (i < n_r) ? a * wg[i] / 2.0 : 0.0;
        for (int j = 0; j < n_phi; ++j) {
            double phi = 2.0 * M_PI * (double)j / (double)n_phi;
            double c, s;
            sincos(phi, &s, &c);   /* glibc sincos (sin and cos may differ from it in the last bit) */
            size_t q = (size_t)i * n_phi + j;
            double x = r * c, y = r * s;
            double z = (kind == 0) ? r * r / (4.0 * f) - f : 0.0;
            pos[3 * q + 0] = x;
            pos[3 * q + 1] = y;
            pos[3 * q + 2] = z;
            /* dr_s/dr x dr_s/dphi = r * (-dF/dr cos, -dF/dr sin, 1) */
            double dFdr = (kind == 0) ? r / (2.0 * f) : 0.0;
            nrm[3 * q + 0] = -dFdr * c;
            nrm[3 * q + 1] = -dFdr * s;
            nrm[3 * q + 2] = 1.0;
            wgt[q] = (i < n_r) ? wr * r * dphi : dphi;
            if (i == n_r) {
                tan[3 * j + 0] = -a * s;
                tan[3 * j + 1] = a * c;
                tan[3 * j + 2] = 0.0;
            }
        }
    }
    free(xg);
    free(wg);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Incident fields at arbitrary points (collimated beam travelling along -z). */
/* kind 0: plane wave   E = p G e^{-ikz}, B = (-z^) x E, G = 1               */
/* kind 1: literal Gaussian, same with G = exp(-(x^2+y^2)/w0^2)               */
/* kind 2: curl-consistent Gaussian (x-polarised frame):                     */
/*         B = psi (0, -1, -2iy/(k w0^2)),  E = (i/k) curl B, psi = G e^{-ikz} */
/*         E = psi (1 + 2/(k^2 w0^2) - 4y^2/(k^2 w0^4), 4xy/(k^2 w0^4),        */
/*                  2ix/(k w0^2))                                            */
/* pol rotates the polarisation (and the field pattern) about z.              */
/* kinds 3-6: cylindrical vector beams, g = exp(-r^2/w0^2) / w0 e^{-ikz}:    */
/*   3 radial (literal)        E = g (x, y, 0),  B = g (y, -x, 0) = (-z^) x E  */
/*   4 radial, consistent      E gains E_z = (2i/k)(r^2/w0^2 - 1) g, so that  */
/*                             E = (i/k) curl B with the same B               */
/*   5 azimuthal (literal)     E = g (-y, x, 0), B = g (x, y, 0) = (-z^) x E  */
/*   6 azimuthal, consistent   B gains B_z = (2i/k)(r^2/w0^2 - 1) g, so that  */
/*                             B = (-i/k) curl E with the same E              */
/* (pol does not enter: these beams are axisymmetric).                        */
/* amp is a complex factor (spectral amplitude and phase).                    */
/* ------------------------------------------------------------------------ */
static void cylindrical_beam(int kind, double X, double Y, double Z, double k, double w0, double amp_re,
                             double amp_im, double *E, double *B)
{
    double r2 = X * X + Y * Y;
    double G = exp(-r2 / (w0 * w0)) / w0;
    ld sl, cl;
    sincosl(-(ld)k * (ld)Z, &sl, &cl);
    double gr = G * (double)(cl * amp_re - sl * amp_im);
    double gi = G * (double)(cl * amp_im + sl * amp_re);
    double c = (kind == 4 || kind == 6) ? (2.0 / k) * (r2 / (w0 * w0) - 1.0) : 0.0;   /* i c g */
    double lr = -c * gi, li = c * gr;
    if (kind == 3 || kind == 4) {
        E[0] = X * gr; E[1] = X * gi;
        E[2] = Y * gr; E[3] = Y * gi;
        E[4] = lr;     E[5] = li;
        B[0] = Y * gr;  B[1] = Y * gi;
        B[2] = -X * gr; B[3] = -X * gi;
        B[4] = 0.0;     B[5] = 0.0;
    } else {
        E[0] = -Y * gr; E[1] = -Y * gi;
        E[2] = X * gr;  E[3] = X * gi;
        E[4] = 0.0;     E[5] = 0.0;
        B[0] = X * gr; B[1] = X * gi;
        B[2] = Y * gr; B[3] = Y * gi;
        B[4] = lr;     B[5] = li;
    }
}

int orc_incident(int kind, int n_pts, const double *pts, double k, double w0, double pol,
                 double amp_re, double amp_im, double *E, double *B)
{
    const double cp = cos(pol), sp = sin(pol);
    for (int q = 0; q < n_pts; ++q) {
        if (kind >= 3) {
            cylindrical_beam(kind, pts[3 * q], pts[3 * q + 1], pts[3 * q + 2], k, w0, amp_re, amp_im, E + 6 * q,
                             B + 6 * q);
            continue;
        }
        double X = pts[3 * q], Y = pts[3 * q + 1], Z = pts[3 * q + 2];
        /* coordinates in the frame where the polarisation is along x */
        double x = cp * X + sp * Y;
        double y = -sp * X + cp * Y;
        double G = (kind == 0) ? 1.0 : exp(-(x * x + y * y) / (w0 * w0));
        ld ph = -(ld)k * (ld)Z;
        ld sl, cl;
        sincosl(ph, &sl, &cl);
        /* psi = amp * G * e^{-ikz} */
        double pr = G * (double)(cl * amp_re - sl * amp_im);
        double pi = G * (double)(cl * amp_im + sl * amp_re);
        double e[3][2], b[3][2]; /* local frame, complex */
        if (kind == 2) {
            double kw2 = k * w0 * w0;
            double c1 = 1.0 + 2.0 / (k * kw2) - 4.0 * y * y / (kw2 * kw2);
            double c2 = 4.0 * x * y / (kw2 * kw2);
            double c3 = 2.0 * x / kw2; /* imaginary coefficient */
            e[0][0] = c1 * pr; e[0][1] = c1 * pi;
            e[1][0] = c2 * pr; e[1][1] = c2 * pi;
            e[2][0] = -c3 * pi; e[2][1] = c3 * pr;
            double c4 = -2.0 * y / kw2; /* B_z = i * c4 * psi */
            b[0][0] = 0.0; b[0][1] = 0.0;
            b[1][0] = -pr; b[1][1] = -pi;
            b[2][0] = -c4 * pi; b[2][1] = c4 * pr;
        } else {
            e[0][0] = pr; e[0][1] = pi;
            e[1][0] = 0.0; e[1][1] = 0.0;
            e[2][0] = 0.0; e[2][1] = 0.0;
            b[0][0] = 0.0; b[0][1] = 0.0;
            b[1][0] = -pr; b[1][1] = -pi;
            b[2][0] = 0.0; b[2][1] = 0.0;
        }
        /* rotate vectors back: V = Rot(pol) v */
        for (int c = 0; c < 2; ++c) {
            E[6 * q + 0 + c] = cp * e[0][c] - sp * e[1][c];
            E[6 * q + 2 + c] = sp * e[0][c] + cp * e[1][c];
            E[6 * q + 4 + c] = e[2][c];
            B[6 * q + 0 + c] = cp * b[0][c] - sp * b[1][c];
            B[6 * q + 2 + c] = sp * b[0][c] + cp * b[1][c];
            B[6 * q + 4 + c] = b[2][c];
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Laguerre-Gauss modes of the paraxial wave equation, the expansion basis of */
/* the incident beams (Sec. III-A), taken in their waist cross-section and    */
/* carried along -z without diffraction (a collimated beam, like the         */
/* Gaussians above):                                                         */
/*   u_{p,l}(r, phi) = C_{p,l} (sqrt(2) r / w0)^|l| L_p^|l|(2 r^2 / w0^2)     */
/*                     exp(-r^2 / w0^2) e^{i l phi},                         */
/*   C_{p,l} = sqrt(2 p! / (pi (p + |l|)!)) / w0,                            */
/* so that the integral of |u|^2 over the plane is 1.  L_p^a is the           */
/* generalized Laguerre polynomial, here from its explicit finite sum         */
/*   L_p^a(x) = sum_{j=0..p} (-1)^j binom(p + a, p - j) x^j / j!.            */
/* A beam is a set of modes m with indices (p_m, l_m) and complex amplitudes  */
/* ex_m, ey_m of its x- and y-polarised parts:                               */
/*   E = amp e^{-ikz} sum_m (ex_m x^ + ey_m y^) u_m,                          */
/*   B = (-z^) x E = amp e^{-ikz} sum_m (ey_m x^ - ex_m y^) u_m.              */
/* pl: [n_modes][2] ints (p, l); exy: [n_modes][4] doubles (ex re, im, ey re, im). */
/* ------------------------------------------------------------------------ */
static ld laguerre_sum(int p, int a, ld x)
{
    ld s = 0.0L;
    for (int j = 0; j <= p; ++j) {
        /* binom(p + a, p - j) = (p + a)! / ((p - j)! (a + j)!) */
        ld b = expl(lgammal((ld)(p + a + 1)) - lgammal((ld)(p - j + 1)) - lgammal((ld)(a + j + 1)));
        ld term = b * powl(x, (ld)j) / expl(lgammal((ld)(j + 1)));
        s += (j % 2) ? -term : term;
    }
    return s;
}

int orc_incident_lg(int n_modes, const int *pl, const double *exy, double w0, int n_pts, const double *pts,
                    double k, double amp_re, double amp_im, double *E, double *B)
{
    for (int q = 0; q < n_pts; ++q) {
        ld X = pts[3 * q], Y = pts[3 * q + 1], Z = pts[3 * q + 2];
        ld r = sqrtl(X * X + Y * Y), phi = atan2l(Y, X);
        ld ex_re = 0, ex_im = 0, ey_re = 0, ey_im = 0;   /* sum over modes of (ex, ey) u */
        for (int m = 0; m < n_modes; ++m) {
            int p = pl[2 * m], l = pl[2 * m + 1], al = l < 0 ? -l : l;
            ld C = sqrtl(2.0L * expl(lgammal((ld)(p + 1)) - lgammal((ld)(p + al + 1))) / PI_L) / (ld)w0;
            ld rho = sqrtl(2.0L) * r / (ld)w0;
            ld u = C * powl(rho, (ld)al) * laguerre_sum(p, al, rho * rho) * expl(-r * r / ((ld)w0 * (ld)w0));
            ld ur = u * cosl((ld)l * phi), ui = u * sinl((ld)l * phi);
            const double *c = exy + 4 * m;
            ex_re += c[0] * ur - c[1] * ui;
            ex_im += c[0] * ui + c[1] * ur;
            ey_re += c[2] * ur - c[3] * ui;
            ey_im += c[2] * ui + c[3] * ur;
        }
        /* times amp e^{-ikz} */
        ld sl, cl;
        sincosl(-(ld)k * Z, &sl, &cl);
        ld fr = cl * amp_re - sl * amp_im, fi = cl * amp_im + sl * amp_re;
        ld Exr = ex_re * fr - ex_im * fi, Exi = ex_re * fi + ex_im * fr;
        ld Eyr = ey_re * fr - ey_im * fi, Eyi = ey_re * fi + ey_im * fr;
        E[6 * q + 0] = (double)Exr; E[6 * q + 1] = (double)Exi;
        E[6 * q + 2] = (double)Eyr; E[6 * q + 3] = (double)Eyi;
        E[6 * q + 4] = 0.0;         E[6 * q + 5] = 0.0;
        B[6 * q + 0] = (double)Eyr;  B[6 * q + 1] = (double)Eyi;
        B[6 * q + 2] = -(double)Exr; B[6 * q + 3] = -(double)Exi;
        B[6 * q + 4] = 0.0;          B[6 * q + 5] = 0.0;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Small complex helpers in long double.                                     */
/* ------------------------------------------------------------------------ */
typedef struct { ld re, im; } cld;

static cld cmul(cld a, cld b) { cld r = { a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re }; return r; }
static cld cadd(cld a, cld b) { cld r = { a.re + b.re, a.im + b.im }; return r; }
static cld cscale(cld a, ld s) { cld r = { a.re * s, a.im * s }; return r; }
static cld cget(const double *p) { cld r = { (ld)p[0], (ld)p[1] }; return r; }

/* g and the scalar factor of grad g at surface point rs for observation ro:
 * returns g, sets fac = (ik - 1/R)/R * g so that grad g = fac * (rs - ro). */
static void green(ld k, const double *rs, const double *ro, ld *Rv, ld *R, cld *g, cld *fac)
{
    Rv[0] = (ld)rs[0] - (ld)ro[0];
    Rv[1] = (ld)rs[1] - (ld)ro[1];
    Rv[2] = (ld)rs[2] - (ld)ro[2];
    *R = sqrtl(Rv[0] * Rv[0] + Rv[1] * Rv[1] + Rv[2] * Rv[2]);
    ld s, c;
    sincosl(k * *R, &s, &c);
    ld inv = 1.0L / (4.0L * PI_L * *R);
    g->re = c * inv;
    g->im = s * inv;
    cld ikm = { -1.0L / *R, k };          /* ik - 1/R */
    *fac = cscale(cmul(ikm, *g), 1.0L / *R);
}

/* ------------------------------------------------------------------------ */
/* Reflected field, Stokes-converted POA form with the rim line integral.    */
/* line_term = 0 drops the line integral (used only to show that it matters). */
/* ------------------------------------------------------------------------ */
int orc_reflected_field(int n_surf, int n_rim, const double *pos, const double *nrm,
                        const double *wgt, const double *tan, int n_k, const double *kv,
                        const double *Einc, const double *Binc, int n_obs, const double *obs,
                        double *Eout, double *Bout, int line_term, int n_threads)
{
    const int n_tot = n_surf + n_rim;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1) collapse(2)
#endif
    for (int o = 0; o < n_obs; ++o) {
        for (int ik = 0; ik < n_k; ++ik) {
            const ld k = (ld)kv[ik];
            const double *ro = obs + 3 * o;
            const double *Et = Einc + (size_t)ik * n_tot * 6;
            const double *Bt = Binc + (size_t)ik * n_tot * 6;
            cld E[3] = {{0, 0}, {0, 0}, {0, 0}}, B[3] = {{0, 0}, {0, 0}, {0, 0}};
            const cld ik2 = { 0.0L, 2.0L * k };   /* 2ik */
            for (int q = 0; q < n_surf; ++q) {
                const double *n = nrm + 3 * q;
                cld Bi[3] = { cget(Bt + 6 * q), cget(Bt + 6 * q + 2), cget(Bt + 6 * q + 4) };
                cld Ei[3] = { cget(Et + 6 * q), cget(Et + 6 * q + 2), cget(Et + 6 * q + 4) };
                /* J = n~ x B_inc (without the POA factor 2, applied below) */
                cld J[3];
                J[0] = cadd(cscale(Bi[2], n[1]), cscale(Bi[1], -n[2]));
                J[1] = cadd(cscale(Bi[0], n[2]), cscale(Bi[2], -n[0]));
                J[2] = cadd(cscale(Bi[1], n[0]), cscale(Bi[0], -n[1]));
                /* rho = n~ . E_inc */
                cld rho = cadd(cadd(cscale(Ei[0], n[0]), cscale(Ei[1], n[1])), cscale(Ei[2], n[2]));
                ld Rv[3], R;
                cld g, fac;
                green(k, pos + 3 * q, ro, Rv, &R, &g, &fac);
                const ld W = (ld)wgt[q];
                /* E += W [2ik J g + 2 rho grad g] */
                cld t1 = cmul(ik2, g);
                cld t2 = cscale(cmul(rho, fac), 2.0L);
                for (int c = 0; c < 3; ++c) {
                    E[c] = cadd(E[c], cscale(cadd(cmul(J[c], t1), cscale(t2, Rv[c])), W));
                }
                /* B += W 2 J x grad g,  grad g = fac * Rv */
                cld f2 = cscale(fac, 2.0L * W);
                cld Jx[3];
                Jx[0] = cadd(cscale(J[1], Rv[2]), cscale(J[2], -Rv[1]));
                Jx[1] = cadd(cscale(J[2], Rv[0]), cscale(J[0], -Rv[2]));
                Jx[2] = cadd(cscale(J[0], Rv[1]), cscale(J[1], -Rv[0]));
                for (int c = 0; c < 3; ++c) B[c] = cadd(B[c], cmul(Jx[c], f2));
            }
            if (line_term) {
                /* -(2/ik) sum_j W_phi grad g(r_j) [n^ x (n^ x B_inc)] . t_j  */
                cld m2ik = { 0.0L, 2.0L / k };  /* -(2/ik) = 2i/k */
                for (int j = 0; j < n_rim; ++j) {
                    int q = n_surf + j;
                    const double *n = nrm + 3 * q;
                    ld nn = (ld)n[0] * n[0] + (ld)n[1] * n[1] + (ld)n[2] * n[2];
                    cld Bi[3] = { cget(Bt + 6 * q), cget(Bt + 6 * q + 2), cget(Bt + 6 * q + 4) };
                    /* n^ x (n^ x B) = n^ (n^ . B) - B  with n^ = n~/|n~| */
                    cld nB = cadd(cadd(cscale(Bi[0], n[0]), cscale(Bi[1], n[1])), cscale(Bi[2], n[2]));
                    cld b = { 0.0L, 0.0L };
                    for (int c = 0; c < 3; ++c) {
                        cld v = cadd(cscale(nB, (ld)n[c] / nn), cscale(Bi[c], -1.0L));
                        b = cadd(b, cscale(v, (ld)tan[3 * j + c]));
                    }
                    ld Rv[3], R;
                    cld g, fac;
                    green(k, pos + 3 * q, ro, Rv, &R, &g, &fac);
                    cld s = cscale(cmul(cmul(m2ik, b), fac), (ld)wgt[q]);
                    for (int c = 0; c < 3; ++c) E[c] = cadd(E[c], cscale(s, Rv[c]));
                }
            }
            size_t off = ((size_t)ik * n_obs + o) * 6;
            for (int c = 0; c < 3; ++c) {
                Eout[off + 2 * c] = (double)E[c].re;
                Eout[off + 2 * c + 1] = (double)E[c].im;
                Bout[off + 2 * c] = (double)B[c].re;
                Bout[off + 2 * c + 1] = (double)B[c].im;
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Reflected E field, double-gradient POA form (no line integral).            */
/* ------------------------------------------------------------------------ */
int orc_reflected_field_dgrad(int n_surf, const double *pos, const double *nrm, const double *wgt,
                              int n_tot, int n_k, const double *kv, const double *Binc,
                              int n_obs, const double *obs, double *Eout, int n_threads)
{
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1) collapse(2)
#endif
    for (int o = 0; o < n_obs; ++o) {
        for (int ik = 0; ik < n_k; ++ik) {
            const ld k = (ld)kv[ik];
            const double *ro = obs + 3 * o;
            const double *Bt = Binc + (size_t)ik * n_tot * 6;
            cld E[3] = {{0, 0}, {0, 0}, {0, 0}};
            for (int q = 0; q < n_surf; ++q) {
                const double *n = nrm + 3 * q;
                cld Bi[3] = { cget(Bt + 6 * q), cget(Bt + 6 * q + 2), cget(Bt + 6 * q + 4) };
                cld J[3];
                J[0] = cadd(cscale(Bi[2], n[1]), cscale(Bi[1], -n[2]));
                J[1] = cadd(cscale(Bi[0], n[2]), cscale(Bi[2], -n[0]));
                J[2] = cadd(cscale(Bi[1], n[0]), cscale(Bi[0], -n[1]));
                ld Rv[3], R;
                cld g, fac;
                green(k, pos + 3 * q, ro, Rv, &R, &g, &fac);
                ld Rh[3] = { Rv[0] / R, Rv[1] / R, Rv[2] / R };
                /* a1 = -(1/R^2 - ik/R) g ;  a2 = (3/R^2 - 3ik/R - k^2) g */
                cld c1 = { -1.0L / (R * R), k / R };
                cld a1 = cmul(c1, g);
                cld c2 = { 3.0L / (R * R) - k * k, -3.0L * k / R };
                cld a2 = cmul(c2, g);
                cld RJ = cadd(cadd(cscale(J[0], Rh[0]), cscale(J[1], Rh[1])), cscale(J[2], Rh[2]));
                cld ikg = cmul((cld){ 0.0L, k }, g);
                cld iok = { 0.0L, 1.0L / k };
                const ld W2 = 2.0L * (ld)wgt[q];
                for (int c = 0; c < 3; ++c) {
                    cld dd = cadd(cmul(a1, J[c]), cscale(cmul(a2, RJ), Rh[c]));
                    cld term = cadd(cmul(ikg, J[c]), cmul(iok, dd));
                    E[c] = cadd(E[c], cscale(term, W2));
                }
            }
            size_t off = ((size_t)ik * n_obs + o) * 6;
            for (int c = 0; c < 3; ++c) {
                Eout[off + 2 * c] = (double)E[c].re;
                Eout[off + 2 * c + 1] = (double)E[c].im;
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Semi-discrete transform to time: Ft[m][x] = sum_n F[n][x] e^{-i k_n t_m} dk */
/* F: [n_k][n_x] complex, Ft: [n_t][n_x] complex.                             */
/* ------------------------------------------------------------------------ */
int orc_time_transform(int n_k, const double *kv, double dk, int n_t, const double *t,
                       long n_x, const double *F, double *Ft, int n_threads)
{
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(static)
#endif
    for (int m = 0; m < n_t; ++m) {
        for (long x = 0; x < n_x; ++x) {
            cld acc = { 0.0L, 0.0L };
            for (int n = 0; n < n_k; ++n) {
                /* the phase -k t formed in quad precision (the product of two doubles is exact
                   there) and reduced by 2 pi in quad precision, then the long-double sincos:
                   k t reaches ~1e6 rad, where a long-double product would already be off by
                   ~1e-13 rad */
                qd ph = -(qd)kv[n] * (qd)t[m];
                qd red = ph - TWO_PI_Q * rintq(ph / TWO_PI_Q);
                ld s, c;
                sincosl((ld)red, &s, &c);
                cld tw = { c, s };
                acc = cadd(acc, cmul(cget(F + 2 * ((size_t)n * n_x + x)), tw));
            }
            Ft[2 * ((size_t)m * n_x + x)] = (double)(acc.re * (ld)dk);
            Ft[2 * ((size_t)m * n_x + x) + 1] = (double)(acc.im * (ld)dk);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Power of each frequency component of the incident beam through the mirror */
/* aperture (Sec. III-B): P_n = 4 pi SS Re(E_n x B_n^*) . dA with dA = -z    */
/* dx dy, the beam travelling along -z.  A surface node's share of the       */
/* aperture is the z component of its n dS = n~ W: on the paraboloid n~_z = 1 */
/* and W = w_r r dphi is the quadrature of the aperture disk, so             */
/*   P_n = 4 pi sum_q (n~_z W)_q [ -Re(E_x B_y^*) + Re(E_y B_x^*) ]          */
/* over the n_surf surface nodes (rim nodes carry the line term only).       */
/* E, B: [n_k][n_tot][3] complex; P: [n_k].                                   */
/* ------------------------------------------------------------------------ */
int orc_incident_power(int n_k, int n_surf, int n_tot, const double *nrm, const double *wgt, const double *E,
                       const double *B, double *P)
{
    for (int n = 0; n < n_k; ++n) {
        ld acc = 0.0L;
        for (int q = 0; q < n_surf; ++q) {
            const double *e = E + 6 * ((size_t)n * n_tot + q), *b = B + 6 * ((size_t)n * n_tot + q);
            /* (E x B^*)_z = E_x B_y^* - E_y B_x^*;  Re(a b^*) = a.re b.re + a.im b.im */
            ld sz = ((ld)e[0] * b[2] + (ld)e[1] * b[3]) - ((ld)e[2] * b[0] + (ld)e[3] * b[1]);
            acc += (ld)wgt[q] * (ld)nrm[3 * q + 2] * (-sz);
        }
        P[n] = (double)(4.0L * PI_L * acc);
    }
    return 0;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
