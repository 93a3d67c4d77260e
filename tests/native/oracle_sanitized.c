/*
 * oracle_sanitized.c -- drives every entry point of the CPU oracle once, on
 * small inputs in buffers of exactly the documented sizes, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_oracle_sanitized.py
 * compiles it together with oracle/sc_oracle.c).  Any out-of-bounds access,
 * use of freed memory, leak or undefined operation aborts the run; the checks
 * below only confirm that each call returned and produced finite numbers.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int orc_gauss_legendre(int n, double *x, double *w);
int orc_mirror(int kind, double f, double a, int n_r, int n_phi, double *pos, double *nrm, double *wgt,
               double *tan);
int orc_incident(int kind, int n_pts, const double *pts, double k, double w0, double pol, double amp_re,
                 double amp_im, double *E, double *B);
int orc_incident_lg(int n_modes, const int *pl, const double *exy, double w0, int n_pts, const double *pts,
                    double k, double amp_re, double amp_im, double *E, double *B);
int orc_reflected_field(int n_surf, int n_rim, const double *pos, const double *nrm, const double *wgt,
                        const double *tan, int n_k, const double *kv, const double *Einc, const double *Binc,
                        int n_obs, const double *obs, double *Eout, double *Bout, int line_term, int n_threads);
int orc_reflected_field_dgrad(int n_surf, const double *pos, const double *nrm, const double *wgt, int n_tot,
                              int n_k, const double *kv, const double *Binc, int n_obs, const double *obs,
                              double *Eout, int n_threads);
int orc_time_transform(int n_k, const double *kv, double dk, int n_t, const double *t, long n_x, const double *F,
                       double *Ft, int n_threads);
int orc_incident_power(int n_k, int n_surf, int n_tot, const double *nrm, const double *wgt, const double *E,
                       const double *B, double *P);

static int failures = 0;

static double *alloc(size_t n)
{
    double *p = (double *)malloc(sizeof(double) * (n ? n : 1));
    if (!p) {
        fprintf(stderr, "allocation failed\n");
        exit(2);
    }
    return p;
}

static void check_finite(const char *what, const double *v, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) {
            fprintf(stderr, "%s: element %zu is not finite\n", what, i);
            ++failures;
            return;
        }
}

static void check_rc(const char *what, int rc, int want)
{
    if (rc != want) {
        fprintf(stderr, "%s: returned %d, expected %d\n", what, rc, want);
        ++failures;
    }
}

int main(void)
{
    /* Gauss-Legendre rule; invalid order */
    for (int n = 1; n <= 9; n += 4) {
        double *x = alloc(n), *w = alloc(n);
        check_rc("gauss_legendre", orc_gauss_legendre(n, x, w), 0);
        check_finite("gauss_legendre", w, n);
        free(x);
        free(w);
    }
    check_rc("gauss_legendre n=0", orc_gauss_legendre(0, NULL, NULL), -1);

    /* mirrors: paraboloid and flat disk; invalid parameters */
    const int n_r = 6, n_phi = 5, n_tot = (n_r + 1) * n_phi, n_surf = n_r * n_phi;
    double *pos = alloc(3 * n_tot), *nrm = alloc(3 * n_tot), *wgt = alloc(n_tot), *tan = alloc(3 * n_phi);
    check_rc("mirror flat", orc_mirror(1, 0.0, 3.0, n_r, n_phi, pos, nrm, wgt, tan), 0);
    check_rc("mirror paraboloid", orc_mirror(0, 2.0, 3.0, n_r, n_phi, pos, nrm, wgt, tan), 0);
    check_finite("mirror pos", pos, 3 * n_tot);
    check_finite("mirror tan", tan, 3 * n_phi);
    check_rc("mirror n_r=0", orc_mirror(0, 2.0, 3.0, 0, n_phi, pos, nrm, wgt, tan), -1);

    /* incident fields of every kind on the nodes, at two frequencies */
    const int n_k = 2;
    const double kv[2] = {6.2831853071795862, 7.5};
    double *Ei = alloc(6 * (size_t)n_k * n_tot), *Bi = alloc(6 * (size_t)n_k * n_tot);
    for (int kind = 0; kind <= 6; ++kind)
        for (int j = 0; j < n_k; ++j)
            orc_incident(kind, n_tot, pos, kv[j], 1.5, 0.3, 1.0, -0.5, Ei + 6 * (size_t)j * n_tot,
                         Bi + 6 * (size_t)j * n_tot);
    check_finite("incident E", Ei, 6 * (size_t)n_k * n_tot);
    const int pl[4] = {0, 0, 2, -1};
    const double exy[8] = {1.0, 0.0, 0.0, 0.0, 0.3, 0.1, -0.2, 0.4};
    double *El = alloc(6 * (size_t)n_tot), *Bl = alloc(6 * (size_t)n_tot);
    orc_incident_lg(2, pl, exy, 1.5, n_tot, pos, kv[0], 1.0, 0.0, El, Bl);
    check_finite("incident LG B", Bl, 6 * (size_t)n_tot);

    /* reflected field in both forms, one and two threads */
    const int n_obs = 3;
    const double obs[9] = {0.0, 0.0, 0.0, 0.1, -0.05, 0.02, 0.0, 0.2, -0.1};
    double *Eo = alloc(6 * (size_t)n_k * n_obs), *Bo = alloc(6 * (size_t)n_k * n_obs);
    for (int th = 1; th <= 2; ++th)
        for (int line = 0; line <= 1; ++line)
            check_rc("reflected_field",
                     orc_reflected_field(n_surf, n_phi, pos, nrm, wgt, tan, n_k, kv, Ei, Bi, n_obs, obs, Eo, Bo,
                                         line, th),
                     0);
    check_finite("reflected E", Eo, 6 * (size_t)n_k * n_obs);
    check_finite("reflected B", Bo, 6 * (size_t)n_k * n_obs);
    check_rc("reflected_field_dgrad",
             orc_reflected_field_dgrad(n_surf, pos, nrm, wgt, n_tot, n_k, kv, Bi, n_obs, obs, Eo, 2), 0);
    check_finite("dgrad E", Eo, 6 * (size_t)n_k * n_obs);

    /* time transform of the reflected field, incident power */
    const int n_t = 4;
    const double t[4] = {-1.0, 0.0, 0.5, 2.0};
    double *Ft = alloc(2 * (size_t)n_t * 3 * n_obs);
    check_rc("time_transform", orc_time_transform(n_k, kv, 0.25, n_t, t, 3L * n_obs, Eo, Ft, 2), 0);
    check_finite("time samples", Ft, 2 * (size_t)n_t * 3 * n_obs);
    double P[2];
    check_rc("incident_power", orc_incident_power(n_k, n_surf, n_tot, nrm, wgt, Ei, Bi, P), 0);
    check_finite("power", P, 2);

    free(pos);
    free(nrm);
    free(wgt);
    free(tan);
    free(Ei);
    free(Bi);
    free(El);
    free(Bl);
    free(Eo);
    free(Bo);
    free(Ft);
    if (failures) return 1;
    printf("oracle entry points clean under the sanitizers\n");
    return 0;
}
