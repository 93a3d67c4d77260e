// sc_kernels.hip -- gfx950 kernels of the Stratton-Chu mirror-focusing path.
//
//  k_node_tables         mirror nodes, normals, weights            (Sec. III-C)
//  k_obs_prep            observation records
//  k_tables_from_fields  POA current / charge tables from given E_inc, B_inc
//  k_tables_gaussian     same for the built-in collimated beams: linearly, radially or
//                        azimuthally polarised Gaussian (Sec. III-A, IV-A)
//  k_tables_cast         FP64 tables -> FP32 (split: as is; naive: node phase removed)
//  k_tables_factor       FP64 tables -> factored FP32 / FP64 tables J~ = u s, when the current
//                        of every node keeps one real direction over the frequencies, and
//                        the real beta of the charge tied to it, rho_t = -i beta s / k
//  k_power_*             incident power per frequency through the aperture (Sec. III-B)
//  k_tables_scale        spectral amplitude / phase applied to the tables (Sec. III-B)
//  k_reduce<MODE>        deterministic split-K reduction into E, B
//  (the quadrature kernel itself is in sc_quad.hip)
//  k_twiddles, k_time    semi-discrete transform to time (Sec. III-B)
//
// All floating-point expressions are written with explicit fma/mul/add and
// the file is compiled with -ffp-contract=off, so the rounding sequence of
// every observation point is fixed by the source: results do not depend on
// the launch shape, only on the chunking.
#include "sc_device.h"
#include "sc_internal.h"

namespace sc {

// ======================================================================= prep

__global__ void k_node_tables(int n_r, int n_phi, double f, const double *__restrict__ r,
                              const double *__restrict__ wr, const double *__restrict__ cphi,
                              const double *__restrict__ sphi, double dphi, double *__restrict__ pos64,
                              float *__restrict__ pos32, double *__restrict__ nrm, double *__restrict__ wgt,
                              double *__restrict__ tan)
{
    const int n_tot = (n_r + 1) * n_phi;
    const int64_t gq = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gq >= n_tot) return;
    const int q = (int)gq;
    const int i = q / n_phi;
    const int j = q - i * n_phi;
    const bool rim = (i == n_r);
    const double ri = r[i];            // r has n_r + 1 entries; r[n_r] = r_max
    const double c = cphi[j], s = sphi[j];
    const double x = ri * c;
    const double y = ri * s;
    const double z = ri * ri / (4.0 * f) - f;
    const dd rs = dd_norm3(x, y, z);
    pos64[4 * q + 0] = x;
    pos64[4 * q + 1] = y;
    pos64[4 * q + 2] = z;
    pos64[4 * q + 3] = rs.hi;
    pos32[4 * q + 0] = (float)x;
    pos32[4 * q + 1] = (float)y;
    pos32[4 * q + 2] = (float)z;
    pos32[4 * q + 3] = (float)rs.hi;
    // d r_s/dr x d r_s/dphi = r (-F'(r) cos, -F'(r) sin, 1), F'(r) = r / 2f
    const double dFdr = ri / (2.0 * f);
    nrm[3 * q + 0] = -dFdr * c;
    nrm[3 * q + 1] = -dFdr * s;
    nrm[3 * q + 2] = 1.0;
    wgt[q] = rim ? dphi : wr[i] * ri * dphi;
    if (rim) {
        tan[3 * j + 0] = -ri * s;
        tan[3 * j + 1] = ri * c;
        tan[3 * j + 2] = 0.0;
    }
}

// Node records of a general surface given by its quadrature: surface nodes with
// their area-weighted normals n dS (weight 1), then the boundary nodes with the
// surface normal there (direction only), weight 1 and the oriented line
// element dl in `tan`.
__global__ void k_surface_records(int n_surf, int n_rim, const double *__restrict__ xyz,
                                  const double *__restrict__ ndS, const double *__restrict__ rim_xyz,
                                  const double *__restrict__ rim_n, const double *__restrict__ rim_dl,
                                  double *__restrict__ pos64, float *__restrict__ pos32, double *__restrict__ nrm,
                                  double *__restrict__ wgt, double *__restrict__ tan)
{
    const int64_t gq = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gq >= (int64_t)n_surf + n_rim) return;
    const int q = (int)gq;
    const bool rim = q >= n_surf;
    const int j = q - n_surf;
    const double *src = rim ? rim_xyz + 3 * j : xyz + 3 * q;
    const double *nv = rim ? rim_n + 3 * j : ndS + 3 * q;
    const double x = src[0], y = src[1], z = src[2];
    const dd rs = dd_norm3(x, y, z);
    pos64[4 * q + 0] = x;
    pos64[4 * q + 1] = y;
    pos64[4 * q + 2] = z;
    pos64[4 * q + 3] = rs.hi;
    pos32[4 * q + 0] = (float)x;
    pos32[4 * q + 1] = (float)y;
    pos32[4 * q + 2] = (float)z;
    pos32[4 * q + 3] = (float)rs.hi;
    for (int c = 0; c < 3; ++c) nrm[3 * q + c] = nv[c];
    wgt[q] = 1.0;
    if (rim)
        for (int c = 0; c < 3; ++c) tan[3 * j + c] = rim_dl[3 * j + c];
}

// 1 / (2|r_s|) per node in FP64 and FP32, for the series forms of delta and
// 1/|R| in the split quadrature (0 for a node at the origin, where the series
// is never used).
__global__ void k_node_half_inverse(int n_tot, const double *__restrict__ pos64, double *__restrict__ hinv64,
                                    float *__restrict__ hinv32)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_tot) return;
    const double rs = pos64[4 * q + 3];
    const double h = rs > 0.0 ? 0.5 / rs : 0.0;
    hinv64[q] = h;
    hinv32[q] = (float)h;
}

__global__ void k_obs_prep(const double *__restrict__ xyz, int n_obs, int n_obs_pad, double *__restrict__ obs64,
                           float *__restrict__ obs32)
{
    const int64_t go = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (go >= n_obs_pad) return;
    const int o = (int)go;
    const int src = (o < n_obs) ? o : 0;   // padding repeats a valid point; its result is discarded
    const double x = xyz[3 * src], y = xyz[3 * src + 1], z = xyz[3 * src + 2];
    const double r2 = __fma_rn(x, x, __fma_rn(y, y, z * z));
    obs64[4 * o + 0] = x;
    obs64[4 * o + 1] = y;
    obs64[4 * o + 2] = z;
    obs64[4 * o + 3] = r2;
    obs32[4 * o + 0] = (float)x;
    obs32[4 * o + 1] = (float)y;
    obs32[4 * o + 2] = (float)z;
    obs32[4 * o + 3] = (float)r2;
}

// complex helpers (FP64)
struct c64 {
    double re, im;
};
__device__ __forceinline__ c64 cmul(c64 a, c64 b)
{
    return {__fma_rn(a.re, b.re, -(a.im * b.im)), __fma_rn(a.re, b.im, a.im * b.re)};
}

// Write one table record from the fields at node q (without/with phase folded by caller).
// P is the node phase factor; for surface nodes uses E, B; for rim nodes B only.
__device__ __forceinline__ void write_record(double *__restrict__ rec, bool rim, double k, double W,
                                             const double *n, const double *t, const c64 *E, const c64 *B,
                                             c64 P)
{
    if (!rim) {
        // J = n~ x B_inc, rho = n~ . E_inc
        c64 J[3], rho;
        J[0] = {n[1] * B[2].re - n[2] * B[1].re, n[1] * B[2].im - n[2] * B[1].im};
        J[1] = {n[2] * B[0].re - n[0] * B[2].re, n[2] * B[0].im - n[0] * B[2].im};
        J[2] = {n[0] * B[1].re - n[1] * B[0].re, n[0] * B[1].im - n[1] * B[0].im};
        rho = {n[0] * E[0].re + n[1] * E[1].re + n[2] * E[2].re, n[0] * E[0].im + n[1] * E[1].im + n[2] * E[2].im};
        const double cJ = 2.0 * k * W / FOUR_PI;   // Jt = i cJ J P
        const double cR = 2.0 * W / FOUR_PI;       // rho_t = cR rho P
        for (int c = 0; c < 3; ++c) {
            c64 v = cmul(J[c], P);
            rec[2 * c + 0] = -cJ * v.im;
            rec[2 * c + 1] = cJ * v.re;
        }
        c64 v = cmul(rho, P);
        rec[6] = cR * v.re;
        rec[7] = cR * v.im;
    } else {
        // b = [n^ x (n^ x B)] . t = (n^ (n^ . B) - B) . t,   n^ = n~ / |n~|
        const double nn = n[0] * n[0] + n[1] * n[1] + n[2] * n[2];
        c64 nB = {n[0] * B[0].re + n[1] * B[1].re + n[2] * B[2].re, n[0] * B[0].im + n[1] * B[1].im + n[2] * B[2].im};
        c64 b = {0.0, 0.0};
        for (int c = 0; c < 3; ++c) {
            b.re += (n[c] * nB.re / nn - B[c].re) * t[c];
            b.im += (n[c] * nB.im / nn - B[c].im) * t[c];
        }
        // line term -(2/ik) sum W grad g b  ->  rho_t = i (2 W / (4 pi k)) b P
        const double cL = 2.0 * W / (FOUR_PI * k);
        c64 v = cmul(b, P);
        for (int c = 0; c < 6; ++c) rec[c] = 0.0;
        rec[6] = -cL * v.im;
        rec[7] = cL * v.re;
    }
}

__global__ void k_tables_from_fields(int n_k, int n_surf, int n_tot, const double *__restrict__ kv,
                                     const double *__restrict__ pos64, const double *__restrict__ nrm,
                                     const double *__restrict__ wgt, const double *__restrict__ tan,
                                     const double *__restrict__ Ein, const double *__restrict__ Bin,
                                     double *__restrict__ tab64)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n_k * n_tot) return;
    const int kk = (int)(idx / n_tot);
    const int q = (int)(idx - (int64_t)kk * n_tot);
    const double k = kv[kk];
    const double *p = pos64 + 4 * q;
    const dd rs = dd_norm3(p[0], p[1], p[2]);
    double sp, cp;
    sincos(phase_mod_2pi(k, rs), &sp, &cp);   // P = e^{ik|r_s|}
    c64 E[3], B[3];
    const double *e = Ein + idx * 6, *b = Bin + idx * 6;
    for (int c = 0; c < 3; ++c) {
        E[c] = {e[2 * c], e[2 * c + 1]};
        B[c] = {b[2 * c], b[2 * c + 1]};
    }
    const bool rim = q >= n_surf;
    write_record(tab64 + idx * 8, rim, k, wgt[q], nrm + 3 * q, rim ? tan + 3 * (q - n_surf) : nullptr, E, B,
                 {cp, sp});
}

// Incident collimated beams travelling along -z at node (X, Y), without their
// propagation phase e^{-ikz} (the table kernel fuses that with the node phase;
// the power kernel does not need it).  Sec. III-A.
//   beam 0, linearly polarised Gaussian, psi = amp exp(-(x^2+y^2)/w0^2) in the
//     frame where the polarisation is along x (`pol` rotates it about z):
//     literal E = x psi, B = -y psi; curl-consistent B = psi (0, -1, -2iy/(k w0^2)),
//     E = (i/k) curl B;
//   beam 1, radially polarised, g = amp exp(-r^2/w0^2) / w0:
//     E = (x, y, c) g, B = (y, -x, 0) g;
//   beam 2, azimuthally polarised: E = (-y, x, 0) g, B = (x, y, c) g;
//   with c = (2i/k)(r^2/w0^2 - 1) for the curl-consistent variants (E = (i/k) curl B,
//   resp. B = (-i/k) curl E) and c = 0 for the literal ones (B = -z x E).  The
//   cylindrical beams are axisymmetric, so `pol` does not enter;
//   beam 3, a Laguerre-Gauss mode set (lg_fields), literal.
// Laguerre-Gauss mode set (Sec. III-A: the Laguerre-Gauss modes of the paraxial wave equation are
// the expansion basis of the incident beams), each mode in its waist cross-section carried along -z:
//   u_{p,l} = C_{p,l} ((X + i sgn(l) Y) sqrt(2) / w0)^|l| L_p^|l|(2 r^2 / w0^2) exp(-r^2 / w0^2),
//   C_{p,l} = sqrt(2 p! / (pi (p + |l|)!)) / w0   (unit power over the plane),
// that is (sqrt(2) r / w0)^|l| e^{i l phi} times the radial factor, with L_p^a by its three-term
// recurrence.  modes: [n_modes][SC_LG_RECORD] = (p, l, ex re, ex im, ey re, ey im, C_{p,l}, unused),
// C from the host (it does not depend on the position; a device lgamma here cost the table
// kernels 72 VGPRs and 380 bytes of scratch per lane);
//   E = sum_m (ex_m x + ey_m y) u_m amp,   B = (-z) x E = sum_m (ey_m x - ex_m y) u_m amp.
__device__ __forceinline__ void lg_fields(const double *__restrict__ modes, int n_modes, double X, double Y,
                                          double w0, c64 amp, c64 *E, c64 *B)
{
    const double s2w = 1.4142135623730951 / w0;
    const double t = 2.0 * (X * X + Y * Y) / (w0 * w0);
    const double gauss = exp(-0.5 * t);
    c64 ex = {0.0, 0.0}, ey = {0.0, 0.0};
    for (int m = 0; m < n_modes; ++m) {
        const double *md = modes + SC_LG_RECORD * m;
        const int p = (int)md[0], l = (int)md[1], al = l < 0 ? -l : l;
        // L_p^al(t): L_0 = 1, L_1 = 1 + al - t, (n + 1) L_{n+1} = (2n + 1 + al - t) L_n - (n + al) L_{n-1}
        double l0 = 1.0, l1 = 1.0 + al - t;
        const double lag = p == 0 ? 1.0 : l1;
        for (int n = 1; n < p; ++n) {
            const double l2 = ((2.0 * n + 1.0 + al - t) * l1 - (n + al) * l0) / (n + 1.0);
            l0 = l1;
            l1 = l2;
        }
        const double L = p <= 1 ? lag : l1;
        // ((X +- iY) sqrt(2) / w0)^|l|
        const c64 z1 = {X * s2w, (l < 0 ? -Y : Y) * s2w};
        c64 zp = {1.0, 0.0};
        for (int j = 0; j < al; ++j) zp = cmul(zp, z1);
        const double radial = md[6] * L * gauss;   // md[6]: the mode's normalisation C_{p,l}
        const c64 u = {radial * zp.re, radial * zp.im};
        const c64 cx = cmul(u, {md[2], md[3]}), cy = cmul(u, {md[4], md[5]});
        ex = {ex.re + cx.re, ex.im + cx.im};
        ey = {ey.re + cy.re, ey.im + cy.im};
    }
    ex = cmul(ex, amp);
    ey = cmul(ey, amp);
    E[0] = ex;
    E[1] = ey;
    E[2] = {0.0, 0.0};
    B[0] = ey;
    B[1] = {-ex.re, -ex.im};
    B[2] = {0.0, 0.0};
}

__device__ __forceinline__ void beam_fields(int beam, double k, double X, double Y, double w0, double pol, c64 amp,
                                            int consistent, const double *modes, int n_modes, c64 *E, c64 *B)
{
    if (beam == 3) {
        lg_fields(modes, n_modes, X, Y, w0, amp, E, B);
        return;
    }
    if (beam != 0) {
        const double r2 = X * X + Y * Y;
        const double G = exp(-r2 / (w0 * w0)) / w0;
        const c64 g = {G * amp.re, G * amp.im};
        const double c = consistent ? 2.0 / k * (r2 / (w0 * w0) - 1.0) : 0.0;   // longitudinal: i c g
        const c64 lg = {-c * g.im, c * g.re};
        const c64 zero = {0.0, 0.0};
        const c64 rx = {X * g.re, X * g.im}, ry = {Y * g.re, Y * g.im};
        if (beam == 1) {
            E[0] = rx;
            E[1] = ry;
            E[2] = lg;
            B[0] = ry;
            B[1] = {-rx.re, -rx.im};
            B[2] = zero;
        } else {
            E[0] = {-ry.re, -ry.im};
            E[1] = rx;
            E[2] = zero;
            B[0] = rx;
            B[1] = ry;
            B[2] = lg;
        }
        return;
    }
    double sl, cl;
    sincos(pol, &sl, &cl);
    // frame where the polarisation is along x
    const double x = cl * X + sl * Y;
    const double y = -sl * X + cl * Y;
    const double G = exp(-(x * x + y * y) / (w0 * w0));
    const c64 psi = {G * amp.re, G * amp.im};
    c64 e[3], bb[3];
    if (consistent) {
        const double kw2 = k * w0 * w0;
        const double c1 = 1.0 + 2.0 / (k * kw2) - 4.0 * y * y / (kw2 * kw2);
        const double c2 = 4.0 * x * y / (kw2 * kw2);
        const double c3 = 2.0 * x / kw2;    // E_z = i c3 psi
        const double c4 = -2.0 * y / kw2;   // B_z = i c4 psi
        e[0] = {c1 * psi.re, c1 * psi.im};
        e[1] = {c2 * psi.re, c2 * psi.im};
        e[2] = {-c3 * psi.im, c3 * psi.re};
        bb[0] = {0.0, 0.0};
        bb[1] = {-psi.re, -psi.im};
        bb[2] = {-c4 * psi.im, c4 * psi.re};
    } else {
        e[0] = psi;
        e[1] = {0.0, 0.0};
        e[2] = {0.0, 0.0};
        bb[0] = {0.0, 0.0};
        bb[1] = {-psi.re, -psi.im};
        bb[2] = {0.0, 0.0};
    }
    E[0] = {cl * e[0].re - sl * e[1].re, cl * e[0].im - sl * e[1].im};
    E[1] = {sl * e[0].re + cl * e[1].re, sl * e[0].im + cl * e[1].im};
    E[2] = e[2];
    B[0] = {cl * bb[0].re - sl * bb[1].re, cl * bb[0].im - sl * bb[1].im};
    B[1] = {sl * bb[0].re + cl * bb[1].re, sl * bb[0].im + cl * bb[1].im};
    B[2] = bb[2];
}

__global__ void k_tables_gaussian(int n_k, int n_surf, int n_tot, const double *__restrict__ kv,
                                  const double *__restrict__ pos64, const double *__restrict__ nrm,
                                  const double *__restrict__ wgt, const double *__restrict__ tan, int beam, double w0,
                                  double pol, const double *__restrict__ spectrum, int consistent,
                                  const double *__restrict__ modes, int n_modes, double *__restrict__ tab64)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n_k * n_tot) return;
    const int kk = (int)(idx / n_tot);
    const int q = (int)(idx - (int64_t)kk * n_tot);
    const double k = kv[kk];
    const double *p = pos64 + 4 * q;
    const double X = p[0], Y = p[1], Z = p[2];
    const c64 amp = spectrum ? c64{spectrum[2 * kk], spectrum[2 * kk + 1]} : c64{1.0, 0.0};
    c64 E[3], B[3];
    beam_fields(beam, k, X, Y, w0, pol, amp, consistent, modes, n_modes, E, B);
    // propagation phase e^{-ikz} fused with the node phase e^{ik|r_s|}: e^{ik(|r_s| - z)},
    // formed in double-double so that no ~1e6 rad phase is ever rounded to double
    const dd rs = dd_norm3(X, Y, Z);
    double sp, cp;
    sincos(phase_mod_2pi(k, dd_sub_d(rs, Z)), &sp, &cp);
    const bool rim = q >= n_surf;
    write_record(tab64 + idx * 8, rim, k, wgt[q], nrm + 3 * q, rim ? tan + 3 * (q - n_surf) : nullptr, E, B,
                 {cp, sp});
}

// ------------------------------------------------------------ incident power
// Power of one frequency component of the incident beam through the mirror
// aperture (Sec. III-B, the Poynting integral that fixes each component's
// energy):  P_n = 4 pi SS Re(E_n x B_n^*) . dA  with dA = -z dx dy, since the
// beam travels along -z.  The surface weights W = w_r r dphi integrate over the
// aperture disk in the (x, y) plane, so P_n = 4 pi sum_q W_q Re(E x B^*) . (-z)
// over the surface nodes; for a general surface the aperture element of a node
// is the z component of its n dS, (n~ W).z (n~.z = 1 on the paraboloid).
// Deterministic: block b of frequency k sums a fixed node range in a fixed
// order; k_power_finish adds the blocks in order.
constexpr int POWER_BLOCKS = 16;

__device__ __forceinline__ double flux_minus_z(const c64 *E, const c64 *B)
{
    // Re(E x B^*)_z = Re(E_x B_y^*) - Re(E_y B_x^*)
    return -((E[0].re * B[1].re + E[0].im * B[1].im) - (E[1].re * B[0].re + E[1].im * B[0].im));
}

__device__ __forceinline__ void block_sum_256(double v, double *out)
{
    __shared__ double red[256];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// grid (POWER_BLOCKS, n_k), 256 threads; E, B: [n_k][n_tot][3] complex
__global__ void __launch_bounds__(256) k_power_fields(int n_surf, int n_tot, const double *__restrict__ nrm,
                                                      const double *__restrict__ wgt,
                                                      const double *__restrict__ Ein,
                                                      const double *__restrict__ Bin, double *__restrict__ part)
{
    const int kk = blockIdx.y;
    const int span = (n_surf + POWER_BLOCKS - 1) / POWER_BLOCKS;
    const int q0 = blockIdx.x * span, q1 = min(q0 + span, n_surf);
    double acc = 0.0;
    for (int q = q0 + (int)threadIdx.x; q < q1; q += 256) {
        const double *e = Ein + ((size_t)kk * n_tot + q) * 6, *b = Bin + ((size_t)kk * n_tot + q) * 6;
        c64 E[3], B[3];
        for (int c = 0; c < 3; ++c) {
            E[c] = {e[2 * c], e[2 * c + 1]};
            B[c] = {b[2 * c], b[2 * c + 1]};
        }
        acc += (nrm[3 * q + 2] * wgt[q]) * flux_minus_z(E, B);
    }
    block_sum_256(acc, part + (size_t)kk * POWER_BLOCKS + blockIdx.x);
}

__global__ void __launch_bounds__(256) k_power_gaussian(int n_surf, const double *__restrict__ kv,
                                                        const double *__restrict__ pos64,
                                                        const double *__restrict__ nrm,
                                                        const double *__restrict__ wgt, int beam, double w0,
                                                        double pol,
                                                        const double *__restrict__ spectrum, int consistent,
                                                        const double *__restrict__ modes, int n_modes,
                                                        double *__restrict__ part)
{
    const int kk = blockIdx.y;
    const int span = (n_surf + POWER_BLOCKS - 1) / POWER_BLOCKS;
    const int q0 = blockIdx.x * span, q1 = min(q0 + span, n_surf);
    const double k = kv[kk];
    const c64 amp = spectrum ? c64{spectrum[2 * kk], spectrum[2 * kk + 1]} : c64{1.0, 0.0};
    double acc = 0.0;
    for (int q = q0 + (int)threadIdx.x; q < q1; q += 256) {
        c64 E[3], B[3];
        beam_fields(beam, k, pos64[4 * q], pos64[4 * q + 1], w0, pol, amp, consistent, modes, n_modes, E, B);
        acc += (nrm[3 * q + 2] * wgt[q]) * flux_minus_z(E, B);
    }
    block_sum_256(acc, part + (size_t)kk * POWER_BLOCKS + blockIdx.x);
}

__global__ void k_power_finish(int n_k, const double *__restrict__ part, double *__restrict__ P)
{
    const int64_t gk = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gk >= n_k) return;
    const int kk = (int)gk;
    double s = 0.0;
    for (int b = 0; b < POWER_BLOCKS; ++b) s += part[(size_t)kk * POWER_BLOCKS + b];
    P[kk] = FOUR_PI * s;
}

// Multiply every record of frequency k by the complex factor fac[k] (spectral
// amplitude and phase, Sec. III-B); tab64 in FP64, or tab32 (FP32 storage).
// n_cplx complex numbers per (k, node) record: 4 for the general tables, 2 for the factored ones (s, rho_t).
__global__ void k_tables_scale(int n_k, int n_tot, int n_cplx, const double *__restrict__ fac,
                               double *__restrict__ tab64, float *__restrict__ tab32)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n_k * n_tot) return;
    const int kk = (int)(idx / n_tot);
    const c64 f = {fac[2 * kk], fac[2 * kk + 1]};
    const int64_t base = idx * 2 * n_cplx;
    for (int c = 0; c < n_cplx; ++c) {
        if (tab64) {
            const c64 v = cmul({tab64[base + 2 * c], tab64[base + 2 * c + 1]}, f);
            tab64[base + 2 * c] = v.re;
            tab64[base + 2 * c + 1] = v.im;
        } else {
            const c64 v = cmul({(double)tab32[base + 2 * c], (double)tab32[base + 2 * c + 1]}, f);
            tab32[base + 2 * c] = (float)v.re;
            tab32[base + 2 * c + 1] = (float)v.im;
        }
    }
}

__global__ void k_tables_cast(int n_k, int n_tot, const double *__restrict__ kv, const double *__restrict__ pos64,
                              const double *__restrict__ tab64, const float *__restrict__ src32,
                              float *__restrict__ tab32, int naive)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n_k * n_tot) return;
    double v[8];
    for (int c = 0; c < 8; ++c) v[c] = tab64 ? tab64[idx * 8 + c] : (double)src32[idx * 8 + c];
    float *dst = tab32 + idx * 8;
    if (!naive) {
        for (int c = 0; c < 8; ++c) dst[c] = (float)v[c];
        return;
    }
    // remove the folded node phase: multiply by e^{-ik|r_s|}
    const int kk = (int)(idx / n_tot);
    const int q = (int)(idx - (int64_t)kk * n_tot);
    const double *p = pos64 + 4 * q;
    const dd rs = dd_norm3(p[0], p[1], p[2]);
    double sp, cp;
    sincos(phase_mod_2pi(kv[kk], rs), &sp, &cp);
    const c64 P = {cp, -sp};
    for (int c = 0; c < 4; ++c) {
        c64 w = cmul({v[2 * c], v[2 * c + 1]}, P);
        dst[2 * c] = (float)w.re;
        dst[2 * c + 1] = (float)w.im;
    }
}

// Factored tables.  The surface current of the integrand (Sec. II: J = n x B,
// folded into Jt with the weights and the node phase) often keeps one real
// direction at every frequency (e.g. a linearly polarised Gaussian with any
// spectrum, or a radially or azimuthally polarised beam): then
// Jt[k][q] = u_q s[k][q] and the quadrature can use u_q and s.  One thread per
// node q: u_q is the unit vector along the longer of Re Jt, Im Jt at the
// frequency kb where |Jt[k][q]| is largest (u_q = 0 if Jt vanishes), s = u_q . Jt.
// Often the charge is tied to that current as well: when E and B of the beam
// share one complex amplitude, n . E and n x B carry the same s, and with
// rho_t = (2W / 4 pi) (n . E) P against Jt = i k (2W / 4 pi) (n x B) P,
//   rho_t[k][q] = -i beta_q s[k][q] / k   with beta_q real,
// beta_q = k (Re rho_t Im s - Im rho_t Re s) / |s|^2 at kb.  A node without current
// (the rim, whose line term is a charge only) takes u_q = 0, beta_q = 1 and
// s = i k rho_t, which ties its charge exactly and leaves Jt = u s = 0.
// Bit 0 of *bad is set if |Jt[k][q] - u_q s[k][q]| > tol32 max_k |Jt[k][q]| for any
// node and k, bit 1 if it exceeds tol64; bits 2 and 3 the same for
// |rho_t[k][q] + i beta_q s[k][q] / k| against max_k (|rho_t[k][q]|^2 + |Jt[k][q] / k|^2)^1/2,
// the node's scale of the charge term (a charge that vanishes but for rounding, as
// n . E of the azimuthally polarised beam does, is tied with beta = 0).  The tables of a
// precision must not be used when its bit is set.  Outputs, each optional (NULL
// skips it): FP32 tabf[k][q] = (s, rho_t), posf[q] = (x, y, z, |r_s|, u_q, 1 / (2|r_s|)),
// betaf[q] = beta_q and tabp[k][q] = (|s|, arg(s) / 2 pi), s in polar form for the tied
// charge (the turn in (-1/2, 1/2]); FP64 tabf64, posf64 and betaf64, the same in double.
__global__ void k_tables_factor(int n_k, int n_tot, const double *__restrict__ kv, const double *__restrict__ tab64,
                                const float *__restrict__ pos32, const double *__restrict__ pos64, double tol32,
                                double tol64, float *__restrict__ tabf, float *__restrict__ posf,
                                float *__restrict__ betaf, float *__restrict__ tabp, double *__restrict__ tabf64,
                                double *__restrict__ posf64, double *__restrict__ betaf64,
                                unsigned int *__restrict__ bad)
{
    const int64_t gq = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gq >= n_tot) return;
    double best = 0.0, bestr = 0.0;
    int kb = 0;
    for (int kk = 0; kk < n_k; ++kk) {
        const double *v = tab64 + ((int64_t)kk * n_tot + gq) * 8;
        double m = 0.0;
        for (int c = 0; c < 6; ++c) m += v[c] * v[c];
        if (m > best) {
            best = m;
            kb = kk;
        }
        const double k = kv[kk];
        bestr = fmax(bestr, v[6] * v[6] + v[7] * v[7] + m / (k * k));
    }
    double u[3] = {0.0, 0.0, 0.0};
    double beta = 1.0;
    if (best > 0.0) {
        const double *v = tab64 + ((int64_t)kb * n_tot + gq) * 8;
        const double re2 = v[0] * v[0] + v[2] * v[2] + v[4] * v[4];
        const double im2 = v[1] * v[1] + v[3] * v[3] + v[5] * v[5];
        const int part = re2 >= im2 ? 0 : 1;
        const double inv = 1.0 / sqrt(part ? im2 : re2);
        for (int c = 0; c < 3; ++c) u[c] = v[2 * c + part] * inv;
        const double sr = u[0] * v[0] + u[1] * v[2] + u[2] * v[4];
        const double si = u[0] * v[1] + u[1] * v[3] + u[2] * v[5];
        const double s2 = sr * sr + si * si;
        beta = s2 > 0.0 ? kv[kb] * (v[6] * si - v[7] * sr) / s2 : 0.0;
    }
    const double lim32 = tol32 * tol32 * best, lim64 = tol64 * tol64 * best;
    const double rlim32 = tol32 * tol32 * bestr, rlim64 = tol64 * tol64 * bestr;
    unsigned int flags = 0;
    for (int kk = 0; kk < n_k; ++kk) {
        const int64_t rec = (int64_t)kk * n_tot + gq;
        const double *v = tab64 + rec * 8;
        const double k = kv[kk];
        double sr, si;
        if (best > 0.0) {
            sr = u[0] * v[0] + u[1] * v[2] + u[2] * v[4];
            si = u[0] * v[1] + u[1] * v[3] + u[2] * v[5];
        } else {   // s = i k rho_t
            sr = -k * v[7];
            si = k * v[6];
        }
        double r2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            const double dr = v[2 * c] - u[c] * sr, di = v[2 * c + 1] - u[c] * si;
            r2 += dr * dr + di * di;
        }
        if (!(r2 <= lim32)) flags |= 1u;
        if (!(r2 <= lim64)) flags |= 2u;
        // rho_t + i beta s / k
        const double tr = v[6] - beta * si / k, ti = v[7] + beta * sr / k;
        const double t2 = tr * tr + ti * ti;
        if (!(t2 <= rlim32)) flags |= 4u;
        if (!(t2 <= rlim64)) flags |= 8u;
        if (tabf) {
            float *t = tabf + rec * 4;
            t[0] = (float)sr;
            t[1] = (float)si;
            t[2] = (float)v[6];
            t[3] = (float)v[7];
            tabp[rec * 2] = (float)sqrt(sr * sr + si * si);
            tabp[rec * 2 + 1] = (float)(atan2(si, sr) * INV_TWO_PI);
        }
        if (tabf64) {
            double *t = tabf64 + rec * 4;
            t[0] = sr;
            t[1] = si;
            t[2] = v[6];
            t[3] = v[7];
        }
    }
    if (posf) {
        float *pr = posf + gq * 8;
        for (int c = 0; c < 4; ++c) pr[c] = pos32[gq * 4 + c];
        for (int c = 0; c < 3; ++c) pr[4 + c] = (float)u[c];
        pr[7] = pos64[gq * 4 + 3] > 0.0 ? (float)(0.5 / pos64[gq * 4 + 3]) : 0.0f;   // 1 / (2 |r_s|)
        betaf[gq] = (float)beta;
    }
    if (posf64) {
        double *pr = posf64 + gq * 8;
        for (int c = 0; c < 4; ++c) pr[c] = pos64[gq * 4 + c];
        for (int c = 0; c < 3; ++c) pr[4 + c] = u[c];
        pr[7] = pos64[gq * 4 + 3] > 0.0 ? 0.5 / pos64[gq * 4 + 3] : 0.0;   // 1 / (2 |r_s|)
        betaf64[gq] = beta;
    }
    if (flags) atomicOr(bad, flags);
}

// The polar records of the tied charge again from the FP32 factored records, after these were
// scaled in place (a spectral factor on FP32-only tables): tabp[r] = (|s|, arg(s) / 2 pi).
__global__ void k_tables_polar(int64_t n_rec, const float *__restrict__ tabf, float *__restrict__ tabp)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rec) return;
    const double sr = tabf[r * 4], si = tabf[r * 4 + 1];
    tabp[r * 2] = (float)sqrt(sr * sr + si * si);
    tabp[r * 2 + 1] = (float)(atan2(si, sr) * INV_TWO_PI);
}

// Split-K reduction: E[k][o][c] = sum over chunks (in FP64, fixed order); B gets the 1/(ik) factor,
// or 1/i where the quadrature's B sums already carry 1/k (b_over_k).
template <typename PT, typename OT>
__global__ void k_reduce(const PT *__restrict__ partial, int n_chunks, int n_k, int n_obs, int n_obs_pad,
                         const double *__restrict__ kv, int b_over_k, OT *__restrict__ E, OT *__restrict__ B)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n_k * n_obs) return;
    const int kk = (int)(idx / n_obs);
    const int o = (int)(idx - (int64_t)kk * n_obs);
    double acc[12];
    for (int c = 0; c < 12; ++c) acc[c] = 0.0;
    for (int ch = 0; ch < n_chunks; ++ch) {
        // partials [chunk][k][point / 64][12][64]
        const PT *p = partial + ((size_t)ch * n_k + kk) * 12 * (size_t)n_obs_pad + (size_t)(o >> 6) * 768 + (o & 63);
        for (int c = 0; c < 12; ++c) acc[c] += (double)p[c * 64];
    }
    const double ik_inv = b_over_k ? 1.0 : 1.0 / kv[kk];   // 1/(ik) = -i/k
    OT *e = E + idx * 6, *b = B + idx * 6;
    for (int c = 0; c < 3; ++c) {
        e[2 * c] = (OT)acc[2 * c];
        e[2 * c + 1] = (OT)acc[2 * c + 1];
        b[2 * c] = (OT)(acc[6 + 2 * c + 1] * ik_inv);
        b[2 * c + 1] = (OT)(-acc[6 + 2 * c] * ik_inv);
    }
}

// ================================================================ time transform

// tw[m][n] = dk * e^{-i k_n t_m}, phase formed in double-double and reduced mod 2pi.
__global__ void k_twiddles(int n_k, const double *__restrict__ kv, int n_t, const double *__restrict__ t, double dk,
                           double *__restrict__ tw)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n_k * n_t) return;
    const int m = (int)(idx / n_k), n = (int)(idx - (int64_t)m * n_k);
    double s, c;
    sincos(phase_mod_2pi(kv[n], dd{-t[m], 0.0}), &s, &c);
    tw[2 * idx] = dk * c;
    tw[2 * idx + 1] = dk * s;
}

// Constant-address-space view: wave-uniform loads through it become scalar loads.
typedef __attribute__((address_space(4))) const double cdouble;

constexpr int TIME_MT = 8;   // time samples per thread (register tile)

// Ft[m][x] = sum_n F[n][x] tw[m][n], accumulated in FP64.  The twiddle rows
// are wave-uniform and read through scalar loads.
template <typename T>
__global__ void __launch_bounds__(256) k_time(int n_k, int n_t, int64_t n_x, const double *__restrict__ tw_,
                                              const T *__restrict__ F, T *__restrict__ Ft)
{
    cdouble *tw = (cdouble *)tw_;
    const int m0 = blockIdx.y * TIME_MT;
    const int mt = min(TIME_MT, n_t - m0);
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n_x) return;
    double ar[TIME_MT], ai[TIME_MT];
#pragma unroll
    for (int mm = 0; mm < TIME_MT; ++mm) ar[mm] = ai[mm] = 0.0;
    for (int n = 0; n < n_k; ++n) {
        const double fr = (double)F[2 * ((size_t)n * n_x + x)];
        const double fi = (double)F[2 * ((size_t)n * n_x + x) + 1];
#pragma unroll
        for (int mm = 0; mm < TIME_MT; ++mm) {
            const int m = min(m0 + mm, n_t - 1);
            const double wr = tw[((size_t)m * n_k + n) * 2], wi = tw[((size_t)m * n_k + n) * 2 + 1];
            ar[mm] = __fma_rn(fr, wr, __fma_rn(-fi, wi, ar[mm]));
            ai[mm] = __fma_rn(fr, wi, __fma_rn(fi, wr, ai[mm]));
        }
    }
    for (int mm = 0; mm < mt; ++mm) {
        Ft[2 * ((size_t)(m0 + mm) * n_x + x)] = (T)ar[mm];
        Ft[2 * ((size_t)(m0 + mm) * n_x + x) + 1] = (T)ai[mm];
    }
}

__global__ void k_fill_u32(unsigned int *p, unsigned int v, int n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// One quadrature job written to device memory from a kernel argument (no host buffer to keep alive).
__global__ void k_store_job(QuadJob job, QuadJob *dst)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = job;
}

// ================================================================== launchers

static inline unsigned int nblocks(int64_t n, int bs) { return (unsigned int)((n + bs - 1) / bs); }

hipError_t launch_node_tables(hipStream_t st, int n_r, int n_phi, double f, const double *r, const double *wr,
                              const double *cphi, const double *sphi, double dphi, double *pos64, float *pos32,
                              double *nrm, double *wgt, double *tan)
{
    const int n = (n_r + 1) * n_phi;
    hipLaunchKernelGGL(k_node_tables, dim3(nblocks(n, 256)), dim3(256), 0, st, n_r, n_phi, f, r, wr, cphi, sphi,
                       dphi, pos64, pos32, nrm, wgt, tan);
    return hipGetLastError();
}

hipError_t launch_node_half_inverse(hipStream_t st, int n_tot, const double *pos64, double *hinv64, float *hinv32)
{
    hipLaunchKernelGGL(k_node_half_inverse, dim3(nblocks(n_tot, 256)), dim3(256), 0, st, n_tot, pos64, hinv64,
                       hinv32);
    return hipGetLastError();
}

hipError_t launch_surface_records(hipStream_t st, int n_surf, int n_rim, const double *xyz, const double *ndS,
                                  const double *rim_xyz, const double *rim_n, const double *rim_dl, double *pos64,
                                  float *pos32, double *nrm, double *wgt, double *tan)
{
    hipLaunchKernelGGL(k_surface_records, dim3(nblocks((int64_t)n_surf + n_rim, 256)), dim3(256), 0, st, n_surf,
                       n_rim, xyz, ndS, rim_xyz, rim_n, rim_dl, pos64, pos32, nrm, wgt, tan);
    return hipGetLastError();
}

hipError_t launch_obs_prep(hipStream_t st, const double *xyz, int n_obs, int n_obs_pad, double *obs64, float *obs32)
{
    hipLaunchKernelGGL(k_obs_prep, dim3(nblocks(n_obs_pad, 256)), dim3(256), 0, st, xyz, n_obs, n_obs_pad, obs64,
                       obs32);
    return hipGetLastError();
}

hipError_t launch_tables_from_fields(hipStream_t st, int n_k, int n_surf, int n_tot, const double *k,
                                     const double *pos64, const double *nrm, const double *wgt, const double *tan,
                                     const double *E, const double *B, double *tab64)
{
    hipLaunchKernelGGL(k_tables_from_fields, dim3(nblocks((int64_t)n_k * n_tot, 256)), dim3(256), 0, st, n_k,
                       n_surf, n_tot, k, pos64, nrm, wgt, tan, E, B, tab64);
    return hipGetLastError();
}

hipError_t launch_tables_gaussian(hipStream_t st, int n_k, int n_surf, int n_tot, const double *k,
                                  const double *pos64, const double *nrm, const double *wgt, const double *tan,
                                  int beam, double w0, double pol, const double *spectrum, int consistent,
                                  const double *modes, int n_modes, double *tab64)
{
    hipLaunchKernelGGL(k_tables_gaussian, dim3(nblocks((int64_t)n_k * n_tot, 256)), dim3(256), 0, st, n_k, n_surf,
                       n_tot, k, pos64, nrm, wgt, tan, beam, w0, pol, spectrum, consistent, modes, n_modes, tab64);
    return hipGetLastError();
}

hipError_t launch_power_fields(hipStream_t st, int n_k, int n_surf, int n_tot, const double *nrm, const double *wgt,
                               const double *E, const double *B, double *part, double *P)
{
    hipLaunchKernelGGL(k_power_fields, dim3(POWER_BLOCKS, n_k), dim3(256), 0, st, n_surf, n_tot, nrm, wgt, E, B,
                       part);
    hipLaunchKernelGGL(k_power_finish, dim3(nblocks(n_k, 256)), dim3(256), 0, st, n_k, part, P);
    return hipGetLastError();
}

hipError_t launch_power_gaussian(hipStream_t st, int n_k, int n_surf, const double *k, const double *pos64,
                                 const double *nrm, const double *wgt, int beam, double w0, double pol,
                                 const double *spectrum, int consistent, const double *modes, int n_modes,
                                 double *part, double *P)
{
    hipLaunchKernelGGL(k_power_gaussian, dim3(POWER_BLOCKS, n_k), dim3(256), 0, st, n_surf, k, pos64, nrm, wgt, beam,
                       w0, pol, spectrum, consistent, modes, n_modes, part);
    hipLaunchKernelGGL(k_power_finish, dim3(nblocks(n_k, 256)), dim3(256), 0, st, n_k, part, P);
    return hipGetLastError();
}

int power_partial_count(int n_k) { return POWER_BLOCKS * n_k; }

hipError_t launch_tables_scale(hipStream_t st, int n_k, int n_tot, int n_cplx, const double *fac, double *tab64,
                               float *tab32)
{
    hipLaunchKernelGGL(k_tables_scale, dim3(nblocks((int64_t)n_k * n_tot, 256)), dim3(256), 0, st, n_k, n_tot,
                       n_cplx, fac, tab64, tab32);
    return hipGetLastError();
}

hipError_t launch_tables_factor(hipStream_t st, int n_k, int n_tot, const double *k, const double *tab64,
                                const float *pos32, const double *pos64, double tol32, double tol64, float *tabf,
                                float *posf, float *betaf, float *tabp, double *tabf64, double *posf64,
                                double *betaf64, unsigned int *bad)
{
    hipLaunchKernelGGL(k_tables_factor, dim3(nblocks(n_tot, 256)), dim3(256), 0, st, n_k, n_tot, k, tab64, pos32,
                       pos64, tol32, tol64, tabf, posf, betaf, tabp, tabf64, posf64, betaf64, bad);
    return hipGetLastError();
}

hipError_t launch_tables_polar(hipStream_t st, int64_t n_rec, const float *tabf, float *tabp)
{
    hipLaunchKernelGGL(k_tables_polar, dim3(nblocks(n_rec, 256)), dim3(256), 0, st, n_rec, tabf, tabp);
    return hipGetLastError();
}

hipError_t launch_tables_cast(hipStream_t st, int n_k, int n_tot, const double *k, const double *pos64,
                              const double *tab64, const float *src32, float *tab32, int naive)
{
    hipLaunchKernelGGL(k_tables_cast, dim3(nblocks((int64_t)n_k * n_tot, 256)), dim3(256), 0, st, n_k, n_tot, k,
                       pos64, tab64, src32, tab32, naive);
    return hipGetLastError();
}

hipError_t launch_reduce(hipStream_t st, int mode, const void *partial, int n_chunks, int n_k, int n_obs,
                         int n_obs_pad, const double *k, int b_over_k, void *E, void *B)
{
    const unsigned int nb = nblocks((int64_t)n_k * n_obs, 256);
    if (mode == MODE_FP64)
        hipLaunchKernelGGL((k_reduce<double, double>), dim3(nb), dim3(256), 0, st, (const double *)partial, n_chunks,
                           n_k, n_obs, n_obs_pad, k, b_over_k, (double *)E, (double *)B);
    else
        hipLaunchKernelGGL((k_reduce<float, float>), dim3(nb), dim3(256), 0, st, (const float *)partial, n_chunks,
                           n_k, n_obs, n_obs_pad, k, b_over_k, (float *)E, (float *)B);
    return hipGetLastError();
}

hipError_t launch_twiddles(hipStream_t st, int n_k, const double *k, int n_t, const double *t, double dk, double *tw)
{
    hipLaunchKernelGGL(k_twiddles, dim3(nblocks((int64_t)n_k * n_t, 256)), dim3(256), 0, st, n_k, k, n_t, t, dk, tw);
    return hipGetLastError();
}

hipError_t launch_time(hipStream_t st, int is_f64, int n_k, int n_t, int64_t n_x, const double *tw, const void *F,
                       void *Ft)
{
    dim3 g(nblocks(n_x, 256), (n_t + TIME_MT - 1) / TIME_MT);
    if (is_f64)
        hipLaunchKernelGGL((k_time<double>), g, dim3(256), 0, st, n_k, n_t, n_x, tw, (const double *)F,
                           (double *)Ft);
    else
        hipLaunchKernelGGL((k_time<float>), g, dim3(256), 0, st, n_k, n_t, n_x, tw, (const float *)F, (float *)Ft);
    return hipGetLastError();
}

hipError_t launch_fill_u32(hipStream_t st, unsigned int *p, unsigned int v, int n)
{
    hipLaunchKernelGGL(k_fill_u32, dim3(nblocks(n, 256)), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

hipError_t launch_store_job(hipStream_t st, const QuadJob &job, QuadJob *dst)
{
    hipLaunchKernelGGL(k_store_job, dim3(1), dim3(64), 0, st, job, dst);
    return hipGetLastError();
}

}  // namespace sc
