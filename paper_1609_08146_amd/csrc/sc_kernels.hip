// sc_kernels.hip -- gfx950 kernels of the Stratton-Chu mirror-focusing path.
//
//  k_node_tables         mirror nodes, normals, weights            (Sec. III-C)
//  k_obs_prep            observation records
//  k_tables_from_fields  POA current / charge tables from given E_inc, B_inc
//  k_tables_gaussian     same for the built-in collimated Gaussian (Sec. III-A)
//  k_tables_cast         FP64 tables -> FP32 (split: as is; naive: node phase removed)
//  k_quad<MODE,OPL>      the surface quadrature, persistent over (job, k, chunk, obs) tiles
//  k_reduce<MODE>        deterministic split-K reduction into E, B
//  k_twiddles, k_time    semi-discrete transform to time (Sec. III-B)
//
// All floating-point expressions are written with explicit fma/mul/add and
// the file is compiled with -ffp-contract=off, so the rounding sequence of
// every observation point is fixed by the source: results do not depend on
// the launch shape (obs per lane, waves per block, grid), only on the chunking.
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
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_tot) return;
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

__global__ void k_obs_prep(const double *__restrict__ xyz, int n_obs, int n_obs_pad, double *__restrict__ obs64,
                           float *__restrict__ obs32)
{
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= n_obs_pad) return;
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

__global__ void k_tables_gaussian(int n_k, int n_surf, int n_tot, const double *__restrict__ kv,
                                  const double *__restrict__ pos64, const double *__restrict__ nrm,
                                  const double *__restrict__ wgt, const double *__restrict__ tan, double w0,
                                  double pol, const double *__restrict__ spectrum, int consistent,
                                  double *__restrict__ tab64)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n_k * n_tot) return;
    const int kk = (int)(idx / n_tot);
    const int q = (int)(idx - (int64_t)kk * n_tot);
    const double k = kv[kk];
    const double *p = pos64 + 4 * q;
    const double X = p[0], Y = p[1], Z = p[2];
    double sl, cl;
    sincos(pol, &sl, &cl);
    // frame where the polarisation is along x
    const double x = cl * X + sl * Y;
    const double y = -sl * X + cl * Y;
    const double G = exp(-(x * x + y * y) / (w0 * w0));
    const c64 amp = spectrum ? c64{spectrum[2 * kk], spectrum[2 * kk + 1]} : c64{1.0, 0.0};
    const c64 psi = {G * amp.re, G * amp.im};   // without the propagation phase e^{-ikz}
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
    c64 E[3], B[3];
    E[0] = {cl * e[0].re - sl * e[1].re, cl * e[0].im - sl * e[1].im};
    E[1] = {sl * e[0].re + cl * e[1].re, sl * e[0].im + cl * e[1].im};
    E[2] = e[2];
    B[0] = {cl * bb[0].re - sl * bb[1].re, cl * bb[0].im - sl * bb[1].im};
    B[1] = {sl * bb[0].re + cl * bb[1].re, sl * bb[0].im + cl * bb[1].im};
    B[2] = bb[2];
    // propagation phase e^{-ikz} fused with the node phase e^{ik|r_s|}: e^{ik(|r_s| - z)},
    // formed in double-double so that no ~1e6 rad phase is ever rounded to double
    const dd rs = dd_norm3(X, Y, Z);
    double sp, cp;
    sincos(phase_mod_2pi(k, dd_sub_d(rs, Z)), &sp, &cp);
    const bool rim = q >= n_surf;
    write_record(tab64 + idx * 8, rim, k, wgt[q], nrm + 3 * q, rim ? tan + 3 * (q - n_surf) : nullptr, E, B,
                 {cp, sp});
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

// ================================================================= quadrature

// Constant-address-space views: uniform loads through them become scalar
// (SMEM) loads into SGPRs, so node data costs no VGPRs and no LDS traffic.
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(4))) const v4f cv4f;
typedef __attribute__((address_space(4))) const double cdouble;
typedef __attribute__((address_space(4))) const QuadJob cjob;

// sin and cos of theta = 2 pi * t, t in turns: hardware v_sin / v_cos on the
// fractional part (the exact reduction modulo one turn, in [0, 1)).
__device__ __forceinline__ void sincos_turns(float t, float &s, float &c)
{
    const float r = __builtin_amdgcn_fractf(t);
    s = __builtin_amdgcn_sinf(r);
    c = __builtin_amdgcn_cosf(r);
}

// The per-pair work is split into a geometry part (one per node and
// observation point) and a per-frequency part, so that a lane holding several
// frequencies reuses the geometry.  The arithmetic sequence of one (point,
// frequency) pair is the same whatever the blocking.

// Geometry of the split form in FP32:  R = r_s - r',  1/|R|,
//   delta = |R| - |r_s| = (|r'|^2 - 2 r_s.r') / (|R| + |r_s|)  (no cancellation).
//   p = (x, y, z, |r_s|), o = (x, y, z, |r'|^2).
struct GeomF {
    float dx, dy, dz, rinv, delta;
};

__device__ __forceinline__ GeomF geom_split(const v4f p, const v4f o)
{
    GeomF g;
    g.dx = p.x - o.x;
    g.dy = p.y - o.y;
    g.dz = p.z - o.z;
    const float R2 = __fmaf_rn(g.dx, g.dx, __fmaf_rn(g.dy, g.dy, g.dz * g.dz));
    g.rinv = __builtin_amdgcn_rsqf(R2);
    const float R = R2 * g.rinv;
    const float dot = __fmaf_rn(p.x, o.x, __fmaf_rn(p.y, o.y, p.z * o.z));
    const float num = __fmaf_rn(-2.0f, dot, o.w);
    g.delta = num * __builtin_amdgcn_rcpf(R + p.w);
    return g;
}

// Accumulate one (node, point, frequency) term given e^{i theta} = (c, s):
//   gt = e^{i theta} / R,  ht = (ik - 1/R) gt / R,
//   acc[0..5] += Jt gt + rho_t ht R   (E),   acc[6..11] += (Jt ht) x R   (B before 1/ik).
//   t0 = (Jt.x, Jt.y), t1 = (Jt.z, rho_t), each complex as (re, im).
__device__ __forceinline__ void accumulate_f32(float dx, float dy, float dz, float rinv, float c, float s,
                                               const v4f t0, const v4f t1, float k, float *acc)
{
    const float gr = c * rinv, gi = s * rinv;
    const float a = -(rinv * rinv), b = k * rinv;
    const float hr = __fmaf_rn(gr, a, -(gi * b));
    const float hi = __fmaf_rn(gr, b, gi * a);
    // E += Jt gt
    acc[0] = __fmaf_rn(t0.x, gr, __fmaf_rn(-t0.y, gi, acc[0]));
    acc[1] = __fmaf_rn(t0.x, gi, __fmaf_rn(t0.y, gr, acc[1]));
    acc[2] = __fmaf_rn(t0.z, gr, __fmaf_rn(-t0.w, gi, acc[2]));
    acc[3] = __fmaf_rn(t0.z, gi, __fmaf_rn(t0.w, gr, acc[3]));
    acc[4] = __fmaf_rn(t1.x, gr, __fmaf_rn(-t1.y, gi, acc[4]));
    acc[5] = __fmaf_rn(t1.x, gi, __fmaf_rn(t1.y, gr, acc[5]));
    // E += rho_t ht R
    const float tr = __fmaf_rn(t1.z, hr, -(t1.w * hi));
    const float ti = __fmaf_rn(t1.z, hi, t1.w * hr);
    acc[0] = __fmaf_rn(tr, dx, acc[0]);
    acc[1] = __fmaf_rn(ti, dx, acc[1]);
    acc[2] = __fmaf_rn(tr, dy, acc[2]);
    acc[3] = __fmaf_rn(ti, dy, acc[3]);
    acc[4] = __fmaf_rn(tr, dz, acc[4]);
    acc[5] = __fmaf_rn(ti, dz, acc[5]);
    // B += (Jt ht) x R
    const float qxr = __fmaf_rn(t0.x, hr, -(t0.y * hi)), qxi = __fmaf_rn(t0.x, hi, t0.y * hr);
    const float qyr = __fmaf_rn(t0.z, hr, -(t0.w * hi)), qyi = __fmaf_rn(t0.z, hi, t0.w * hr);
    const float qzr = __fmaf_rn(t1.x, hr, -(t1.y * hi)), qzi = __fmaf_rn(t1.x, hi, t1.y * hr);
    acc[6] = __fmaf_rn(qyr, dz, __fmaf_rn(-qzr, dy, acc[6]));
    acc[7] = __fmaf_rn(qyi, dz, __fmaf_rn(-qzi, dy, acc[7]));
    acc[8] = __fmaf_rn(qzr, dx, __fmaf_rn(-qxr, dz, acc[8]));
    acc[9] = __fmaf_rn(qzi, dx, __fmaf_rn(-qxi, dz, acc[9]));
    acc[10] = __fmaf_rn(qxr, dy, __fmaf_rn(-qyr, dx, acc[10]));
    acc[11] = __fmaf_rn(qxi, dy, __fmaf_rn(-qyi, dx, acc[11]));
}

// Split form, one frequency: phase k delta (kt = k / 2 pi, in turns).
__device__ __forceinline__ void freq_split(const GeomF &g, const v4f t0, const v4f t1, float k, float kt, float *acc)
{
    float s, c;
    sincos_turns(kt * g.delta, s, c);
    accumulate_f32(g.dx, g.dy, g.dz, g.rinv, c, s, t0, t1, k, acc);
}

// Naive FP32 form, one frequency: the whole phase k |R| in FP32 (the table carries no node phase).
__device__ __forceinline__ void freq_naive(const GeomF &g, float R, const v4f t0, const v4f t1, float k, float *acc)
{
    float s, c;
    sincosf(k * R, &s, &c);
    accumulate_f32(g.dx, g.dy, g.dz, g.rinv, c, s, t0, t1, k, acc);
}

__device__ __forceinline__ void geom_naive(const v4f p, const v4f o, GeomF &g, float &R)
{
    g.dx = p.x - o.x;
    g.dy = p.y - o.y;
    g.dz = p.z - o.z;
    const float R2 = __fmaf_rn(g.dx, g.dx, __fmaf_rn(g.dy, g.dy, g.dz * g.dz));
    g.rinv = __builtin_amdgcn_rsqf(R2);
    R = R2 * g.rinv;
    g.delta = 0.0f;
}

// Geometry and per-frequency term of the split form in FP64.
struct GeomD {
    double dx, dy, dz, rinv, delta;
};

__device__ __forceinline__ GeomD geom_f64(const double *p, const double4 o)
{
    GeomD g;
    g.dx = p[0] - o.x;
    g.dy = p[1] - o.y;
    g.dz = p[2] - o.z;
    const double R2 = __fma_rn(g.dx, g.dx, __fma_rn(g.dy, g.dy, g.dz * g.dz));
    g.rinv = rsqrt(R2);
    const double R = R2 * g.rinv;
    const double dot = __fma_rn(p[0], o.x, __fma_rn(p[1], o.y, p[2] * o.z));
    const double num = __fma_rn(-2.0, dot, o.w);
    g.delta = num / (R + p[3]);
    return g;
}

__device__ __forceinline__ void freq_f64(const GeomD &g, const double *t, double k, double *acc)
{
    double s, c;
    sincos(k * g.delta, &s, &c);
    const double dx = g.dx, dy = g.dy, dz = g.dz, rinv = g.rinv;
    const double gr = c * rinv, gi = s * rinv;
    const double a = -(rinv * rinv), b = k * rinv;
    const double hr = __fma_rn(gr, a, -(gi * b));
    const double hi = __fma_rn(gr, b, gi * a);
    acc[0] = __fma_rn(t[0], gr, __fma_rn(-t[1], gi, acc[0]));
    acc[1] = __fma_rn(t[0], gi, __fma_rn(t[1], gr, acc[1]));
    acc[2] = __fma_rn(t[2], gr, __fma_rn(-t[3], gi, acc[2]));
    acc[3] = __fma_rn(t[2], gi, __fma_rn(t[3], gr, acc[3]));
    acc[4] = __fma_rn(t[4], gr, __fma_rn(-t[5], gi, acc[4]));
    acc[5] = __fma_rn(t[4], gi, __fma_rn(t[5], gr, acc[5]));
    const double tr = __fma_rn(t[6], hr, -(t[7] * hi));
    const double ti = __fma_rn(t[6], hi, t[7] * hr);
    acc[0] = __fma_rn(tr, dx, acc[0]);
    acc[1] = __fma_rn(ti, dx, acc[1]);
    acc[2] = __fma_rn(tr, dy, acc[2]);
    acc[3] = __fma_rn(ti, dy, acc[3]);
    acc[4] = __fma_rn(tr, dz, acc[4]);
    acc[5] = __fma_rn(ti, dz, acc[5]);
    const double qxr = __fma_rn(t[0], hr, -(t[1] * hi)), qxi = __fma_rn(t[0], hi, t[1] * hr);
    const double qyr = __fma_rn(t[2], hr, -(t[3] * hi)), qyi = __fma_rn(t[2], hi, t[3] * hr);
    const double qzr = __fma_rn(t[4], hr, -(t[5] * hi)), qzi = __fma_rn(t[4], hi, t[5] * hr);
    acc[6] = __fma_rn(qyr, dz, __fma_rn(-qzr, dy, acc[6]));
    acc[7] = __fma_rn(qyi, dz, __fma_rn(-qzi, dy, acc[7]));
    acc[8] = __fma_rn(qzr, dx, __fma_rn(-qxr, dz, acc[8]));
    acc[9] = __fma_rn(qzi, dx, __fma_rn(-qxi, dz, acc[9]));
    acc[10] = __fma_rn(qxr, dy, __fma_rn(-qyr, dx, acc[10]));
    acc[11] = __fma_rn(qxi, dy, __fma_rn(-qyi, dx, acc[11]));
}

// Map a global tile index to its job (binary search over tile0; uniform).
__device__ __forceinline__ int find_job(cjob *jobs, int n_jobs, int64_t t)
{
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].tile0 <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

constexpr int KAHAN_BLOCK = 32;   // nodes summed plainly before each compensated add (FP32)

// Persistent quadrature kernel.  Every wave repeatedly takes the next tile
// from a device counter: one node chunk, 64*OPL observation points, FPB
// consecutive frequencies.  Node and table data are wave-uniform (scalar
// loads); each lane owns OPL points x FPB frequencies x 12 accumulators.
// Every wave exits once the counter passes n_tiles.
template <int MODE, int OPL, int FPB>
__global__ void __launch_bounds__(256) k_quad(const QuadJob *__restrict__ jobs_, int n_jobs, int64_t n_tiles,
                                              unsigned int *__restrict__ counter)
{
    cjob *jobs = (cjob *)jobs_;
    const int lane = threadIdx.x & 63;
    for (;;) {
        unsigned int tt = 0;
        if (lane == 0) tt = atomicAdd(counter, 1u);
        const int64_t t = (int64_t)__builtin_amdgcn_readfirstlane(tt);
        if (t >= n_tiles) break;
        const int j = find_job(jobs, n_jobs, t);
        const int64_t local = t - jobs[j].tile0 + jobs[j].tile_offset;
        const int obs_blocks = jobs[j].obs_blocks, n_chunks = jobs[j].n_chunks;
        const int ob = (int)(local % obs_blocks);
        const int64_t rest = local / obs_blocks;
        const int chunk = (int)(rest % n_chunks);
        const int kb = (int)(rest / n_chunks);
        const int n_tot = jobs[j].n_tot, n_k = jobs[j].n_k, n_obs_pad = jobs[j].n_obs_pad;
        const int n0 = chunk * jobs[j].chunk;
        const int n1 = min(n0 + jobs[j].chunk, n_tot);
        const int obase = ob * 64 * OPL + lane;
        // frequencies of this tile; past the last one, repeat it and skip the store
        int kidx[FPB];
        double k64[FPB];
#pragma unroll
        for (int f = 0; f < FPB; ++f) {
            kidx[f] = min(kb * FPB + f, n_k - 1);
            k64[f] = ((cdouble *)jobs[j].k)[kidx[f]];
        }
        const int n_valid = min(FPB, n_k - kb * FPB);

        if constexpr (MODE == MODE_FP64) {
            cdouble *pos = (cdouble *)jobs[j].pos;
            cdouble *tab[FPB];
#pragma unroll
            for (int f = 0; f < FPB; ++f) tab[f] = (cdouble *)jobs[j].tab + (size_t)kidx[f] * n_tot * 8;
            const double4 *obs = (const double4 *)jobs[j].obs;
            double4 o[OPL];
            double acc[OPL][FPB][12];
#pragma unroll
            for (int s = 0; s < OPL; ++s) {
                o[s] = obs[obase + 64 * s];
#pragma unroll
                for (int f = 0; f < FPB; ++f)
#pragma unroll
                    for (int c = 0; c < 12; ++c) acc[s][f][c] = 0.0;
            }
            for (int n = n0; n < n1; ++n) {
                double pn[4], tn[FPB][8];
#pragma unroll
                for (int c = 0; c < 4; ++c) pn[c] = pos[4 * (size_t)n + c];
#pragma unroll
                for (int f = 0; f < FPB; ++f)
#pragma unroll
                    for (int c = 0; c < 8; ++c) tn[f][c] = tab[f][8 * (size_t)n + c];
#pragma unroll
                for (int s = 0; s < OPL; ++s) {
                    const GeomD g = geom_f64(pn, o[s]);
#pragma unroll
                    for (int f = 0; f < FPB; ++f) freq_f64(g, tn[f], k64[f], acc[s][f]);
                }
            }
#pragma unroll
            for (int f = 0; f < FPB; ++f) {
                if (f >= n_valid) break;
                double *part = (double *)jobs[j].partial + ((size_t)chunk * n_k + kidx[f]) * 12 * (size_t)n_obs_pad;
#pragma unroll
                for (int s = 0; s < OPL; ++s)
#pragma unroll
                    for (int c = 0; c < 12; ++c) part[(size_t)c * n_obs_pad + obase + 64 * s] = acc[s][f][c];
            }
        } else {
            cv4f *pos = (cv4f *)jobs[j].pos;
            cv4f *tab[FPB];
            float k[FPB], kt[FPB];
#pragma unroll
            for (int f = 0; f < FPB; ++f) {
                tab[f] = (cv4f *)jobs[j].tab + (size_t)kidx[f] * n_tot * 2;
                k[f] = (float)k64[f];
                kt[f] = (float)(k64[f] * INV_TWO_PI);
            }
            const v4f *obs = (const v4f *)jobs[j].obs;
            v4f o[OPL];
            // Running sums stay in registers; their Kahan compensations live in LDS
            // (touched once per KAHAN_BLOCK nodes), which frees VGPRs for occupancy.
            // dynamic LDS: [waves per block][OPL * FPB * 12][64] floats
            extern __shared__ float lds_dyn[];
            float(*cmp)[64] = (float(*)[64])(lds_dyn + (size_t)(threadIdx.x >> 6) * (OPL * FPB * 12 * 64));
            float sum[OPL][FPB][12];
#pragma unroll
            for (int s = 0; s < OPL; ++s) {
                o[s] = obs[obase + 64 * s];
#pragma unroll
                for (int f = 0; f < FPB; ++f)
#pragma unroll
                    for (int c = 0; c < 12; ++c) sum[s][f][c] = 0.0f;
            }
#pragma unroll
            for (int a = 0; a < OPL * FPB * 12; ++a) cmp[a][lane] = 0.0f;
            float blk[OPL][FPB][12];
#pragma unroll
            for (int s = 0; s < OPL; ++s)
#pragma unroll
                for (int f = 0; f < FPB; ++f)
#pragma unroll
                    for (int c = 0; c < 12; ++c) blk[s][f][c] = 0.0f;
            // node data of node n+1 is loaded while node n is computed
            v4f pn = pos[n0];
            v4f t0[FPB], t1[FPB];
#pragma unroll
            for (int f = 0; f < FPB; ++f) {
                t0[f] = tab[f][2 * n0];
                t1[f] = tab[f][2 * n0 + 1];
            }
            for (int n = n0; n < n1; ++n) {
                const int nx = min(n + 1, n1 - 1);
                const v4f pnx = pos[nx];
                v4f t0x[FPB], t1x[FPB];
#pragma unroll
                for (int f = 0; f < FPB; ++f) {
                    t0x[f] = tab[f][2 * nx];
                    t1x[f] = tab[f][2 * nx + 1];
                }
#pragma unroll
                for (int s = 0; s < OPL; ++s) {
                    if constexpr (MODE == MODE_SPLIT) {
                        const GeomF g = geom_split(pn, o[s]);
#pragma unroll
                        for (int f = 0; f < FPB; ++f) freq_split(g, t0[f], t1[f], k[f], kt[f], blk[s][f]);
                    } else {
                        GeomF g;
                        float R;
                        geom_naive(pn, o[s], g, R);
#pragma unroll
                        for (int f = 0; f < FPB; ++f) freq_naive(g, R, t0[f], t1[f], k[f], blk[s][f]);
                    }
                }
                // every KAHAN_BLOCK nodes (counted from the chunk start), a compensated add
                if ((n - n0) % KAHAN_BLOCK == KAHAN_BLOCK - 1 || n == n1 - 1) {
#pragma unroll
                    for (int s = 0; s < OPL; ++s)
#pragma unroll
                        for (int f = 0; f < FPB; ++f)
#pragma unroll
                            for (int c = 0; c < 12; ++c) {
                                const int a = (s * FPB + f) * 12 + c;
                                const float y = blk[s][f][c] - cmp[a][lane];
                                const float tsum = sum[s][f][c] + y;
                                cmp[a][lane] = (tsum - sum[s][f][c]) - y;
                                sum[s][f][c] = tsum;
                                blk[s][f][c] = 0.0f;
                            }
                }
                pn = pnx;
#pragma unroll
                for (int f = 0; f < FPB; ++f) {
                    t0[f] = t0x[f];
                    t1[f] = t1x[f];
                }
            }
#pragma unroll
            for (int f = 0; f < FPB; ++f) {
                if (f >= n_valid) break;
                float *part = (float *)jobs[j].partial + ((size_t)chunk * n_k + kidx[f]) * 12 * (size_t)n_obs_pad;
#pragma unroll
                for (int s = 0; s < OPL; ++s)
#pragma unroll
                    for (int c = 0; c < 12; ++c)
                        part[(size_t)c * n_obs_pad + obase + 64 * s] = sum[s][f][c] - cmp[(s * FPB + f) * 12 + c][lane];
            }
        }
    }
}

// Split-K reduction: E[k][o][c] = sum over chunks (in FP64, fixed order); B gets the 1/(ik) factor.
template <typename PT, typename OT>
__global__ void k_reduce(const PT *__restrict__ partial, int n_chunks, int n_k, int n_obs, int n_obs_pad,
                         const double *__restrict__ kv, OT *__restrict__ E, OT *__restrict__ B)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n_k * n_obs) return;
    const int kk = (int)(idx / n_obs);
    const int o = (int)(idx - (int64_t)kk * n_obs);
    double acc[12];
    for (int c = 0; c < 12; ++c) acc[c] = 0.0;
    for (int ch = 0; ch < n_chunks; ++ch) {
        const PT *p = partial + ((size_t)ch * n_k + kk) * 12 * (size_t)n_obs_pad + o;
        for (int c = 0; c < 12; ++c) acc[c] += (double)p[(size_t)c * n_obs_pad];
    }
    const double ik_inv = 1.0 / kv[kk];   // 1/(ik) = -i/k
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
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_k * n_t) return;
    const int m = idx / n_k, n = idx - m * n_k;
    double s, c;
    sincos(phase_mod_2pi(kv[n], dd{-t[m], 0.0}), &s, &c);
    tw[2 * idx] = dk * c;
    tw[2 * idx + 1] = dk * s;
}

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
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
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
                                  double w0, double pol, const double *spectrum, int consistent, double *tab64)
{
    hipLaunchKernelGGL(k_tables_gaussian, dim3(nblocks((int64_t)n_k * n_tot, 256)), dim3(256), 0, st, n_k, n_surf,
                       n_tot, k, pos64, nrm, wgt, tan, w0, pol, spectrum, consistent, tab64);
    return hipGetLastError();
}

hipError_t launch_tables_cast(hipStream_t st, int n_k, int n_tot, const double *k, const double *pos64,
                              const double *tab64, const float *src32, float *tab32, int naive)
{
    hipLaunchKernelGGL(k_tables_cast, dim3(nblocks((int64_t)n_k * n_tot, 256)), dim3(256), 0, st, n_k, n_tot, k,
                       pos64, tab64, src32, tab32, naive);
    return hipGetLastError();
}

// Instantiated shapes (obs per lane x frequencies per lane).
#define SC_QUAD_SHAPES(X, M) X(M, 1, 1) X(M, 2, 1) X(M, 1, 2) X(M, 2, 2) X(M, 1, 4)

static bool shape_ok(int opl, int fpb)
{
    return (opl == 1 && (fpb == 1 || fpb == 2 || fpb == 4)) || (opl == 2 && (fpb == 1 || fpb == 2));
}

static const void *quad_fn_dyn(int mode, int opl, int fpb)
{
#define SC_QUAD_FN(M, O, F) \
    if (mode == M && opl == O && fpb == F) return (const void *)&k_quad<M, O, F>;
    SC_QUAD_SHAPES(SC_QUAD_FN, MODE_FP64)
    SC_QUAD_SHAPES(SC_QUAD_FN, MODE_SPLIT)
    SC_QUAD_SHAPES(SC_QUAD_FN, MODE_NAIVE)
#undef SC_QUAD_FN
    return nullptr;
}

// Dynamic LDS of one quadrature block: the FP32 forms keep their Kahan compensations there.
static size_t quad_lds_bytes(int mode, int opl, int fpb, int waves_per_block)
{
    return mode == MODE_FP64 ? 0 : sizeof(float) * 64 * 12 * (size_t)opl * fpb * waves_per_block;
}

int quad_max_blocks_per_cu(int mode, int opl, int fpb, int waves_per_block)
{
    const void *fn = quad_fn_dyn(mode, opl, fpb);
    int nb = 0;
    if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 64 * waves_per_block,
                                                            quad_lds_bytes(mode, opl, fpb, waves_per_block)) !=
                   hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

hipError_t launch_quad(hipStream_t st, int mode, int opl, int fpb, int waves_per_block, int grid,
                       const QuadJob *jobs, int n_jobs, int64_t n_tiles, unsigned int *counter)
{
    if (!shape_ok(opl, fpb)) return hipErrorInvalidValue;
    dim3 g(grid), b(64 * waves_per_block);
    const size_t lds = quad_lds_bytes(mode, opl, fpb, waves_per_block);
#define SC_QUAD_LAUNCH(M, O, F)                                                                          \
    if (mode == M && opl == O && fpb == F) {                                                            \
        hipLaunchKernelGGL((k_quad<M, O, F>), g, b, lds, st, jobs, n_jobs, n_tiles, counter);           \
        return hipGetLastError();                                                                       \
    }
    SC_QUAD_SHAPES(SC_QUAD_LAUNCH, MODE_FP64)
    SC_QUAD_SHAPES(SC_QUAD_LAUNCH, MODE_SPLIT)
    SC_QUAD_SHAPES(SC_QUAD_LAUNCH, MODE_NAIVE)
#undef SC_QUAD_LAUNCH
    return hipErrorInvalidValue;
}

hipError_t launch_reduce(hipStream_t st, int mode, const void *partial, int n_chunks, int n_k, int n_obs,
                         int n_obs_pad, const double *k, void *E, void *B)
{
    const unsigned int nb = nblocks((int64_t)n_k * n_obs, 256);
    if (mode == MODE_FP64)
        hipLaunchKernelGGL((k_reduce<double, double>), dim3(nb), dim3(256), 0, st, (const double *)partial, n_chunks,
                           n_k, n_obs, n_obs_pad, k, (double *)E, (double *)B);
    else
        hipLaunchKernelGGL((k_reduce<float, float>), dim3(nb), dim3(256), 0, st, (const float *)partial, n_chunks,
                           n_k, n_obs, n_obs_pad, k, (float *)E, (float *)B);
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

}  // namespace sc
