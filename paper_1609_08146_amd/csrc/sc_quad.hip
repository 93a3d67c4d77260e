// sc_quad.hip -- the surface quadrature of the Stratton-Chu mirror-focusing
// path on gfx950: k_quad<MODE,OPL,FPB>, persistent over (job, frequency block,
// node chunk, observation block) tiles, and its launcher.
//
//   MODE_SPLIT  per-pair FP32 with the node phase folded into the tables;
//               per job either general tables or the factored current
//               J~ = u s (a real direction u per node, a complex s per
//               frequency and node), which needs fewer operations per pair,
//               and fewer still when the charge is tied to it as
//               rho_t = -i beta s / k (a real beta per node)
//   MODE_FP64   the same split form in FP64, on either table layout
//   MODE_NAIVE  the whole phase k|R| per pair in FP32 (the precision ablation)
//
// All floating-point expressions are written with explicit fma/mul/add and
// the file is compiled with -ffp-contract=off, so the rounding sequence of
// every observation point is fixed by the source: results do not depend on
// the launch shape (obs per lane, frequencies per lane, waves per block,
// grid), only on the node chunking.
#include "sc_device.h"
#include "sc_internal.h"

namespace sc {

// ================================================================= quadrature

// Constant-address-space views: uniform loads through them become scalar
// (SMEM) loads into SGPRs, so node data costs no VGPRs and no LDS traffic.
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(4))) const v4f cv4f;
typedef __attribute__((address_space(4))) const v2f cv2f;
typedef __attribute__((address_space(4))) const double cdouble;
typedef __attribute__((address_space(4))) const float cfloat;
typedef __attribute__((address_space(4))) const QuadJob cjob;

// sin and cos of theta = 2 pi * t, t in turns, with the hardware v_sin / v_cos.
// They accept |t| <= 256 turns directly, as accurately as the fractional part
// (1.2e-7 absolute either way); RAW = false first reduces to the fractional
// part (exact, in [0, 1)), which any t allows.
template <bool RAW>
__device__ __forceinline__ void sincos_turns(float t, float &s, float &c)
{
    const float r = RAW ? t : __builtin_amdgcn_fractf(t);
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

// The same geometry by series, near the focus.  delta (2|r_s| + delta) = num,
// so with h = 1 / (2|r_s|), delta_1 = num h and x = delta_1 h,
//   delta = delta_1 (1 - x + 2 x^2 - 5 x^3 + ...)   (Catalan numbers),
// and |R| = |r_s| + delta gives, with y = 2 h delta = delta / |r_s|,
//   1 / |R| = 2h (1 - y + y^2 - y^3 + ...).
// The caller guarantees |r'| <= 4e-4 |r_s|, so |x| <= 2e-4 and |y| <= 4e-4:
// the omitted terms (5 |x|^3 and |y|^3 relative, below 1e-10) are far below
// the FP32 rounding.  Neither a reciprocal nor a square root.
__device__ __forceinline__ GeomF geom_series(const v4f p, const v4f o, float h)
{
    GeomF g;
    g.dx = p.x - o.x;
    g.dy = p.y - o.y;
    g.dz = p.z - o.z;
    const float dot = __fmaf_rn(p.x, o.x, __fmaf_rn(p.y, o.y, p.z * o.z));
    const float num = __fmaf_rn(-2.0f, dot, o.w);
    const float d1 = num * h;
    const float x = d1 * h;
    g.delta = d1 * __fmaf_rn(x, __fmaf_rn(2.0f, x, -1.0f), 1.0f);
    const float h2 = h + h;
    const float y = g.delta * h2;
    g.rinv = h2 * __fmaf_rn(y, y - 1.0f, 1.0f);
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
template <bool RAW>
__device__ __forceinline__ void freq_split(const GeomF &g, const v4f t0, const v4f t1, float k, float kt, float *acc)
{
    float s, c;
    sincos_turns<RAW>(kt * g.delta, s, c);
    accumulate_f32(g.dx, g.dy, g.dz, g.rinv, c, s, t0, t1, k, acc);
}

// Factored current, one frequency.  When the surface current of a node has a
// real direction u for every frequency, J~ = u s.  With Z = e^{i theta} and
// m = ik - 1/R, gt = Z / R and ht = m Z / R^2, so
//   J~ gt = (u / R) (s Z),   rho_t ht R = (rho_t Z m) (R / R^2),
//   (J~ ht) x R = (s Z m) (u x R / R^2):
// the factors 1/R and 1/R^2 ride on the real per-(node, point) vectors
// v = u / R, e = R / R^2 and w = u x e, shared by the frequencies of a lane,
// and each frequency forms only the complex products s Z, rho_t Z and their
// products with m.  t = (s, rho_t) as (re, im) pairs.  acc as in accumulate_f32.
template <bool RAW>
__device__ __forceinline__ void freq_factored(float rinv, float delta, float vx, float vy, float vz, float ex,
                                              float ey, float ez, float wx, float wy, float wz, const v4f t, float k,
                                              float kt, float *acc)
{
    float c, sn;
    sincos_turns<RAW>(kt * delta, sn, c);
    // A = s Z, C = rho_t Z, and their products with m = -1/R + ik
    const float ar = __fmaf_rn(t.x, c, -(t.y * sn)), ai = __fmaf_rn(t.x, sn, t.y * c);
    const float cr = __fmaf_rn(t.z, c, -(t.w * sn)), ci = __fmaf_rn(t.z, sn, t.w * c);
    const float amr = __fmaf_rn(-rinv, ar, -(k * ai)), ami = __fmaf_rn(-rinv, ai, k * ar);
    const float cmr = __fmaf_rn(-rinv, cr, -(k * ci)), cmi = __fmaf_rn(-rinv, ci, k * cr);
    // E += v A
    acc[0] = __fmaf_rn(vx, ar, acc[0]);
    acc[1] = __fmaf_rn(vx, ai, acc[1]);
    acc[2] = __fmaf_rn(vy, ar, acc[2]);
    acc[3] = __fmaf_rn(vy, ai, acc[3]);
    acc[4] = __fmaf_rn(vz, ar, acc[4]);
    acc[5] = __fmaf_rn(vz, ai, acc[5]);
    // E += (C m) e
    acc[0] = __fmaf_rn(cmr, ex, acc[0]);
    acc[1] = __fmaf_rn(cmi, ex, acc[1]);
    acc[2] = __fmaf_rn(cmr, ey, acc[2]);
    acc[3] = __fmaf_rn(cmi, ey, acc[3]);
    acc[4] = __fmaf_rn(cmr, ez, acc[4]);
    acc[5] = __fmaf_rn(cmi, ez, acc[5]);
    // B += (A m) w
    acc[6] = __fmaf_rn(wx, amr, acc[6]);
    acc[7] = __fmaf_rn(wx, ami, acc[7]);
    acc[8] = __fmaf_rn(wy, amr, acc[8]);
    acc[9] = __fmaf_rn(wy, ami, acc[9]);
    acc[10] = __fmaf_rn(wz, amr, acc[10]);
    acc[11] = __fmaf_rn(wz, ami, acc[11]);
}

// Factored current with the charge tied to it, one frequency.  When moreover
// rho_t = -i beta s / k with a real beta per node (the charge of the beams
// whose E and B share one complex amplitude: n . E and n x B then carry the
// same s, and rho_t = (2W / 4 pi) n.E P against Jt = i k (2W / 4 pi) (n x B) P),
// then with A = s Z and m = ik - 1/R,
//   rho_t ht R = (rho_t Z m) e = beta e (-i A m / k),   (Jt ht) x R = k (A m / k) w,
// and A m / k = A (i - q) with q = 1 / (k R): no product rho_t Z, no product
// with m of its own, and the factor k of the B term is left to the reduction.
// s comes in polar form, t = (|s|, arg(s) / 2 pi): its phase joins the sine's
// argument (one FMA) and A = |s| (cos, sin), two MULs instead of a complex
// product.  e carries beta (e = beta R / R^2, formed once per node and point);
// kinv = 1/k.
template <bool RAW>
__device__ __forceinline__ void freq_tied(float rinv, float delta, float vx, float vy, float vz, float ex, float ey,
                                          float ez, float wx, float wy, float wz, const v2f t, float kinv, float kt,
                                          float *acc)
{
    float c, sn;
    sincos_turns<RAW>(__fmaf_rn(kt, delta, t.y), sn, c);
    const float ar = t.x * c, ai = t.x * sn;
    const float q = rinv * kinv;
    // M = A m / k = (-q ar - ai) + i (ar - q ai);  -i M = M.im - i M.re
    const float mr = __fmaf_rn(-q, ar, -ai), mi = __fmaf_rn(-q, ai, ar);
    // E += v A + e (-i M)
    acc[0] = __fmaf_rn(mi, ex, __fmaf_rn(vx, ar, acc[0]));
    acc[1] = __fmaf_rn(-mr, ex, __fmaf_rn(vx, ai, acc[1]));
    acc[2] = __fmaf_rn(mi, ey, __fmaf_rn(vy, ar, acc[2]));
    acc[3] = __fmaf_rn(-mr, ey, __fmaf_rn(vy, ai, acc[3]));
    acc[4] = __fmaf_rn(mi, ez, __fmaf_rn(vz, ar, acc[4]));
    acc[5] = __fmaf_rn(-mr, ez, __fmaf_rn(vz, ai, acc[5]));
    // B += M w   (B before 1/i)
    acc[6] = __fmaf_rn(wx, mr, acc[6]);
    acc[7] = __fmaf_rn(wx, mi, acc[7]);
    acc[8] = __fmaf_rn(wy, mr, acc[8]);
    acc[9] = __fmaf_rn(wy, mi, acc[9]);
    acc[10] = __fmaf_rn(wz, mr, acc[10]);
    acc[11] = __fmaf_rn(wz, mi, acc[11]);
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

// sin and cos of 2 pi j / 256, j = -128 ... 128, as (cos, sin) pairs in LDS: filled by the
// workgroup at the start of an FP64 launch (sincospi of the exact argument j / 128).
constexpr int TURN_STEPS = 256;
__device__ __forceinline__ const double2 *turn_table_lds()
{
    __shared__ double2 tab[TURN_STEPS + 1];
    for (int i = threadIdx.x; i <= TURN_STEPS; i += blockDim.x) {
        double sv, cv;
        sincospi((double)(i - TURN_STEPS / 2) / (double)(TURN_STEPS / 2), &sv, &cv);
        tab[i] = make_double2(cv, sv);
    }
    __syncthreads();
    return tab;
}

// sin and cos of 2 pi t in FP64.  The fractional turn r = t - rint(t) is exact, and so is
// z = r - j / 256 with j = rint(256 r) (|z| <= 1/512 turn): then 2 pi t = 2 pi j / 256 + x,
// x = 2 pi z, |x| <= pi / 256, and the angle sum combines the tabulated (cos, sin) of 2 pi j / 256
// with sin x = x - x^3/6 + x^5/120 and cos x = 1 - x^2/2 + x^4/24 - x^6/720 (the first omitted
// terms are below 1e-17 and 2e-20).
__device__ __forceinline__ void sincos_turns_f64(double t, const double2 *tab, double &s, double &c)
{
    const double r = t - rint(t);
    const double j = rint((double)TURN_STEPS * r);
    const double z = __fma_rn(-1.0 / TURN_STEPS, j, r);
    const double x = z * TWO_PI_1;
    const double u = x * x;
    const double ps = __fma_rn(u, 1.0 / 120.0, -1.0 / 6.0);
    const double sx = __fma_rn(x * u, ps, x);
    double pc = __fma_rn(u, -1.0 / 720.0, 1.0 / 24.0);
    pc = __fma_rn(u, pc, -0.5);
    const double cx = __fma_rn(u, pc, 1.0);
    const double2 w = tab[(int)j + TURN_STEPS / 2];
    s = __fma_rn(w.y, cx, w.x * sx);
    c = __fma_rn(w.x, cx, -(w.y * sx));
}

// The FP64 geometry by series near the focus (see geom_series): with
// |x| <= 2e-4 and |y| <= 4e-4 the terms through x^4 and y^4 leave omitted
// terms below 2e-17 relative.  h = 1 / (2|r_s|) from the factored node record
// or the job's per-node array.
__device__ __forceinline__ GeomD geom_f64_series(const double *p, const double4 o, double h)
{
    GeomD g;
    g.dx = p[0] - o.x;
    g.dy = p[1] - o.y;
    g.dz = p[2] - o.z;
    const double dot = __fma_rn(p[0], o.x, __fma_rn(p[1], o.y, p[2] * o.z));
    const double num = __fma_rn(-2.0, dot, o.w);
    const double d1 = num * h;
    const double x = d1 * h;
    // 1 - x + 2x^2 - 5x^3 + 14x^4
    double q = __fma_rn(14.0, x, -5.0);
    q = __fma_rn(q, x, 2.0);
    q = __fma_rn(q, x, -1.0);
    g.delta = d1 * __fma_rn(q, x, 1.0);
    const double h2 = h + h;
    const double y = g.delta * h2;
    // 1 - y + y^2 - y^3 + y^4
    double r = __fma_rn(y - 1.0, y, 1.0);
    r = __fma_rn(r, y, -1.0);
    g.rinv = h2 * __fma_rn(r, y, 1.0);
    return g;
}

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
    // delta = num / den: hardware reciprocal, two Newton steps, one residual correction
    const double den = R + p[3];
    double inv = __builtin_amdgcn_rcp(den);
    inv = __fma_rn(inv, __fma_rn(-den, inv, 1.0), inv);
    inv = __fma_rn(inv, __fma_rn(-den, inv, 1.0), inv);
    const double q = num * inv;
    g.delta = __fma_rn(__fma_rn(-den, q, num), inv, q);
    return g;
}

__device__ __forceinline__ void freq_f64(const GeomD &g, const double *t, double k, double kt, const double2 *ttab,
                                         double *acc)
{
    double s, c;
    sincos_turns_f64(kt * g.delta, ttab, s, c);
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

// Factored current in FP64, one frequency: the algebra of freq_factored
// (A = s Z, C = rho_t Z, m = ik - 1/R; E += v A + (C m) e, B += (A m) w) with
// t = (s, rho_t) as (re, im) pairs.
__device__ __forceinline__ void freq_f64_factored(double rinv, double delta, const double *v, const double *e,
                                                  const double *w, const double *t, double k, double kt,
                                                  const double2 *ttab, double *acc)
{
    double sn, c;
    sincos_turns_f64(kt * delta, ttab, sn, c);
    const double ar = __fma_rn(t[0], c, -(t[1] * sn)), ai = __fma_rn(t[0], sn, t[1] * c);
    const double cr = __fma_rn(t[2], c, -(t[3] * sn)), ci = __fma_rn(t[2], sn, t[3] * c);
    const double amr = __fma_rn(-rinv, ar, -(k * ai)), ami = __fma_rn(-rinv, ai, k * ar);
    const double cmr = __fma_rn(-rinv, cr, -(k * ci)), cmi = __fma_rn(-rinv, ci, k * cr);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        acc[2 * d] = __fma_rn(cmr, e[d], __fma_rn(v[d], ar, acc[2 * d]));
        acc[2 * d + 1] = __fma_rn(cmi, e[d], __fma_rn(v[d], ai, acc[2 * d + 1]));
        acc[6 + 2 * d] = __fma_rn(w[d], amr, acc[6 + 2 * d]);
        acc[7 + 2 * d] = __fma_rn(w[d], ami, acc[7 + 2 * d]);
    }
}

// The tied charge in FP64, one frequency: the algebra of freq_tied (M = A m / k = A (i - q),
// q = 1 / (k R); E += v A + e (-i M) with e = beta R / R^2, B += M w).
__device__ __forceinline__ void freq_f64_tied(double rinv, double delta, const double *v, const double *e,
                                              const double *w, const double *t, double kinv, double kt,
                                              const double2 *ttab, double *acc)
{
    double sn, c;
    sincos_turns_f64(kt * delta, ttab, sn, c);
    const double ar = __fma_rn(t[0], c, -(t[1] * sn)), ai = __fma_rn(t[0], sn, t[1] * c);
    const double q = rinv * kinv;
    const double mr = __fma_rn(-q, ar, -ai), mi = __fma_rn(-q, ai, ar);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        acc[2 * d] = __fma_rn(mi, e[d], __fma_rn(v[d], ar, acc[2 * d]));
        acc[2 * d + 1] = __fma_rn(-mr, e[d], __fma_rn(v[d], ai, acc[2 * d + 1]));
        acc[6 + 2 * d] = __fma_rn(w[d], mr, acc[6 + 2 * d]);
        acc[7 + 2 * d] = __fma_rn(w[d], mi, acc[7 + 2 * d]);
    }
}

// One tile of the FP64 form: nodes [n0, n1) of a chunk, 64*OPL points, FPB
// frequencies.  General layout: node records (x, y, z, |r_s|) and table
// records (Jt.x, Jt.y, Jt.z, rho_t) as (re, im) pairs, 4 and 8 doubles;
// factored (FACT): node records (x, y, z, |r_s|, u, 1 / (2|r_s|)) and table
// records (s, rho_t), 8 and 4 doubles; with the tied charge (TIE) only s of a
// table record is read, and beta from the job's per-node array.  Plain FP64 sums.
template <int OPL, int FPB, bool FACT, bool SER = false, bool TIE = false>
__device__ __forceinline__ void tile_f64(cjob *job, int lane, int chunk, int n0, int n1, int obase, const int *kidx,
                                         const double *k64, int n_valid, const double2 *ttab)
{
    static_assert(!TIE || FACT, "the tied charge needs the factored layout");
    constexpr int TL = TIE ? 2 : (FACT ? 4 : 8);   // doubles of a table record that are read
    constexpr int PS = FACT ? 8 : 4;   // doubles per node record
    constexpr int TS = FACT ? 4 : 8;   // doubles per table record
    const int n_tot = job->n_tot, n_k = job->n_k, n_obs_pad = job->n_obs_pad;
    cdouble *pos = (cdouble *)job->pos;
    cdouble *tab[FPB];
    double kt64[FPB], kinv64[FPB];   // wavenumbers in turns per unit length, 1 / k
#pragma unroll
    for (int f = 0; f < FPB; ++f) {
        tab[f] = (cdouble *)job->tab + (size_t)kidx[f] * n_tot * TS;
        kt64[f] = k64[f] * INV_TWO_PI;
        kinv64[f] = 1.0 / k64[f];
    }
    const double4 *obs = (const double4 *)job->obs;
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
        double pn[PS], tn[FPB][TL];
#pragma unroll
        for (int c = 0; c < PS; ++c) pn[c] = pos[PS * (size_t)n + c];
        double bn = 0.0;
        if constexpr (TIE) bn = ((cdouble *)job->beta)[n];
        // h = 1 / (2|r_s|): last entry of the factored node record, else the per-node array
        double hn = 0.0;
        if constexpr (SER && FACT) hn = pn[PS - 1];
        else if constexpr (SER) hn = ((cdouble *)job->hinv)[n];
#pragma unroll
        for (int f = 0; f < FPB; ++f)
#pragma unroll
            for (int c = 0; c < TL; ++c) tn[f][c] = tab[f][TS * (size_t)n + c];
#pragma unroll
        for (int s = 0; s < OPL; ++s) {
            GeomD g;
            if constexpr (SER) g = geom_f64_series(pn, o[s], hn);
            else g = geom_f64(pn, o[s]);
            if constexpr (FACT) {
                // v = u / R, e = R / R^2, w = u x e, shared by the frequencies
                const double r2 = g.rinv * g.rinv;
                const double v[3] = {pn[4] * g.rinv, pn[5] * g.rinv, pn[6] * g.rinv};
                const double e[3] = {g.dx * r2, g.dy * r2, g.dz * r2};
                const double w[3] = {__fma_rn(pn[5], e[2], -(pn[6] * e[1])), __fma_rn(pn[6], e[0], -(pn[4] * e[2])),
                                     __fma_rn(pn[4], e[1], -(pn[5] * e[0]))};
                if constexpr (TIE) {
                    const double eb[3] = {e[0] * bn, e[1] * bn, e[2] * bn};
#pragma unroll
                    for (int f = 0; f < FPB; ++f)
                        freq_f64_tied(g.rinv, g.delta, v, eb, w, tn[f], kinv64[f], kt64[f], ttab, acc[s][f]);
                } else {
#pragma unroll
                    for (int f = 0; f < FPB; ++f)
                        freq_f64_factored(g.rinv, g.delta, v, e, w, tn[f], k64[f], kt64[f], ttab, acc[s][f]);
                }
            } else {
#pragma unroll
                for (int f = 0; f < FPB; ++f) freq_f64(g, tn[f], k64[f], kt64[f], ttab, acc[s][f]);
            }
        }
    }
#pragma unroll
    for (int f = 0; f < FPB; ++f) {
        if (f >= n_valid) break;
        // partials [chunk][k][point / 64][12][64]
        double *part = (double *)job->partial + ((size_t)chunk * n_k + kidx[f]) * 12 * (size_t)n_obs_pad +
                       (size_t)((obase - lane) >> 6) * 768;
#pragma unroll
        for (int s = 0; s < OPL; ++s)
#pragma unroll
            for (int c = 0; c < 12; ++c) part[s * 768 + c * 64 + lane] = acc[s][f][c];
    }
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

// Nodes summed plainly in FP32 registers before each block sum is added into
// the chunk's running sum.  A plain FP32 sum of 512 terms errs by at most
// 511 u (3e-5) of the sum of their magnitudes and typically by about
// sqrt(512) u (1.3e-6); the running sum over the blocks of a chunk adds at most
// chunk / 512 - 1 further roundings.
constexpr int SUM_BLOCK = 512;

// One tile of the FP32 forms: nodes [n0, n1) of a chunk, 64*OPL points, FPB
// frequencies.  FACT selects the factored layout: node records of two v4f
// (x, y, z, |r_s|), (u, 1 / (2|r_s|)) and one v4f (s, rho_t) per table record, instead of
// one v4f node record and two v4f (Jt.x, Jt.y), (Jt.z, rho_t) per table record.
// TIE (factored only) takes the charge tied to the current (freq_tied): s in
// polar form from the job's tabp records, beta from its per-node array.
// RAW passes the split phase k delta / 2 pi to the hardware sin / cos without
// taking its fractional part (the job guarantees it stays below 250 turns).
// SER forms delta by its series (geom_series) from h = 1 / (2|r_s|), in the
// node record of the factored layout or the job's per-node array otherwise
// (the job guarantees |r'| <= 4e-4 |r_s|).
// The sums: each block of SUM_BLOCK nodes (counted from the chunk start) is
// summed plainly in registers, and the block sums are added in order into the
// chunk's running sum (the first block stores, the later ones load, add and
// store; every address belongs to one lane of one wave).  No second set of 12
// accumulators per (point, frequency) in registers, so a lane can hold four
// frequencies at five waves per SIMD.  The running sums of E sit in the wave's
// slice of the dynamic LDS ([OPL][FPB][6][64] floats: 6 KB per wave at four
// frequencies, 120 KB per CU at five waves per SIMD) and are stored into the
// partials after the last block; those of B are kept in the tile's own slice
// of the partials in device memory, whose slices in use outgrow an XCD's L2,
// so that load-add-store goes to memory: traffic, but no time, since the tile
// is bound by its VALU issue.  The order of the additions, and so every bit of
// the result, does not depend on where a running sum is kept.
template <int MODE, int OPL, int FPB, bool FACT, bool RAW, bool SER = false, bool TIE = false>
__device__ __forceinline__ void tile_f32(cjob *job, int lane, int chunk, int n0, int n1, int obase, const int *kidx,
                                         const double *k64, int n_valid)
{
    static_assert(!TIE || FACT, "the tied charge needs the factored layout");
    constexpr int PS = FACT ? 2 : 1;   // v4f per node record
    constexpr int TS = FACT ? 1 : 2;   // v4f per table record
    const int n_tot = job->n_tot, n_k = job->n_k, n_obs_pad = job->n_obs_pad;
    cv4f *pos = (cv4f *)job->pos;
    cv4f *tab[FPB];
    float k[FPB], kt[FPB], kinv[FPB];
    float *part[FPB];
    const int ob64 = (obase - lane) >> 6;   // the tile's first block of 64 points
#pragma unroll
    for (int f = 0; f < FPB; ++f) {
        tab[f] = (cv4f *)job->tab + (size_t)kidx[f] * n_tot * TS;
        k[f] = (float)k64[f];
        kt[f] = (float)(k64[f] * INV_TWO_PI);
        kinv[f] = (float)(1.0 / k64[f]);
        // partials [chunk][k][point / 64][12][64]: the tile's [12][64 * OPL] slice is contiguous
        part[f] = (float *)job->partial + ((size_t)chunk * n_k + kidx[f]) * 12 * (size_t)n_obs_pad +
                  (size_t)ob64 * 768;
    }
    const v4f *obs = (const v4f *)job->obs;
    v4f o[OPL];
#pragma unroll
    for (int s = 0; s < OPL; ++s) o[s] = obs[obase + 64 * s];
    constexpr bool HV = SER && !FACT;   // h from the per-node array
    cfloat *hv = (cfloat *)job->hinv;
    cfloat *bv = (cfloat *)job->beta;
    cv2f *tabp[FPB];
#pragma unroll
    for (int f = 0; f < FPB; ++f) tabp[f] = TIE ? (cv2f *)job->tabp + (size_t)kidx[f] * n_tot : nullptr;
    // the wave's running sums of E in LDS: [OPL][FPB][6][64]
    extern __shared__ float run_lds[];
    float *run = run_lds + (size_t)(threadIdx.x >> 6) * (OPL * FPB * 6 * 64) + lane;
    for (int b0 = n0; b0 < n1; b0 += SUM_BLOCK) {
        const int b1 = min(b0 + SUM_BLOCK, n1);
        float blk[OPL][FPB][12];
#pragma unroll
        for (int s = 0; s < OPL; ++s)
#pragma unroll
            for (int f = 0; f < FPB; ++f)
#pragma unroll
                for (int c = 0; c < 12; ++c) blk[s][f][c] = 0.0f;
        for (int n = b0; n < b1; ++n) {
            const v4f pn = pos[PS * n];
            v4f un = {0.0f, 0.0f, 0.0f, 0.0f};
            if constexpr (FACT) un = pos[PS * n + 1];
            float hn = 0.0f, bn = 0.0f;
            if constexpr (HV) hn = hv[n];
            if constexpr (TIE) bn = bv[n];
            v4f t0[FPB], t1[FPB];
            v2f ts[FPB];
#pragma unroll
            for (int f = 0; f < FPB; ++f) {
                if constexpr (TIE) ts[f] = tabp[f][n];
                else t0[f] = tab[f][TS * n];
                if constexpr (!FACT) t1[f] = tab[f][TS * n + 1];
            }
#pragma unroll
            for (int s = 0; s < OPL; ++s) {
                if constexpr (MODE == MODE_SPLIT && FACT) {
                    const GeomF g = SER ? geom_series(pn, o[s], un.w) : geom_split(pn, o[s]);
                    // v = u / R, e = R / R^2, w = u x e, shared by the frequencies
                    const float r2 = g.rinv * g.rinv;
                    const float vx = un.x * g.rinv, vy = un.y * g.rinv, vz = un.z * g.rinv;
                    const float ex = g.dx * r2, ey = g.dy * r2, ez = g.dz * r2;
                    const float wx = __fmaf_rn(un.y, ez, -(un.z * ey));
                    const float wy = __fmaf_rn(un.z, ex, -(un.x * ez));
                    const float wz = __fmaf_rn(un.x, ey, -(un.y * ex));
                    if constexpr (TIE) {
                        const float bx = ex * bn, by = ey * bn, bz = ez * bn;
#pragma unroll
                        for (int f = 0; f < FPB; ++f)
                            freq_tied<RAW>(g.rinv, g.delta, vx, vy, vz, bx, by, bz, wx, wy, wz, ts[f], kinv[f], kt[f],
                                           blk[s][f]);
                    } else {
#pragma unroll
                        for (int f = 0; f < FPB; ++f)
                            freq_factored<RAW>(g.rinv, g.delta, vx, vy, vz, ex, ey, ez, wx, wy, wz, t0[f], k[f],
                                               kt[f], blk[s][f]);
                    }
                } else if constexpr (MODE == MODE_SPLIT) {
                    const GeomF g = SER ? geom_series(pn, o[s], hn) : geom_split(pn, o[s]);
#pragma unroll
                    for (int f = 0; f < FPB; ++f) freq_split<RAW>(g, t0[f], t1[f], k[f], kt[f], blk[s][f]);
                } else {
                    GeomF g;
                    float R;
                    geom_naive(pn, o[s], g, R);
#pragma unroll
                    for (int f = 0; f < FPB; ++f) freq_naive(g, R, t0[f], t1[f], k[f], blk[s][f]);
                }
            }
        }
        // the block sum into the chunk's running sum (a frequency past the last one is not stored)
        const bool first = b0 == n0;
#pragma unroll
        for (int f = 0; f < FPB; ++f) {
            if (f >= n_valid) break;
#pragma unroll
            for (int s = 0; s < OPL; ++s) {
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    float *q = run + ((s * FPB + f) * 6 + c) * 64;
                    *q = first ? blk[s][f][c] : *q + blk[s][f][c];
                }
#pragma unroll
                for (int c = 6; c < 12; ++c) {
                    float *q = part[f] + s * 768 + c * 64 + lane;
                    *q = first ? blk[s][f][c] : *q + blk[s][f][c];
                }
            }
        }
    }
#pragma unroll
    for (int f = 0; f < FPB; ++f) {
        if (f >= n_valid) break;
#pragma unroll
        for (int s = 0; s < OPL; ++s)
#pragma unroll
            for (int c = 0; c < 6; ++c) part[f][s * 768 + c * 64 + lane] = run[((s * FPB + f) * 6 + c) * 64];
    }
}

// Persistent quadrature kernel.  Every wave repeatedly takes the next tile
// (one node chunk, 64*OPL observation points, FPB consecutive frequencies)
// from the device counters counter[QUAD_SEGMENTS], zeroed before the launch.
// Node and table data are wave-uniform (scalar loads); each lane owns OPL
// points x FPB frequencies x 12 accumulators.  Every wave exits once all
// segments are exhausted.
// Resident waves per SIMD the register allocation plans for.  One point x four frequencies per
// lane in FP32 holds 48 accumulators; unconstrained, the compiler interleaves the four
// frequencies' chains with up to ~116 VGPRs (4 waves); at 5 waves (<= 102 VGPRs) it keeps most of
// that overlap without spilling, which measured fastest.  The FP64 form at one point x two
// frequencies takes 131 VGPRs unconstrained (3 waves) and 127 at 4 waves, without spilling: the
// fourth wave hides more of the scalar-load latency of each node step (at 5 waves it spills).
// Other shapes (and the naive ablation, whose library sine and cosine spill at 5 waves): no
// constraint.
template <int MODE, int OPL, int FPB>
constexpr int quad_waves_per_eu()
{
    if (OPL != 1) return 1;
    if (MODE == MODE_FP64) return FPB == 2 ? 4 : 1;
    return MODE == MODE_SPLIT && FPB == 4 ? 5 : 1;
}

template <int MODE, int OPL, int FPB>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(quad_waves_per_eu<MODE, OPL, FPB>())))
k_quad(const QuadJob *__restrict__ jobs_, int n_jobs, int64_t n_tiles,
                                              unsigned int *__restrict__ counter)
{
    cjob *jobs = (cjob *)jobs_;
    const int lane = threadIdx.x & 63;
    const double2 *ttab = nullptr;   // the FP64 form's (cos, sin) table
    if constexpr (MODE == MODE_FP64) ttab = turn_table_lds();
    // The tile list is cut into QUAD_SEGMENTS contiguous segments with a counter
    // each.  Workgroups are dispatched to the 8 XCDs round robin, so block b
    // starts on segment b % 8: the tiles that share a (frequency block, node
    // chunk) run on one XCD and its L2 serves their table reads.  A wave that
    // drains its segment moves on to the next one; it leaves when every
    // segment it has visited (all of them, in the end) is exhausted.
    int seg = (int)(blockIdx.x % QUAD_SEGMENTS), visited = 1;
    for (;;) {
        int64_t t, s1;
        for (;;) {
            unsigned int tt = 0;
            if (lane == 0) tt = atomicAdd(counter + seg, 1u);
            const int64_t s0 = (int64_t)seg * n_tiles / QUAD_SEGMENTS;
            s1 = (int64_t)(seg + 1) * n_tiles / QUAD_SEGMENTS;
            t = s0 + (int64_t)__builtin_amdgcn_readfirstlane(tt);
            if (t < s1 || visited == QUAD_SEGMENTS) break;
            seg = (seg + 1) % QUAD_SEGMENTS;
            ++visited;
        }
        if (t >= s1) break;
        const int j = find_job(jobs, n_jobs, t);
        const int64_t local = t - jobs[j].tile0 + jobs[j].tile_offset;
        const int obs_blocks = jobs[j].obs_blocks, n_chunks = jobs[j].n_chunks;
        const int ob = (int)(local % obs_blocks);
        const int64_t rest = local / obs_blocks;
        const int chunk = (int)(rest % n_chunks);
        const int kb = (int)(rest / n_chunks);
        const int n_tot = jobs[j].n_tot, n_k = jobs[j].n_k;
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
            const bool ser = jobs[j].series_delta != 0;
            if (jobs[j].tied && ser)
                tile_f64<OPL, FPB, true, true, true>(jobs + j, lane, chunk, n0, n1, obase, kidx, k64, n_valid, ttab);
            else if (jobs[j].tied)
                tile_f64<OPL, FPB, true, false, true>(jobs + j, lane, chunk, n0, n1, obase, kidx, k64, n_valid, ttab);
            else if (jobs[j].factored && ser)
                tile_f64<OPL, FPB, true, true>(jobs + j, lane, chunk, n0, n1, obase, kidx, k64, n_valid, ttab);
            else if (jobs[j].factored)
                tile_f64<OPL, FPB, true, false>(jobs + j, lane, chunk, n0, n1, obase, kidx, k64, n_valid, ttab);
            else if (ser)
                tile_f64<OPL, FPB, false, true>(jobs + j, lane, chunk, n0, n1, obase, kidx, k64, n_valid, ttab);
            else
                tile_f64<OPL, FPB, false, false>(jobs + j, lane, chunk, n0, n1, obase, kidx, k64, n_valid, ttab);
        } else if constexpr (MODE == MODE_SPLIT) {
            // per job (not per tile), so the bits of a point do not depend on the launch shape
            const bool raw = jobs[j].raw_phase != 0;
            if (jobs[j].tied) {
                const bool ser = jobs[j].series_delta != 0;
                if (raw && ser)
                    tile_f32<MODE, OPL, FPB, true, true, true, true>(jobs + j, lane, chunk, n0, n1, obase, kidx, k64,
                                                                     n_valid);
                else if (raw)
                    tile_f32<MODE, OPL, FPB, true, true, false, true>(jobs + j, lane, chunk, n0, n1, obase, kidx, k64,
                                                                      n_valid);
                else if (ser)
                    tile_f32<MODE, OPL, FPB, true, false, true, true>(jobs + j, lane, chunk, n0, n1, obase, kidx, k64,
                                                                      n_valid);
                else
                    tile_f32<MODE, OPL, FPB, true, false, false, true>(jobs + j, lane, chunk, n0, n1, obase, kidx,
                                                                       k64, n_valid);
            } else if (jobs[j].factored) {
                const bool ser = jobs[j].series_delta != 0;
                if (raw && ser)
                    tile_f32<MODE, OPL, FPB, true, true, true>(jobs + j, lane, chunk, n0, n1, obase, kidx, k64, n_valid);
                else if (raw)
                    tile_f32<MODE, OPL, FPB, true, true, false>(jobs + j, lane, chunk, n0, n1, obase, kidx, k64, n_valid);
                else if (ser)
                    tile_f32<MODE, OPL, FPB, true, false, true>(jobs + j, lane, chunk, n0, n1, obase, kidx, k64, n_valid);
                else
                    tile_f32<MODE, OPL, FPB, true, false, false>(jobs + j, lane, chunk, n0, n1, obase, kidx, k64,
                                                                 n_valid);
            } else {
                const bool ser = jobs[j].series_delta != 0;
                if (raw && ser)
                    tile_f32<MODE, OPL, FPB, false, true, true>(jobs + j, lane, chunk, n0, n1, obase, kidx, k64, n_valid);
                else if (raw)
                    tile_f32<MODE, OPL, FPB, false, true, false>(jobs + j, lane, chunk, n0, n1, obase, kidx, k64,
                                                                 n_valid);
                else if (ser)
                    tile_f32<MODE, OPL, FPB, false, false, true>(jobs + j, lane, chunk, n0, n1, obase, kidx, k64,
                                                                 n_valid);
                else
                    tile_f32<MODE, OPL, FPB, false, false, false>(jobs + j, lane, chunk, n0, n1, obase, kidx, k64,
                                                                  n_valid);
            }
        } else {
            tile_f32<MODE, OPL, FPB, false, false>(jobs + j, lane, chunk, n0, n1, obase, kidx, k64, n_valid);
        }
    }
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

// Dynamic LDS of a launch: the FP32 forms' running sums of E, 6 floats per (point, frequency) of a lane.
static size_t quad_lds_bytes(int mode, int opl, int fpb, int waves_per_block)
{
    return mode == MODE_FP64 ? 0 : sizeof(float) * 6 * 64 * (size_t)(opl * fpb * waves_per_block);
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
#define SC_QUAD_LAUNCH(M, O, F)                                                                          \
    if (mode == M && opl == O && fpb == F) {                                                            \
        hipLaunchKernelGGL((k_quad<M, O, F>), g, b, quad_lds_bytes(M, O, F, waves_per_block), st, jobs, n_jobs, \
                           n_tiles, counter);                                                           \
        return hipGetLastError();                                                                       \
    }
    SC_QUAD_SHAPES(SC_QUAD_LAUNCH, MODE_FP64)
    SC_QUAD_SHAPES(SC_QUAD_LAUNCH, MODE_SPLIT)
    SC_QUAD_SHAPES(SC_QUAD_LAUNCH, MODE_NAIVE)
#undef SC_QUAD_LAUNCH
    return hipErrorInvalidValue;
}

}  // namespace sc
