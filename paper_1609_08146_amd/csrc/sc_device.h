// sc_device.h -- device-side helpers for the gfx950 Stratton-Chu kernels:
// double-double arithmetic for the large mirror phases, phase reduction
// modulo 2 pi, and the per-node data layouts shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sc {

// 2 pi = TWO_PI_1 + TWO_PI_2 + TWO_PI_3 (each term the double nearest the remainder)
constexpr double TWO_PI_1 = 0x1.921fb54442d18p+2;
constexpr double TWO_PI_2 = 0x1.1a62633145c07p-52;
constexpr double TWO_PI_3 = -0x1.f1976b7ed8fbcp-108;
constexpr double INV_TWO_PI = 0x1.45f306dc9c883p-3;
constexpr double FOUR_PI = 12.566370614359172;

// ---------------------------------------------------------------- double-double
struct dd {
    double hi, lo;
};

__device__ __forceinline__ dd two_prod(double a, double b)
{
    double p = a * b;
    return {p, __fma_rn(a, b, -p)};
}

__device__ __forceinline__ dd two_sum(double a, double b)
{
    double s = a + b;
    double bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}

__device__ __forceinline__ dd fast_two_sum(double a, double b)
{
    double s = a + b;
    return {s, b - (s - a)};
}

__device__ __forceinline__ dd dd_add(dd a, dd b)
{
    dd s = two_sum(a.hi, b.hi);
    return fast_two_sum(s.hi, s.lo + (a.lo + b.lo));
}

__device__ __forceinline__ dd dd_sub_d(dd a, double b)
{
    dd s = two_sum(a.hi, -b);
    return fast_two_sum(s.hi, s.lo + a.lo);
}

// |(x, y, z)| to ~1e-32 relative: sum of squares exactly in dd, one Newton step on sqrt.
__device__ __forceinline__ dd dd_norm3(double x, double y, double z)
{
    dd s = two_prod(x, x);
    s = dd_add(s, two_prod(y, y));
    s = dd_add(s, two_prod(z, z));
    double h = sqrt(s.hi);
    if (h == 0.0) return {0.0, 0.0};
    double e = __fma_rn(-h, h, s.hi) + s.lo;
    return fast_two_sum(h, e / (2.0 * h));
}

// (k * d) mod 2pi in [-pi, pi] for |k d| up to ~1e9 rad, error ~1e-15 rad.
// Cody-Waite with a three-part 2 pi; n * TWO_PI_1 is formed exactly with an FMA.
__device__ __forceinline__ double phase_mod_2pi(double k, dd d)
{
    dd p = two_prod(k, d.hi);
    p = fast_two_sum(p.hi, __fma_rn(k, d.lo, p.lo));
    double n = rint(p.hi * INV_TWO_PI);
    dd q = two_prod(n, TWO_PI_1);
    double r = (p.hi - q.hi) - q.lo;   // exact difference (Sterbenz), then the product's tail
    r += p.lo;
    r = __fma_rn(-n, TWO_PI_2, r);
    r = __fma_rn(-n, TWO_PI_3, r);
    return r;
}

// ---------------------------------------------------------------- layouts
// Node record (FP64): x, y, z, |r_s|      Node record (FP32): same, rounded.
// Observation record: x, y, z, |r'|^2.
// Table record per (k, node), 8 reals: Jt.x (re, im), Jt.y, Jt.z, rho_t (re, im), where
//   surface node:  Jt  = 2ik W/(4pi) (n~ x B_inc) P,   rho_t = 2 W/(4pi) (n~ . E_inc) P
//   rim node:      Jt  = 0,                           rho_t = (2i/k) dphi/(4pi) [n^ x (n^ x B_inc)] . t P
// with W the quadrature weight, t = d r_s / d phi and P the folded node phase
// (e^{ik|r_s|} for the split forms, 1 for the naive FP32 form).  The per-pair
// sums are then
//   E = sum Jt gt + rho_t ht R,   B = (1/ik) sum (Jt x R) ht,
//   gt = e^{ik(R - |r_s|)} / R,   ht = (ik - 1/R) gt / R,   R = r_s - r'.

}  // namespace sc
