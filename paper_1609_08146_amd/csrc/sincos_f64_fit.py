"""Coefficients of the FP64 sine and cosine of the quadrature kernel (sincos_turns_f64 in
sc_quad.hip): degree-5 Chebyshev fits, in u = x^2 on [0, (pi/4)^2], of

    S(u) = (sin x - x) / x^3        and        C(u) = (cos x - 1 + x^2/2) / x^4,

so that sin x = x + x^3 S(x^2) and cos x = 1 - x^2/2 + x^4 C(x^2) on |x| <= pi/4.  Prints the
coefficients (highest power first, as the kernel's Horner chains use them) and the fit errors.
Needs mpmath; not part of the build.
"""
import mpmath as mp

mp.mp.dps = 50
U = (mp.pi / 4) ** 2


def S(u):
    if u == 0:
        return mp.mpf(-1) / 6
    x = mp.sqrt(u)
    return (mp.sin(x) - x) / (u * x)


def C(u):
    if u == 0:
        return mp.mpf(1) / 24
    x = mp.sqrt(u)
    return (mp.cos(x) - 1 + u / 2) / (u * u)


if __name__ == "__main__":
    for name, fn in (("S", S), ("C", C)):
        poly, err = mp.chebyfit(fn, [0, U], 6, error=True)
        print(name, "fit error", mp.nstr(err, 4), "coefficients", [repr(float(c)) for c in poly])
