// sc_gauss_host.cpp -- the Gauss-Legendre rule used for the radial quadrature
// (Sec. III-C).  Host-only C++ built with the system compiler (it needs
// __float128, which the device compiler does not accept).
//
// Roots of P_n start from Tricomi's asymptotic estimate, are refined by
// Newton's method in long double, and finished with Newton steps in quad
// precision; P_n and P_n' come from their three-term recurrences (P'_{m+1} =
// P'_{m-1} + (2m+1) P_m).  Every node and weight is therefore the correctly
// rounded double of the exact rule.  The rule is symmetric, so only the
// non-negative roots are computed.
#include <cmath>
#include <vector>

namespace sc {

template <typename T>
static void legendre_and_derivative(int n, T z, T &p, T &d)
{
    T p0 = 1, p1 = z, d0 = 0, d1 = 1;
    for (int m = 1; m < n; ++m) {
        const T p2 = ((T)(2 * m + 1) * z * p1 - (T)m * p0) / (T)(m + 1);
        const T d2 = d0 + (T)(2 * m + 1) * p1;
        p0 = p1;
        p1 = p2;
        d0 = d1;
        d1 = d2;
    }
    p = p1;
    d = d1;
}

void gauss_legendre_rule(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    const long double pi = 3.141592653589793238462643383279502884L;
    const long double nn = n;
    for (int i = 1; i <= (n + 1) / 2; ++i) {
        long double z =
            (1.0L - (nn - 1.0L) / (8.0L * nn * nn * nn)) * cosl(pi * (4.0L * i - 1.0L) / (4.0L * nn + 2.0L));
        __float128 zq;
        if (2 * i - 1 == n) {
            zq = 0;   // middle node of an odd rule
        } else {
            for (int it = 0; it < 100; ++it) {
                long double p, d;
                legendre_and_derivative(n, z, p, d);
                const long double step = p / d;
                z -= step;
                if (fabsl(step) < 1e-17L) break;
            }
            zq = z;
            for (int it = 0; it < 2; ++it) {
                __float128 p, d;
                legendre_and_derivative<__float128>(n, zq, p, d);
                zq -= p / d;
            }
        }
        __float128 p, d;
        legendre_and_derivative<__float128>(n, zq, p, d);
        const __float128 wq = 2 / ((1 - zq * zq) * d * d);
        x[n - i] = (double)zq;
        x[i - 1] = -(double)zq;
        w[n - i] = (double)wq;
        w[i - 1] = (double)wq;
    }
}

}  // namespace sc
