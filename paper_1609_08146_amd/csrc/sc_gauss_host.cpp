// sc_gauss_host.cpp -- the Gauss-Legendre rule used for the radial quadrature
// (Sec. III-C).  Host-only C++ built with the system compiler (it needs
// __float128, which the device compiler does not accept).
//
// Roots of P_n start from Tricomi's asymptotic estimate, are refined by
// Newton's method in long double, and finished with a Newton step in quad
// precision; P_n and P_n' come from their three-term recurrences
// (P_{m+1} = a_m z P_m - b_m P_{m-1} with a_m = (2m+1)/(m+1), b_m = m/(m+1),
// and P'_{m+1} = P'_{m-1} + (2m+1) P_m).  Every node and weight is therefore
// the correctly rounded double of the exact rule.  The rule is symmetric, so
// only the non-negative roots are computed; they are independent, so large
// rules spread them over a few host threads (the result does not depend on
// how they are spread).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <thread>
#include <vector>

namespace sc {

namespace {

// Recurrence coefficients a_m, b_m (m = 1 .. n-1) in the precision T, computed once per rule.
template <typename T>
struct LegendreCoef {
    std::vector<T> a, b, c;   // c_m = 2m + 1
    explicit LegendreCoef(int n) : a(n), b(n), c(n)
    {
        for (int m = 1; m < n; ++m) {
            a[m] = (T)(2 * m + 1) / (T)(m + 1);
            b[m] = (T)m / (T)(m + 1);
            c[m] = (T)(2 * m + 1);
        }
    }
};

template <typename T>
void legendre_and_derivative(int n, const LegendreCoef<T> &k, T z, T &p, T &d)
{
    T p0 = 1, p1 = z, d0 = 0, d1 = 1;
    for (int m = 1; m < n; ++m) {
        const T p2 = k.a[m] * z * p1 - k.b[m] * p0;
        const T d2 = d0 + k.c[m] * p1;
        p0 = p1;
        p1 = p2;
        d0 = d1;
        d1 = d2;
    }
    p = p1;
    d = d1;
}

// Roots i0 <= i < i1 (1-based, the i-th largest) of P_n and their weights.
void roots(int n, int i0, int i1, const LegendreCoef<long double> &kl, const LegendreCoef<__float128> &kq,
           std::vector<double> &x, std::vector<double> &w)
{
    const long double pi = 3.141592653589793238462643383279502884L;
    const long double nn = n;
    for (int i = i0; i < i1; ++i) {
        long double z =
            (1.0L - (nn - 1.0L) / (8.0L * nn * nn * nn)) * cosl(pi * (4.0L * i - 1.0L) / (4.0L * nn + 2.0L));
        __float128 zq;
        if (2 * i - 1 == n) {
            zq = 0;   // middle node of an odd rule
        } else {
            for (int it = 0; it < 100; ++it) {
                long double p, d;
                legendre_and_derivative(n, kl, z, p, d);
                const long double step = p / d;
                z -= step;
                if (fabsl(step) < 1e-17L) break;
            }
            // the long-double root is good to ~1e-19; one quad Newton step squares that error
            zq = z;
            __float128 p, d;
            legendre_and_derivative(n, kq, zq, p, d);
            zq -= p / d;
        }
        __float128 p, d;
        legendre_and_derivative(n, kq, zq, p, d);
        const __float128 wq = 2 / ((1 - zq * zq) * d * d);
        x[n - i] = (double)zq;
        x[i - 1] = -(double)zq;
        w[n - i] = (double)wq;
        w[i - 1] = (double)wq;
    }
}

}  // namespace

void gauss_legendre_rule(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    const LegendreCoef<long double> kl(n);
    const LegendreCoef<__float128> kq(n);
    const int half = (n + 1) / 2;
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int n_threads = std::max(1, std::min<int>({(int)std::min(hw, 16u), half / 16, 16}));
    if (n_threads == 1) {
        roots(n, 1, half + 1, kl, kq, x, w);
        return;
    }
    // contiguous slices of roots: every root costs the same, so the slices balance
    std::vector<std::thread> pool;
    for (int t = 0; t < n_threads; ++t) {
        const int i0 = 1 + (int)((int64_t)half * t / n_threads), i1 = 1 + (int)((int64_t)half * (t + 1) / n_threads);
        pool.emplace_back(roots, n, i0, i1, std::cref(kl), std::cref(kq), std::ref(x), std::ref(w));
    }
    for (auto &th : pool) th.join();
}

}  // namespace sc
