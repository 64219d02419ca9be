// incl_quadrature.h -- the inclination quadrature of the 2D-invariant
// formal solution (Osborne & Sannikov, arXiv:2408.14425, Sec. 3.1): each
// flatland ray stands for rays with the same x-z projection at inclinations
// mu = cos(angle to the invariant y axis) in [0, 1] (one hemisphere; the
// other is its mirror image), integrated with a Gauss-Radau rule. Plain C++
// (host only).
#pragma once

#include <cmath>
#include <vector>

namespace rcx {

// Gauss-Radau rule with n nodes for the integral over mu in [0, 1], the
// node mu = 0 fixed (the in-plane ray): the other nodes are the roots of
// (P_{n-1}(x) + P_n(x)) / (1 + x) on (-1, 1) (Legendre P, x = 2 mu - 1), the
// weights (1 - x) / (n^2 P_{n-1}(x)^2) on [-1, 1] and 2 / n^2 for the fixed
// node, halved for [0, 1]. Roots by Newton's method from the cosine guesses.
inline void radau_nodes(int32_t n, std::vector<double>& mu, std::vector<double>& wt)
{
    mu.assign(n, 0.0);
    wt.assign(n, 0.0);
    wt[0] = 1.0 / ((double)n * n);
    auto legendre = [](int32_t m, double x, double& pm, double& pm1) {
        // pm = P_m(x), pm1 = P_{m-1}(x)
        double a = 1.0, b = x;  // P_0, P_1
        if (m == 0) {
            pm = 1.0;
            pm1 = 0.0;
            return;
        }
        for (int32_t k = 2; k <= m; ++k) {
            const double c = ((2 * k - 1) * x * b - (k - 1) * a) / k;
            a = b;
            b = c;
        }
        pm = b;
        pm1 = a;
    };
    for (int32_t k = 1; k < n; ++k) {
        double x = -std::cos(2.0 * 3.14159265358979323846 * k / (2.0 * n - 1.0));
        for (int it = 0; it < 100; ++it) {
            double pn, pn1;
            legendre(n, x, pn, pn1);
            // f = P_{n-1} + P_n; (1 - x^2) P_m' = m (P_{m-1} - x P_m)
            double pnm2 = 0.0, dummy;
            if (n >= 2) legendre(n - 1, x, dummy, pnm2);
            const double f = pn1 + pn;
            const double d1 = (n - 1) * (pnm2 - x * pn1) / (1.0 - x * x);
            const double d2 = n * (pn1 - x * pn) / (1.0 - x * x);
            const double dx = f / (d1 + d2);
            x -= dx;
            if (std::fabs(dx) < 1e-15) break;
        }
        double pn, pn1;
        legendre(n, x, pn, pn1);
        mu[k] = 0.5 * (x + 1.0);
        wt[k] = 0.5 * (1.0 - x) / ((double)n * n * pn1 * pn1);
    }
}

}  // namespace rcx
