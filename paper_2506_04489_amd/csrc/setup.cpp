// setup.cpp - Algorithm 1, step S0 on the host: the Gaussian-sum fit (its R
// weights and exponents).  The 1D integrals (S1) run on the device
// (tables.hip).
#include <algorithm>
#include <cmath>

#include "host_common.hpp"

namespace psp {

// --------------------------------------------------------------------- S0
// Section 2, eq. sin_1_x: with t = e^u,
//   1/r = (2/sqrt(pi)) int_R exp(-r^2 e^{2u} + u) du,
// and the trapezoid rule with R nodes u_s = u0 + s tau gives
//   1/(8 pi r) ~ sum_s w_s exp(-a_s r^2),  a_s = e^{2 u_s},  w_s = tau e^{u_s} / (4 pi^{3/2}).
// tau and u0 balance three error estimates at one level e^{-x}: the
// trapezoid error exp(-pi^2 / (2 tau)) (the integrand is analytic in the
// strip |Im u| < pi/4), the left truncation (2/sqrt(pi)) delta e^{u0} at
// r = delta, and the right truncation, negligible once eps^2 e^{2 u_max} = x.
// x solves (R-1) tau = u_max - u0, found by a fixed 100-step bisection.
static double steps_needed(double x, double eps, double delta) {
    const double pi = 3.14159265358979323846;
    const double tau = pi * pi / (2.0 * x);
    const double u0 = -x - std::log(2.0 * delta / std::sqrt(pi));
    const double umax = std::log(std::sqrt(x) / eps);
    return (umax - u0) / tau;
}

void gs_fit(int R, double eps, double delta, std::vector<double> &omega, std::vector<double> &alpha) {
    const double pi = 3.14159265358979323846;
    const double want = (double)(R - 1);
    double lo = 1.0, hi = 80.0;
    for (int it = 0; it < 100; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (steps_needed(mid, eps, delta) > want)
            hi = mid;
        else
            lo = mid;
    }
    const double x = lo;
    const double tau = pi * pi / (2.0 * x);
    const double u0 = -x - std::log(2.0 * delta / std::sqrt(pi));
    const double c = tau / (4.0 * std::pow(pi, 1.5));
    omega.resize(R);
    alpha.resize(R);
    for (int s = 0; s < R; ++s) {
        const double u = u0 + s * tau;
        alpha[s] = std::exp(2.0 * u);
        omega[s] = c * std::exp(u);
    }
}

}  // namespace psp
