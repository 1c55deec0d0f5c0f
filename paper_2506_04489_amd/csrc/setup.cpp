// setup.cpp - Algorithm 1 on the host: Gaussian-sum fit (S0) and the 1D
// integrals of the separable kernel transform (S1), both in FP64.
#include <algorithm>
#include <cmath>
#include <thread>

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

// --------------------------------------------------------------------- S1
// eq. Gten_sep: J_p(k) = 2 int_0^{L/2} y^p exp(-a y^2) cos(xi_k y) dy,
// xi_k = 2 pi k / L, p in {0, 2}.
//  * a (L/2)^2 >= 50: the part beyond L/2 is below e^-50 of the whole, and
//    the full-line closed forms apply:
//      J0 = sqrt(pi/a) e^{-xi^2/(4a)},
//      J2 = sqrt(pi/a) (1/(2a)) (1 - xi^2/(2a)) e^{-xi^2/(4a)}.
//  * otherwise: adaptive Gauss-Kronrod (7-point Gauss / 15-point Kronrod)
//    on [0, min(L/2, 8.6/sqrt(a))], as the paper precomputes these
//    integrals.  A panel is bisected until the Gauss-Kronrod error estimate
//    s (200 |K15 - G7| / s)^{3/2} (s: the integral's scale) of the hardest
//    integrands (k = 0 and k = n, p = 0 and 2) is below 1e-19 s times the
//    panel's share of the interval; the K15 values of the final panels are
//    summed for every k.
typedef long double ld;
static const ld kXgk[8] = {
    0.991455371120812639206854697526329L, 0.949107912342758524526189684047851L,
    0.864864423359769072789712788640926L, 0.741531185599394439863864773280788L,
    0.586087235467691130294144845693013L, 0.405845151377397166906606412076961L,
    0.207784955007898467600689403773245L, 0.000000000000000000000000000000000L};
static const ld kWgk[8] = {
    0.022935322010529224963732008058970L, 0.063092092629978553290700663189204L,
    0.104790010322250183839876322541518L, 0.140653259715525918745189590510238L,
    0.169004726639267902826583426598550L, 0.190350578064785409913256402421014L,
    0.204432940075298892414161999234649L, 0.209482141084727828012999174891714L};
static const ld kWg[4] = {  // Gauss weights of the nodes kXgk[1], [3], [5], [7]
    0.129484966168869693270611432679082L, 0.279705391489276667901467771423780L,
    0.381830050505118944950369775488975L, 0.417959183673469387755102040816327L};

// K15 and G7 of the probe integrands y^p exp(-a y^2) cos(xi y) on [l, r]
static void gk_probe(ld a, const ld *xis, int nxi, ld l, ld r, ld *K, ld *G) {
    const ld c = 0.5L * (l + r), hw = 0.5L * (r - l);
    for (int q = 0; q < 2 * nxi; ++q) K[q] = G[q] = 0.0L;
    for (int i = 0; i < 15; ++i) {
        const int j = i < 8 ? i : 14 - i;
        const ld y = i < 8 ? c - hw * kXgk[j] : c + hw * kXgk[j];
        const ld g = expl(-a * y * y);
        const bool gauss = (j % 2) == 1;
        for (int q = 0; q < nxi; ++q) {
            const ld f0 = g * cosl(xis[q] * y), f2 = y * y * f0;
            K[2 * q] += kWgk[j] * f0;
            K[2 * q + 1] += kWgk[j] * f2;
            if (gauss) {
                G[2 * q] += kWg[j / 2] * f0;
                G[2 * q + 1] += kWg[j / 2] * f2;
            }
        }
    }
    for (int q = 0; q < 2 * nxi; ++q) {
        K[q] *= hw;
        G[q] *= hw;
    }
}

static void split_panels(ld a, const ld *xis, int nxi, ld l, ld r, ld b, const ld *scale, int depth,
                         std::vector<std::pair<ld, ld>> &out) {
    ld K[4], G[4];
    gk_probe(a, xis, nxi, l, r, K, G);
    bool ok = true;
    for (int q = 0; q < 2 * nxi; ++q) {
        const ld sc = scale[q & 1];
        const ld est = sc * powl(200.0L * fabsl(K[q] - G[q]) / sc, 1.5L);
        if (est > 1e-19L * sc * (r - l) / b) ok = false;
    }
    if (ok || depth >= 40) {
        out.emplace_back(l, r);
        return;
    }
    const ld m = 0.5L * (l + r);
    split_panels(a, xis, nxi, l, m, b, scale, depth + 1, out);
    split_panels(a, xis, nxi, m, r, b, scale, depth + 1, out);
}

// The quadrature runs in x87 extended precision (long double) and rounds to
// double at the end: for wide Gaussians the box-truncated integrals at high k
// are ~k^2 smaller than the integrand, so double node positions and cosine
// arguments alone would leave ~1e-12 relative errors there.
static void tables_one(double a64, int n, double L, double *J0, double *J2) {
    const double pi = 3.14159265358979323846;
    const double half = 0.5 * L;
    if (a64 * half * half >= 50.0) {
        const double w = 2.0 * pi / L;
        const double s0 = std::sqrt(pi / a64);
        for (int k = 0; k <= n; ++k) {
            const double xi = w * k;
            const double e = s0 * std::exp(-xi * xi / (4.0 * a64));
            J0[k] = e;
            J2[k] = e * (1.0 / (2.0 * a64)) * (1.0 - xi * xi / (2.0 * a64));
        }
        return;
    }
    const ld a = a64;
    const ld two_pi = 6.283185307179586476925286766559005768L;
    const ld w = two_pi / (ld)L;
    const ld b = std::min((ld)half, 8.6L / sqrtl(a));
    // scales: the integrals of the non-oscillating envelopes
    ld scale[2] = {0.0L, 0.0L};
    {
        const ld xi0 = 0.0L;
        ld K[2], G[2];
        const int m = 64;
        for (int i = 0; i < m; ++i) {
            gk_probe(a, &xi0, 1, b * i / m, b * (i + 1) / m, K, G);
            scale[0] += K[0];
            scale[1] += K[1];
        }
    }
    const ld probe[2] = {0.0L, w * n};
    std::vector<std::pair<ld, ld>> panels;
    // start from panels no wider than the Gaussian width or a cosine period
    const ld w0 = std::min(b, std::min(1.0L / sqrtl(a), two_pi / (w * std::max(n, 1))));
    const int p0 = std::max(1, (int)ceill(b / w0 - 1e-12L));
    for (int i = 0; i < p0; ++i) split_panels(a, probe, 2, b * i / p0, b * (i + 1) / p0, b, scale, 0, panels);
    std::vector<ld> s0(n + 1, 0.0L), s2(n + 1, 0.0L);
    for (const auto &pr : panels) {
        const ld c = 0.5L * (pr.first + pr.second), hw = 0.5L * (pr.second - pr.first);
        for (int i = 0; i < 15; ++i) {
            const int j = i < 8 ? i : 14 - i;
            const ld y = i < 8 ? c - hw * kXgk[j] : c + hw * kXgk[j];
            const ld g = hw * kWgk[j] * expl(-a * y * y);
            const ld g2 = g * y * y;
            // cos(k w y) for k = 0..n by rotation in extended precision,
            // re-anchored with cosl/sinl every 32 steps (drift below 1e-17)
            const ld th = w * y, c1 = cosl(th), s1 = sinl(th);
            ld ck = 1.0L, sk = 0.0L;
            for (int k = 0; k <= n; ++k) {
                if ((k & 31) == 0 && k > 0) {
                    ck = cosl((ld)k * th);
                    sk = sinl((ld)k * th);
                }
                s0[k] += g * ck;
                s2[k] += g2 * ck;
                const ld cn = ck * c1 - sk * s1;
                sk = sk * c1 + ck * s1;
                ck = cn;
            }
        }
    }
    for (int k = 0; k <= n; ++k) {
        J0[k] = (double)(2.0L * s0[k]);
        J2[k] = (double)(2.0L * s2[k]);
    }
}

void tables_1d(const std::vector<double> &alpha, int n, double L, std::vector<double> &J0,
               std::vector<double> &J2) {
    const int R = (int)alpha.size();
    J0.assign((size_t)R * (n + 1), 0.0);
    J2.assign((size_t)R * (n + 1), 0.0);
    unsigned hw = std::thread::hardware_concurrency();
    int nth = (int)std::max(1u, std::min(hw == 0 ? 1u : hw, 16u));
    nth = std::min(nth, R);
    std::vector<std::thread> pool;
    for (int t = 0; t < nth; ++t) {
        pool.emplace_back([&, t]() {
            for (int s = t; s < R; s += nth)
                tables_one(alpha[s], n, L, &J0[(size_t)s * (n + 1)], &J2[(size_t)s * (n + 1)]);
        });
    }
    for (auto &th : pool) th.join();
}

}  // namespace psp
